// Gain of the matrix-normal Kalman update, Eq. (10a) / Eq. (14b):
//   K = Sigma^{XY} (Sigma^Y)^{-1},
// solved in FP64 through the Cholesky factor Sigma^Y = L L^T.  The matrix
// inverted is p x p with p = n + l (the rows of the virtual observation).
#include "oic_internal.h"

namespace oic {
namespace {

// One workgroup: right-looking Cholesky of the p x p matrix Syy into L (lower triangle).
__global__ __launch_bounds__(1024) void k_chol(int p, const double* __restrict__ Syy,
                                               double* __restrict__ L, int* __restrict__ flag) {
  __shared__ double piv;
  __shared__ int bad;
  const int tid = threadIdx.x, bd = blockDim.x;
  for (long long idx = tid; idx < (long long)p * p; idx += bd) L[idx] = Syy[idx];
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < p; ++k) {
    if (tid == 0) {
      const double dkk = L[(size_t)k * p + k];
      if (!(dkk > 0.0) || !isfinite(dkk)) {
        bad = 1;
        piv = 1.0;
      } else {
        piv = sqrt(dkk);
      }
      L[(size_t)k * p + k] = piv;
    }
    __syncthreads();
    if (bad) break;
    for (int i = k + 1 + tid; i < p; i += bd) L[(size_t)i * p + k] /= piv;
    __syncthreads();
    const int rem = p - k - 1;
    for (long long idx = tid; idx < (long long)rem * rem; idx += bd) {
      const int ii = k + 1 + (int)(idx / rem);
      const int jj = k + 1 + (int)(idx % rem);
      if (jj <= ii) L[(size_t)ii * p + jj] -= L[(size_t)ii * p + k] * L[(size_t)jj * p + k];
    }
    __syncthreads();
  }
  if (tid == 0 && bad) *flag = 1;
}

// One thread per gain row a: solve L z = S[a]^T, then L^T k = z; K[a] = k (rounded to FP32).
// Zt (p x Ma, FP64) keeps each row's vector with consecutive rows adjacent.
__global__ void k_gain_rows(int p, int Ma, const double* __restrict__ S, const double* __restrict__ L,
                            double* __restrict__ Zt, float* __restrict__ K,
                            const int* __restrict__ flag) {
  if (*flag) return;
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= Ma) return;
  for (int b = 0; b < p; ++b) {
    double v = S[(size_t)a * p + b];
    const double* Lb = L + (size_t)b * p;
    for (int c = 0; c < b; ++c) v -= Lb[c] * Zt[(size_t)c * Ma + a];
    Zt[(size_t)b * Ma + a] = v / Lb[b];
  }
  for (int b = p - 1; b >= 0; --b) {
    double v = Zt[(size_t)b * Ma + a];
    for (int c = b + 1; c < p; ++c) v -= L[(size_t)c * p + b] * Zt[(size_t)c * Ma + a];
    v /= L[(size_t)b * p + b];
    Zt[(size_t)b * Ma + a] = v;
  }
  for (int b = 0; b < p; ++b) K[(size_t)a * p + b] = (float)Zt[(size_t)b * Ma + a];
}

}  // namespace

void launch_chol_gain(hipStream_t s, Timer& t, const Dims& d, int Ma, const double* S, double* Lwork,
                      double* scratch, float* K, int* flag) {
  const int p = d.p();
  OIC_LAUNCH(t, KC_CHOL, s, k_chol, dim3(1), dim3(1024), 0, p, S + (size_t)Ma * p, Lwork, flag);
  OIC_LAUNCH(t, KC_GAIN, s, k_gain_rows, dim3((unsigned)((Ma + 127) / 128)), dim3(128), 0, p, Ma, S,
             Lwork, scratch, K, flag);
}

}  // namespace oic
