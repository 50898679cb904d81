// Gain of the matrix-normal Kalman update, Eq. (10a) / Eq. (14b):
//   K = Sigma^{XY} (Sigma^Y)^{-1},
// in FP64.  The matrix inverted is p x p with p = n + l (the rows of the virtual
// observation).  One workgroup factors Sigma^Y = L L^T (Cholesky), inverts L in
// place and forms (Sigma^Y)^{-1} = L^{-T} L^{-1}; a second, wide kernel multiplies
// Sigma^{XY} by it.  For p <= 128 the factor lives in LDS; larger p work on an
// L2-resident global copy with the same code.
#include "oic_internal.h"

namespace oic {
namespace {

constexpr int kCholThreads = 512;
constexpr int kTX = 32, kTY = kCholThreads / kTX;  // 2-D thread grid for the updates
constexpr int kLdsMaxP = 90;                       // two p x p FP64 arrays in the 160 KiB LDS
constexpr int NBK = 8;                             // panel width

// Factor, invert and square the p x p SPD matrix in A (row-major; LDS or global),
// with W (p x p, same memory kind) as workspace; writes (Sigma^Y)^{-1} to Sinv and
// sets *flag when a pivot is not positive and finite.
//
// Blocked right-looking Cholesky with 8-wide panels: one thread factors the 8 x 8
// diagonal block in registers, the rows below solve against it in parallel, and
// the trailing lower triangle takes the rank-8 update; three barriers per panel.
// W = L^{-1} is formed the same way by panels of rows (triangular solve of the
// panel against its diagonal block, then a rank-8 update of the rows below), and
// (Sigma^Y)^{-1} = W^T W.
__device__ __forceinline__ void chol_inverse(int p, double* A, double* W, double* __restrict__ Sinv,
                                             int* __restrict__ flag) {
  // A and W use the leading dimension ld = p + 1: an odd number of doubles puts the
  // rows read by consecutive lanes in distinct LDS banks.
  const int ld = p + 1;
  __shared__ int bad;
  __shared__ double rdiag[NBK];
  const int tid = threadIdx.x;
  const int ty = tid / kTX, tx = tid % kTX;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int kb = 0; kb < p; kb += NBK) {
    const int nb = min(NBK, p - kb);
    if (tid == 0) {  // diagonal block, in registers (no early exit: keeps the array in VGPRs)
      double a[NBK][NBK];
      bool ok = true;
#pragma unroll
      for (int r = 0; r < NBK; ++r)
#pragma unroll
        for (int c = 0; c < NBK; ++c) a[r][c] = (r < nb && c <= r) ? A[(kb + r) * ld + kb + c] : 0.0;
#pragma unroll
      for (int k = 0; k < NBK; ++k) {
        double d = a[k][k];
        const bool live = k < nb;
        if (live && !(d > 0.0 && isfinite(d))) ok = false;
        if (!(d > 0.0)) d = 1.0;  // keep the arithmetic finite after a failure
        const double sq = sqrt(d), rs = 1.0 / sq;
        a[k][k] = live ? sq : a[k][k];
#pragma unroll
        for (int r = k + 1; r < NBK; ++r) a[r][k] *= rs;
#pragma unroll
        for (int c = k + 1; c < NBK; ++c)
#pragma unroll
          for (int r = c; r < NBK; ++r) a[r][c] -= a[r][k] * a[c][k];
      }
#pragma unroll
      for (int r = 0; r < NBK; ++r)
#pragma unroll
        for (int c = 0; c < NBK; ++c)
          if (r < nb && c <= r) A[(kb + r) * ld + kb + c] = a[r][c];
#pragma unroll
      for (int r = 0; r < NBK; ++r) rdiag[r] = 1.0 / a[r][r];
      if (!ok) bad = 1;
    }
    __syncthreads();
    if (bad) break;  // uniform
    // rows below: x = a_i L_kk^{-T}
    for (int i = kb + nb + tid; i < p; i += kCholThreads) {
      double x[NBK];
#pragma unroll
      for (int c = 0; c < NBK; ++c) x[c] = c < nb ? A[i * ld + kb + c] : 0.0;
#pragma unroll
      for (int c = 0; c < NBK; ++c) {
        if (c < nb) {
#pragma unroll
          for (int q = 0; q < c; ++q) x[c] -= x[q] * A[(kb + c) * ld + kb + q];
          x[c] *= rdiag[c];
        }
      }
#pragma unroll
      for (int c = 0; c < NBK; ++c)
        if (c < nb) A[i * ld + kb + c] = x[c];
    }
    __syncthreads();
    // trailing lower triangle: A[i][j] -= sum_c L[i][kb+c] L[j][kb+c]
    for (int i = kb + nb + ty; i < p; i += kTY) {
      double li[NBK];
#pragma unroll
      for (int c = 0; c < NBK; ++c) li[c] = c < nb ? A[i * ld + kb + c] : 0.0;
      for (int j = kb + nb + tx; j <= i; j += kTX) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < NBK; ++c)
          if (c < nb) acc = fma(li[c], A[j * ld + kb + c], acc);
        A[i * ld + j] -= acc;
      }
    }
    __syncthreads();
  }
  if (bad) {
    if (tid == 0) *flag = 1;
    return;
  }
  // W = L^{-1}: start from the identity, then panels of rows.
  for (int ii = ty; ii < p; ii += kTY)
    for (int jj = tx; jj < p; jj += kTX) W[ii * ld + jj] = ii == jj ? 1.0 : 0.0;
  __syncthreads();
  for (int kb = 0; kb < p; kb += NBK) {
    const int nb = min(NBK, p - kb);
    const int cols = kb + nb;
    if (tid < NBK) rdiag[tid] = tid < nb ? 1.0 / A[(kb + tid) * ld + kb + tid] : 1.0;
    __syncthreads();
    for (int j = tid; j < cols; j += kCholThreads) {  // W[kb:kb+nb, j] = L_kk^{-1} B[kb:kb+nb, j]
      double x[NBK];
#pragma unroll
      for (int r = 0; r < NBK; ++r) x[r] = r < nb ? W[(kb + r) * ld + j] : 0.0;
#pragma unroll
      for (int r = 0; r < NBK; ++r) {
        if (r < nb) {
#pragma unroll
          for (int q = 0; q < r; ++q) x[r] -= A[(kb + r) * ld + kb + q] * x[q];
          x[r] *= rdiag[r];
        }
      }
#pragma unroll
      for (int r = 0; r < NBK; ++r)
        if (r < nb) W[(kb + r) * ld + j] = x[r];
    }
    __syncthreads();
    for (int i = kb + nb + ty; i < p; i += kTY) {  // B[i][j] -= sum_r L[i][kb+r] W[kb+r][j]
      double li[NBK];
#pragma unroll
      for (int r = 0; r < NBK; ++r) li[r] = r < nb ? A[i * ld + kb + r] : 0.0;
      for (int j = tx; j < cols; j += kTX) {
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < NBK; ++r)
          if (r < nb) acc = fma(li[r], W[(kb + r) * ld + j], acc);
        W[i * ld + j] -= acc;
      }
    }
    __syncthreads();
  }
  // (Sigma^Y)^{-1}[a][b] = sum_{k >= max(a,b)} W[k][a] W[k][b]
  for (int a = ty; a < p; a += kTY)
    for (int b = tx; b <= a; b += kTX) {
      double acc = 0.0;
      for (int k = a; k < p; ++k) acc = fma(W[k * ld + a], W[k * ld + b], acc);
      Sinv[a * p + b] = acc;
      Sinv[b * p + a] = acc;
    }
}

__global__ __launch_bounds__(kCholThreads) void k_chol_inv_lds(int p, const double* __restrict__ Syy,
                                                               double* __restrict__ Sinv,
                                                               int* __restrict__ flag) {
  extern __shared__ double lds[];
  for (int idx = threadIdx.x; idx < p * p; idx += kCholThreads) lds[(idx / p) * (p + 1) + idx % p] = Syy[idx];
  __syncthreads();
  chol_inverse(p, lds, lds + p * (p + 1), Sinv, flag);
}

__global__ __launch_bounds__(kCholThreads) void k_chol_inv_global(int p, const double* __restrict__ Syy,
                                                                  double* __restrict__ work,
                                                                  double* __restrict__ Sinv,
                                                                  int* __restrict__ flag) {
  for (int idx = threadIdx.x; idx < p * p; idx += kCholThreads)
    work[(idx / p) * (p + 1) + idx % p] = Syy[idx];
  __syncthreads();
  chol_inverse(p, work, work + p * (p + 1), Sinv, flag);
}

// K[a][b] = sum_c Sxy[a][c] Sinv[c][b], FP64, rounded to FP32 (any p).  Block (64, 4).
__global__ __launch_bounds__(256) void k_gain_product(int p, int Ma, const double* __restrict__ Sxy,
                                                      const double* __restrict__ Sinv,
                                                      float* __restrict__ K,
                                                      const int* __restrict__ flag) {
  if (*flag) return;
  const int b = blockIdx.y * 64 + threadIdx.x;
  const int a = blockIdx.x * 4 + threadIdx.y;
  if (a >= Ma || b >= p) return;
  const double* row = Sxy + (size_t)a * p;
  double s = 0.0;
  for (int c = 0; c < p; ++c) s = fma(row[c], Sinv[(size_t)c * p + b], s);
  K[(size_t)a * p + b] = (float)s;
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// K = Sxy Sinv on the FP64 matrix cores.  A block of 4 waves owns 64 gain rows; wave w
// computes rows 16w..16w+15 against every 16-column block of Sinv (staged in LDS,
// zero-padded to a multiple of 16).  Lane layout as in the statistics kernel.
template <int NB>
__global__ __launch_bounds__(256) void k_gain_mfma(int p, int Ma, const double* __restrict__ Sxy,
                                                   const double* __restrict__ Sinv,
                                                   float* __restrict__ K,
                                                   const int* __restrict__ flag) {
  constexpr int P16 = NB * 16;
  __shared__ double sS[P16 * (P16 + 1)];
  if (*flag) return;
  for (int e = threadIdx.x; e < P16 * P16; e += 256) {
    const int r = e / P16, c = e % P16;
    sS[r * (P16 + 1) + c] = (r < p && c < p) ? Sinv[r * p + c] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int a = blockIdx.x * 64 + w * 16 + li;  // A-fragment row of this lane
  f64x4 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = f64x4{0.0, 0.0, 0.0, 0.0};
  double av[NB * 4];  // this lane's A fragments for every k-step, loaded up front
#pragma unroll
  for (int s4 = 0; s4 < NB * 4; ++s4) {
    const int k = s4 * 4 + lk;
    av[s4] = (a < Ma && k < p) ? Sxy[(size_t)a * p + k] : 0.0;
  }
#pragma unroll
  for (int s4 = 0; s4 < NB * 4; ++s4) {
    const int k = s4 * 4 + lk;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s4], sS[k * (P16 + 1) + nb * 16 + li], acc[nb],
                                                     0, 0, 0);
  }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = blockIdx.x * 64 + w * 16 + lk + 4 * r;
      const int col = nb * 16 + li;
      if (row < Ma && col < p) K[(size_t)row * p + col] = (float)acc[nb][r];
    }
}

}  // namespace

void launch_chol_gain(hipStream_t s, Timer& t, const Dims& d, int Ma, const double* S, double* Lwork,
                      double* scratch, float* K, int* flag) {
  const int p = d.p();
  const double* Syy = S + (size_t)Ma * p;
  double* Sinv = scratch;  // p*p
  if (p <= kLdsMaxP) {
    static bool attr_set = false;
    if (!attr_set) {
      hipFuncSetAttribute((const void*)k_chol_inv_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                          2 * kLdsMaxP * (kLdsMaxP + 1) * (int)sizeof(double));
      attr_set = true;
    }
    OIC_LAUNCH(t, KC_CHOL, s, k_chol_inv_lds, dim3(1), dim3(kCholThreads),
               2 * (size_t)p * (p + 1) * sizeof(double), p, Syy, Sinv, flag);
  } else {
    OIC_LAUNCH(t, KC_CHOL, s, k_chol_inv_global, dim3(1), dim3(kCholThreads), 0, p, Syy, Lwork, Sinv,
               flag);
  }
  const int nbk = (p + 15) / 16;
  const dim3 g((unsigned)((Ma + 63) / 64));
  switch (nbk) {
#define OIC_GAIN_CASE(NBV) \
  case NBV: OIC_LAUNCH(t, KC_GAIN, s, k_gain_mfma<NBV>, g, dim3(256), 0, p, Ma, S, Sinv, K, flag); return;
    OIC_GAIN_CASE(1) OIC_GAIN_CASE(2) OIC_GAIN_CASE(3) OIC_GAIN_CASE(4)
    OIC_GAIN_CASE(5) OIC_GAIN_CASE(6) OIC_GAIN_CASE(7) OIC_GAIN_CASE(8)
#undef OIC_GAIN_CASE
    default:
      OIC_LAUNCH(t, KC_GAIN, s, k_gain_product, dim3((unsigned)((Ma + 3) / 4), (unsigned)((p + 63) / 64)),
                 dim3(64, 4), 0, p, Ma, S, Sinv, K, flag);
  }
}

}  // namespace oic
