// Ensemble analysis over the whole stored trajectory, Eq. (14b) with Eq. (15c):
//   Xcal^i <- Xcal^i + K (Ybar_t - Ybar^i)   for every member i and every slice k..t,
// which is the lag update that turns the forward pass into a smoother (Eq. (7)).
// As a matrix product: (rows x p) times (p x N*m), added in place.
#include "oic_internal.h"

namespace oic {
namespace {

constexpr int UT_R = 64;  // trajectory rows per tile
constexpr int UT_C = 64;  // columns per tile
constexpr int UT_K = 16;  // observation rows per LDS stage

// traj[a][c] += sum_b K[a][b] (Ybar[b][c mod m] - Y[b][c]),  Ybar = [X^ref_t; 0].
__global__ __launch_bounds__(256) void k_update(Dims d, float* __restrict__ traj, int Ma,
                                                const float* __restrict__ K,
                                                const float* __restrict__ Y,
                                                const float* __restrict__ xref) {
  __shared__ float sK[UT_K][UT_R + 1];
  __shared__ float sE[UT_K][UT_C];
  const long long NM = d.NM();
  const int m = d.m, n = d.n, p = d.p();
  const int r0 = blockIdx.y * UT_R;
  const long long c0 = (long long)blockIdx.x * UT_C;
  const int tid = threadIdx.x;
  const int ty = tid / 16, tx = tid % 16;
  float acc[4][4] = {};
  for (int b0 = 0; b0 < p; b0 += UT_K) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;  // 0..1023
      {  // K tile: 64 rows x 16 observation rows
        const int rl = e / UT_K, bl = e % UT_K;
        const int a = r0 + rl, b = b0 + bl;
        sK[bl][rl] = (a < Ma && b < p) ? K[(size_t)a * p + b] : 0.f;
      }
      {  // innovation tile: 16 observation rows x 64 columns
        const int bl = e / UT_C, cl = e % UT_C;
        const int b = b0 + bl;
        const long long c = c0 + cl;
        float v = 0.f;
        if (b < p && c < NM) {
          const int x = (int)(c % m);
          const float ybar = b < n ? xref[(size_t)b * m + x] : 0.f;
          v = ybar - Y[(size_t)b * NM + c];
        }
        sE[bl][cl] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < UT_K; ++k) {
      float kv[4], ev[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) kv[u] = sK[k][ty + 16 * u];
#pragma unroll
      for (int v = 0; v < 4; ++v) ev[v] = sE[k][tx + 16 * v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fmaf(kv[u], ev[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int a = r0 + ty + 16 * u;
    if (a >= Ma) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const long long c = c0 + tx + 16 * v;
      if (c < NM) traj[(size_t)a * NM + c] += acc[u][v];
    }
  }
}

// Smoothed means of every slice -> U_out (H+1, l, m), X_out (H+1, n, m) and U_hat_k.
__global__ void k_extract(Dims d, const float* __restrict__ mu, float* __restrict__ Uout,
                          float* __restrict__ Xout, float* __restrict__ Uprev) {
  const int rr = d.rr(), m = d.m, n = d.n, l = d.l;
  const long long total = (long long)(d.H + 1) * rr * m;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int x = (int)(idx % m);
  const long long sr = idx / m;
  const int q = (int)(sr % rr);
  const int s = (int)(sr / rr);
  const float v = mu[idx];
  if (q < n) {
    if (Xout) Xout[((size_t)s * n + q) * m + x] = v;
  } else {
    Uout[((size_t)s * l + (q - n)) * m + x] = v;
    if (s == 0) Uprev[(size_t)(q - n) * m + x] = v;
  }
}

}  // namespace

void launch_update(hipStream_t s, Timer& t, const Dims& d, float* traj, int Ma, const float* K,
                   const float* Y, const float* xref_t) {
  const dim3 grid((unsigned)((d.NM() + UT_C - 1) / UT_C), (unsigned)((Ma + UT_R - 1) / UT_R));
  OIC_LAUNCH(t, KC_UPDATE, s, k_update, grid, dim3(256), 0, d, traj, Ma, K, Y, xref_t);
}

void launch_extract(hipStream_t s, Timer& t, const Dims& d, const float* mu_traj, float* Uout,
                    float* Xout, float* Uprev) {
  const long long total = (long long)(d.H + 1) * d.rr() * d.m;
  OIC_LAUNCH(t, KC_EXTRACT, s, k_extract, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, d,
             mu_traj, Uout, Xout, Uprev);
}

}  // namespace oic
