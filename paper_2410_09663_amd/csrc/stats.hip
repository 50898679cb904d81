// Ensemble means and pooled cross-covariances, Eqs. (11), (13a)-(13c).
//
// With the members of each row side by side (N*m columns), the pooled sums
//   Sigma^{XY} ~ sum_i A^i D^iT  and  Sigma^Y ~ sum_i D^i D^iT
// are row-by-row dot products over N*m columns of centred rows.  The factor
// lambda/N of Eq. (13) is dropped: it cancels in the gain.  Products of the
// FP32 anomalies are exact in FP64 and are accumulated in FP64; split-K partial
// sums are reduced in a fixed order (no atomics), so results are deterministic.
#include "oic_internal.h"

namespace oic {
namespace {

// mean[row][x] = (1/N) sum_i A[row][i*m + x], accumulated in FP64.
__global__ void k_means(const float* __restrict__ A, int rows, int N, int m, float* __restrict__ mean) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)rows * m) return;
  const int row = (int)(idx / m), x = (int)(idx - (long long)row * m);
  const float* p = A + (size_t)row * N * m + x;
  double s = 0.0;
  for (int i = 0; i < N; ++i) s += (double)p[(size_t)i * m];
  mean[idx] = (float)(s / N);
}

constexpr int TA = 32;  // rows of the left operand per tile
constexpr int TB = 32;  // rows of the right operand (Y) per tile
constexpr int KT = 32;  // columns per LDS stage

// part[z][a][b] = sum over columns of chunk z of (L[a][c] - muL[a][c mod m]) (Y[b][c] - muY[b][c mod m]),
// where left row a < Ma is trajectory row a and a >= Ma is Y row a - Ma.
__global__ __launch_bounds__(256) void k_stats(Dims d, const float* __restrict__ traj,
                                               const float* __restrict__ mu_traj, int Ma,
                                               const float* __restrict__ Y,
                                               const float* __restrict__ muY, long long chunk,
                                               double* __restrict__ part) {
  __shared__ float sA[KT][TA + 1];
  __shared__ float sB[KT][TB + 1];
  const long long NM = d.NM();
  const int m = d.m, p = d.p();
  const int Mtot = Ma + p;
  const int a0 = blockIdx.x * TA;
  const int b0 = blockIdx.y * TB;
  const long long c_begin = (long long)blockIdx.z * chunk;
  long long c_end = c_begin + chunk;
  if (c_end > NM) c_end = NM;
  const int tid = threadIdx.x;
  const int ty = tid / 16, tx = tid % 16;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};

  for (long long c0 = c_begin; c0 < c_end; c0 += KT) {
    // Load 32 x 32 tiles, centred, transposed into LDS.
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int rloc = tid / KT + 8 * u;
      const int kloc = tid % KT;
      const long long c = c0 + kloc;
      float va = 0.f, vb = 0.f;
      if (c < c_end) {
        const int x = (int)(c % m);
        const int a = a0 + rloc;
        if (a < Mtot) {
          if (a < Ma)
            va = traj[(size_t)a * NM + c] - mu_traj[(size_t)a * m + x];
          else
            va = Y[(size_t)(a - Ma) * NM + c] - muY[(size_t)(a - Ma) * m + x];
        }
        const int b = b0 + rloc;
        if (b < p) vb = Y[(size_t)b * NM + c] - muY[(size_t)b * m + x];
      }
      sA[kloc][rloc] = va;
      sB[kloc][rloc] = vb;
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < KT; ++k) {
      const double x0 = sA[k][2 * ty], x1 = sA[k][2 * ty + 1];
      const double y0 = sB[k][2 * tx], y1 = sB[k][2 * tx + 1];
      acc[0][0] = fma(x0, y0, acc[0][0]);
      acc[0][1] = fma(x0, y1, acc[0][1]);
      acc[1][0] = fma(x1, y0, acc[1][0]);
      acc[1][1] = fma(x1, y1, acc[1][1]);
    }
    __syncthreads();
  }
  double* out = part + (size_t)blockIdx.z * Mtot * p;
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int a = a0 + 2 * ty + u, b = b0 + 2 * tx + v;
      if (a < Mtot && b < p) out[(size_t)a * p + b] = acc[u][v];
    }
}

__global__ void k_stats_reduce(const double* __restrict__ part, int splits, long long count,
                               double* __restrict__ S) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += part[(size_t)z * count + idx];
  S[idx] = s;
}

}  // namespace

void launch_means(hipStream_t s, Timer& t, const float* A, int rows, int N, int m, float* mean) {
  const long long total = (long long)rows * m;
  if (!total) return;
  OIC_LAUNCH(t, KC_MEANS, s, k_means, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, A, rows,
             N, m, mean);
}

void launch_stats(hipStream_t s, Timer& t, const Dims& d, const float* traj, const float* mu_traj,
                  int Ma, const float* Y, const float* muY, double* part, int max_splits,
                  double* S) {
  const int p = d.p();
  const int Mtot = Ma + p;
  const long long NM = d.NM();
  const int tiles = ((Mtot + TA - 1) / TA) * ((p + TB - 1) / TB);
  // Enough split-K chunks to give the chip >= ~1024 workgroups, each chunk >= 256 columns.
  int splits = (1024 + tiles - 1) / tiles;
  const long long max_by_len = (NM + 255) / 256;
  if (splits > max_by_len) splits = (int)max_by_len;
  if (splits > max_splits) splits = max_splits;
  if (splits < 1) splits = 1;
  long long chunk = (NM + splits - 1) / splits;
  chunk = (chunk + KT - 1) / KT * KT;
  splits = (int)((NM + chunk - 1) / chunk);
  const dim3 grid((unsigned)((Mtot + TA - 1) / TA), (unsigned)((p + TB - 1) / TB), (unsigned)splits);
  OIC_LAUNCH(t, KC_STATS, s, k_stats, grid, dim3(256), 0, d, traj, mu_traj, Ma, Y, muY, chunk, part);
  const long long count = (long long)Mtot * p;
  OIC_LAUNCH(t, KC_STATS_REDUCE, s, k_stats_reduce, dim3((unsigned)((count + 255) / 256)), dim3(256),
             0, part, splits, count, S);
}

}  // namespace oic
