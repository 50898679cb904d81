// Ensemble means and pooled cross-covariances, Eqs. (11), (13a)-(13c).
//
// With the members of each row side by side (N*m columns), the pooled sums
//   Sigma^{XY} ~ sum_i A^i D^iT  and  Sigma^Y ~ sum_i D^i D^iT
// are row-by-row dot products over N*m columns.  The factor lambda/N of Eq. (13)
// is dropped: it cancels in the gain.  The products accumulate in FP64 and the
// split-K partial sums are reduced in a fixed order (no atomics), so results are
// deterministic.
#include <atomic>

#include "oic_internal.h"

namespace oic {
namespace {

// mean[row][x] = (1/N) sum_i A[row][i*m + x], accumulated in FP64.
__global__ void k_means(const float* __restrict__ A, int rows, int N, int m, float* __restrict__ mean, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(A);
  OIC_GSH(mean);
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)rows * m) return;
  const int row = (int)(idx / m), x = (int)(idx - (long long)row * m);
  const float* p = A + (size_t)row * N * m + x;
  double s = 0.0;
  for (int i = 0; i < N; ++i) s += (double)p[(size_t)i * m];
  mean[idx] = (float)(s / N);
}

// One block per row when m divides 256: thread t always sees column x = t mod m, sums
// its members in FP64, and the 256/m partial sums of each column are added in a
// fixed order in LDS.
__global__ __launch_bounds__(256) void k_means_rows(const float* __restrict__ A, int N, int m,
                                                    float* __restrict__ mean, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(A);
  OIC_GSH(mean);
  __shared__ double part[256];
  const int row = blockIdx.x;
  const long long NM = (long long)N * m;
  const float* src = A + (size_t)row * NM;
  const int t = threadIdx.x;
  double s = 0.0;
  for (long long c = t; c < NM; c += 256) s += (double)src[c];
  part[t] = s;
  __syncthreads();
  if (t < m) {
    double tot = 0.0;
    for (int g = t; g < 256; g += m) tot += part[g];
    mean[(size_t)row * m + t] = (float)(tot / N);
  }
}

typedef float f32x4m __attribute__((ext_vector_type(4)));

// One block per row, float4 loads: when m is a multiple of 4 that divides 1024, thread
// t always sees columns x = (4t mod m) .. +3; it accumulates them in FP64 over its
// members (loads batched 8 at a time), and the 1024/m partial sums of each column
// are added in a fixed order in LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_means_rows_v4(const float* __restrict__ A, int N, int m,
                                                       T* __restrict__ mean, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(A);
  OIC_GSH(mean);
  __shared__ double part[256][4];
  const int row = blockIdx.x;
  const int NM4 = (N * m) / 4;
  const f32x4m* src = (const f32x4m*)(A + (size_t)row * N * m);
  const int t = threadIdx.x;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int q = t;
  for (; q + 7 * 256 < NM4; q += 8 * 256) {
    f32x4m v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[q + u * 256];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      s0 += (double)v[u][0];
      s1 += (double)v[u][1];
      s2 += (double)v[u][2];
      s3 += (double)v[u][3];
    }
  }
  for (; q < NM4; q += 256) {
    const f32x4m v = src[q];
    s0 += (double)v[0];
    s1 += (double)v[1];
    s2 += (double)v[2];
    s3 += (double)v[3];
  }
  part[t][0] = s0;
  part[t][1] = s1;
  part[t][2] = s2;
  part[t][3] = s3;
  __syncthreads();
  if (t < m) {
    const int g = t / 4, j = t % 4, stride = m / 4;
    double tot = 0.0;
    for (int u = g; u < 256; u += stride) tot += part[u][j];
    mean[(size_t)row * m + t] = (T)(tot / N);
  }
}

// mean[row][x] in FP64 (same reduction order as k_means_rows).
__global__ __launch_bounds__(256) void k_means_rows_f64(const float* __restrict__ A, int N, int m,
                                                        double* __restrict__ mean, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(A);
  OIC_GSH(mean);
  __shared__ double part[256];
  const int row = blockIdx.x;
  const long long NM = (long long)N * m;
  const float* src = A + (size_t)row * NM;
  const int t = threadIdx.x;
  double s = 0.0;
  for (long long c = t; c < NM; c += 256) s += (double)src[c];
  part[t] = s;
  __syncthreads();
  if (t < m) {
    double tot = 0.0;
    for (int g = t; g < 256; g += m) tot += part[g];
    mean[(size_t)row * m + t] = tot / N;
  }
}

__global__ void k_means_f64(const float* __restrict__ A, int rows, int N, int m, double* __restrict__ mean,
                            Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(A);
  OIC_GSH(mean);
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)rows * m) return;
  const int row = (int)(idx / m), x = (int)(idx - (long long)row * m);
  const float* p = A + (size_t)row * N * m + x;
  double s = 0.0;
  for (int i = 0; i < N; ++i) s += (double)p[(size_t)i * m];
  mean[idx] = s / N;
}

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

// Left operands with at least this many rows use 8-wave blocks (128 left rows sharing
// each staged right tile; the right tile is then loaded once per 128 rows, not 64).
constexpr int kStatsTall = 256;
constexpr int MK = 64;  // columns per LDS stage

// part[z][a][b] = sum over the columns c of chunk z of L[a][c] * D[b][c], where the
// left row a is trajectory row a (a < Ma) or Ybar row a - Ma, and the right operand
// D[b][c] = R[b][c] - mean_i R[b][c mod m] is centred in FP64 (R = Ybar for the
// statistics of Eq. (13); R = trajectory rows for the covariances of Eqs. (14c),
// (15d)-(15f)).  Because the
// FP64-centred D sums to zero over the members (to FP64 rounding), the left rows
// need no centring: sum_i X^i D^iT = sum_i (X^i - mean) D^iT.
//
// FP64 matrix cores (v_mfma_f64_16x16x4_f64); a block of WL waves owns 16*WL left rows
// and NB*16 right rows; wave w computes left rows 16w..16w+15 against all NB
// blocks.  Lane layout: A[i][k] from lane i + 16k, B[k][j] from lane j + 16k,
// element r of lane j + 16g holds D[g + 4r][j].  VEC: rows are 16-byte aligned
// (N*m divisible by 4) and loaded as float4, one stage ahead of the compute.
template <int NB, bool VEC, int WL>  // WL waves, 16 left rows each
__global__ __launch_bounds__(64 * WL) void k_stats_mfma(Dims d, const float* __restrict__ traj, int Ma,
                                                    int ny, const float* __restrict__ Y,
                                                    const float* __restrict__ R, int p,
                                                    const double* __restrict__ muY, int chunk,
                                                    double* __restrict__ part) {
  // right operand: the p rows of R (Ybar for the statistics), centred by muY
  constexpr int RB = NB * 16;
  constexpr int MA_ = 16 * WL, NT = 64 * WL;
  __shared__ float sA[MA_][MK + 1];
  __shared__ double sB[RB][MK + 1];
  const int NM = (int)d.NM();
  const int m = d.m;
  const int Mtot = Ma + ny;
  const int a0 = blockIdx.x * MA_;
  const int b0 = blockIdx.y * RB;
  const int c_begin = blockIdx.z * chunk;
  const int c_end = min(c_begin + chunk, NM);
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  f64x4 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = f64x4{0.0, 0.0, 0.0, 0.0};

  // per-thread load slots: A tile = MA_ rows x 64 cols; B tile = RB rows x 64 cols
  constexpr int AV = MA_ * MK / 4 / NT;  // float4 slots per thread (4)
  constexpr int BQ = RB * MK / 4;  // float4 slots of the right tile
  constexpr int BV = (BQ + NT - 1) / NT;  // (last slot guarded when NT does not divide BQ)
  f32x4v ra[AV], rb[BV];
  auto left_row = [&](int a) -> const float* {
    return a < Ma ? traj + (size_t)a * NM : Y + (size_t)(a - Ma) * NM;
  };
  auto load_stage = [&](int c0) {
#pragma unroll
    for (int u = 0; u < AV; ++u) {
      const int e = tid + NT * u;
      const int r = e / (MK / 4), q = e % (MK / 4);
      const int a = a0 + r, c = c0 + 4 * q;
      f32x4v v = {0.f, 0.f, 0.f, 0.f};
      if (a < Mtot) {
        const float* src = left_row(a);
        if (VEC) {
          if (c < c_end) v = *(const f32x4v*)(src + c);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] = (c + j < c_end) ? src[c + j] : 0.f;
        }
      }
      ra[u] = v;
    }
#pragma unroll
    for (int u = 0; u < BV; ++u) {
      const int e = tid + NT * u;
      const int r = e / (MK / 4), q = e % (MK / 4);
      const int b = b0 + r, c = c0 + 4 * q;
      f32x4v v = {0.f, 0.f, 0.f, 0.f};
      if (e < BQ && b < p) {
        const float* src = R + (size_t)b * NM;
        if (VEC) {
          if (c < c_end) v = *(const f32x4v*)(src + c);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] = (c + j < c_end) ? src[c + j] : 0.f;
        }
      }
      rb[u] = v;
    }
  };
  if (c_begin < c_end) load_stage(c_begin);
  for (int c0 = c_begin; c0 < c_end; c0 += MK) {
    // registers -> LDS (right operand centred in FP64)
#pragma unroll
    for (int u = 0; u < AV; ++u) {
      const int e = tid + NT * u;
      const int r = e / (MK / 4), q = e % (MK / 4);
#pragma unroll
      for (int j = 0; j < 4; ++j) sA[r][4 * q + j] = ra[u][j];
    }
#pragma unroll
    for (int u = 0; u < BV; ++u) {
      const int e = tid + NT * u;
      if (e >= BQ) continue;
      const int r = e / (MK / 4), q = e % (MK / 4);
      const int b = b0 + r, c = c0 + 4 * q;
      int x = c % m;
      const double* mu = muY + (size_t)(b < p ? b : 0) * m;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool live = b < p && c + j < c_end;
        sB[r][4 * q + j] = live ? (double)rb[u][j] - mu[x] : 0.0;
        x = (x + 1 == m) ? 0 : x + 1;
      }
    }
    __syncthreads();
    if (c0 + MK < c_end) load_stage(c0 + MK);  // prefetch the next stage
#pragma unroll 4
    for (int kk = 0; kk < MK; kk += 4) {
      const double av = (double)sA[w * 16 + li][kk + lk];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, sB[nb * 16 + li][kk + lk], acc[nb], 0, 0, 0);
    }
    __syncthreads();
  }
  double* out = part + (size_t)blockIdx.z * Mtot * p;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = a0 + w * 16 + lk + 4 * r;
      const int b = b0 + nb * 16 + li;
      if (a < Mtot && b < p) out[(size_t)a * p + b] = acc[nb][r];
    }
}

// The same products for the mixed-precision modes on the FP32 matrix cores
// (v_mfma_f32_16x16x4_f32, twice the FP64 rate): the right operand is centred in FP64 and
// rounded to FP32, products accumulate in FP32 over at most four 64-column stages and are
// then folded into FP64 registers, and the split partials are summed in FP64 as before.
// Lane layout (16x16x4 f32): A[i][k] from lane i + 16k, B[k][j] from lane j + 16k,
// element r of lane j + 16g holds D[4g + r][j].
template <int NB, bool VEC, int WL>  // WL waves, 16 left rows each
__global__ __launch_bounds__(64 * WL) void k_stats_mfma32(Dims d, const float* __restrict__ traj, int Ma,
                                                      int ny, const float* __restrict__ Y,
                                                      const float* __restrict__ R, int p,
                                                      const double* __restrict__ muY, int chunk,
                                                      double* __restrict__ part) {
  constexpr int RB = NB * 16;
  constexpr int MA_ = 16 * WL, NT = 64 * WL;
  __shared__ float sA[MA_][MK + 1];
  __shared__ float sB[RB][MK + 1];
  const int NM = (int)d.NM();
  const int m = d.m;
  const int Mtot = Ma + ny;
  const int a0 = blockIdx.x * MA_;
  const int b0 = blockIdx.y * RB;
  const int c_begin = blockIdx.z * chunk;
  const int c_end = min(c_begin + chunk, NM);
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  f32x4v acc[NB];
  f64x4 tot[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    acc[nb] = f32x4v{0.f, 0.f, 0.f, 0.f};
    tot[nb] = f64x4{0.0, 0.0, 0.0, 0.0};
  }
  constexpr int AV = MA_ * MK / 4 / NT;
  constexpr int BQ = RB * MK / 4;  // float4 slots of the right tile
  constexpr int BV = (BQ + NT - 1) / NT;
  f32x4v ra[AV], rb[BV];
  auto left_row = [&](int a) -> const float* {
    return a < Ma ? traj + (size_t)a * NM : Y + (size_t)(a - Ma) * NM;
  };
  auto load_stage = [&](int c0) {
#pragma unroll
    for (int u = 0; u < AV; ++u) {
      const int e = tid + NT * u;
      const int r = e / (MK / 4), q = e % (MK / 4);
      const int a = a0 + r, c = c0 + 4 * q;
      f32x4v v = {0.f, 0.f, 0.f, 0.f};
      if (a < Mtot) {
        const float* src = left_row(a);
        if (VEC) {
          if (c < c_end) v = *(const f32x4v*)(src + c);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] = (c + j < c_end) ? src[c + j] : 0.f;
        }
      }
      ra[u] = v;
    }
#pragma unroll
    for (int u = 0; u < BV; ++u) {
      const int e = tid + NT * u;
      const int r = e / (MK / 4), q = e % (MK / 4);
      const int b = b0 + r, c = c0 + 4 * q;
      f32x4v v = {0.f, 0.f, 0.f, 0.f};
      if (e < BQ && b < p) {
        const float* src = R + (size_t)b * NM;
        if (VEC) {
          if (c < c_end) v = *(const f32x4v*)(src + c);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] = (c + j < c_end) ? src[c + j] : 0.f;
        }
      }
      rb[u] = v;
    }
  };
  if (c_begin < c_end) load_stage(c_begin);
  int stage = 0;
  for (int c0 = c_begin; c0 < c_end; c0 += MK, ++stage) {
#pragma unroll
    for (int u = 0; u < AV; ++u) {
      const int e = tid + NT * u;
      const int r = e / (MK / 4), q = e % (MK / 4);
#pragma unroll
      for (int j = 0; j < 4; ++j) sA[r][4 * q + j] = ra[u][j];
    }
#pragma unroll
    for (int u = 0; u < BV; ++u) {
      const int e = tid + NT * u;
      if (e >= BQ) continue;
      const int r = e / (MK / 4), q = e % (MK / 4);
      const int b = b0 + r, c = c0 + 4 * q;
      int x = c % m;
      const double* mu = muY + (size_t)(b < p ? b : 0) * m;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool live = b < p && c + j < c_end;
        sB[r][4 * q + j] = live ? (float)((double)rb[u][j] - mu[x]) : 0.f;
        x = (x + 1 == m) ? 0 : x + 1;
      }
    }
    __syncthreads();
    if (c0 + MK < c_end) load_stage(c0 + MK);  // prefetch the next stage
#pragma unroll 4
    for (int kk = 0; kk < MK; kk += 4) {
      const float av = sA[w * 16 + li][kk + lk];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, sB[nb * 16 + li][kk + lk], acc[nb], 0, 0, 0);
    }
    if ((stage & 3) == 3) {  // fold the FP32 sums of the last four stages into FP64
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) tot[nb][r] += (double)acc[nb][r];
        acc[nb] = f32x4v{0.f, 0.f, 0.f, 0.f};
      }
    }
    __syncthreads();
  }
  double* out = part + (size_t)blockIdx.z * Mtot * p;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = a0 + w * 16 + 4 * lk + r;
      const int b = b0 + nb * 16 + li;
      if (a < Mtot && b < p) out[(size_t)a * p + b] = tot[nb][r] + (double)acc[nb][r];
    }
}

// The FP32-matrix-core products again, for row lengths N*m divisible by 4, with less LDS
// traffic: a lane reads its A fragments straight from global memory into registers (each
// left row belongs to one wave, so it gains nothing from LDS), eight 16-column groups of a
// 128-column stage as 16-byte loads, and only the centred right tile goes through LDS,
// double-buffered so that one barrier per stage suffices.  K is permuted inside each
// 16-column group: lane (i, g) supplies columns 4g..4g+3 of its row to four MFMAs, the
// j-th taking column 4g+j in k-slot g, and reads the same four columns of the right rows
// as one 16-byte LDS load.  Sums as in k_stats_mfma32: FP32 over 256 columns, then FP64.
constexpr int SV_W = 8;          // waves per block, 16 left rows each
constexpr int SV_MK = 128;       // columns per stage: 8 groups of 16, about 2 us of MFMAs per wave
constexpr int SV_CP = SV_MK + 4;  // right-tile row stride in LDS (16-byte reads without bank conflicts)
template <int NB, bool CENTRED>  // CENTRED: R holds the centred rows already (muY unused)
__global__ __launch_bounds__(64 * SV_W) void k_stats_v4(Dims d, const float* __restrict__ traj, int Ma, int ny,
                                                        const float* __restrict__ Y, const float* __restrict__ R,
                                                        int p, const double* __restrict__ muY, int chunk,
                                                        int xt, int ytiles, int tiles,
                                                        double* __restrict__ part) {
  constexpr int RB = NB * 16, NT = 64 * SV_W;
  // XCD-aware tile order (workgroup b runs on XCD b mod 8): the workgroups of one XCD take
  // consecutive logical tiles, whose right tiles vary fastest, so the left rows they share
  // and the right-tile stages of one split are read into that XCD's L2 once
  const int G = gridDim.x;
  const int L = (G & 7) ? (int)blockIdx.x : (int)(blockIdx.x & 7) * (G >> 3) + (int)(blockIdx.x >> 3);
  if (L >= tiles) return;
  const int ty = L % ytiles, tx = (L / ytiles) % xt, tz = L / (ytiles * xt);
  constexpr int GR = SV_MK / 16;             // 16-column groups per stage
  constexpr int BQ = RB * SV_MK / 4;         // float4 of the right tile
  constexpr int BV = (BQ + NT - 1) / NT;
  __shared__ __attribute__((aligned(16))) float sB[2][RB * SV_CP];
  const int NM = (int)d.NM();
  const int m = d.m;
  const int Mtot = Ma + ny;
  const int a0 = tx * (16 * SV_W);
  const int b0 = ty * RB;
  const int c_begin = tz * chunk;
  const int c_end = min(c_begin + chunk, NM);
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int arow = a0 + 16 * w + li;
  const float* asrc = arow < Mtot ? (arow < Ma ? traj + (size_t)arow * NM : Y + (size_t)(arow - Ma) * NM) : nullptr;
  f32x4v acc[NB];
  f64x4 tot[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    acc[nb] = f32x4v{0.f, 0.f, 0.f, 0.f};
    tot[nb] = f64x4{0.0, 0.0, 0.0, 0.0};
  }
  f32x4v an[GR], bn[BV];
  auto load_stage = [&](int c0) {
#pragma unroll
    for (int g = 0; g < GR; ++g) {
      const int c = c0 + 16 * g + 4 * lk;
      an[g] = (asrc && c < c_end) ? *(const f32x4v*)(asrc + c) : f32x4v{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int u = 0; u < BV; ++u) {
      const int e = tid + NT * u;
      const int r = e / (SV_MK / 4), q = e % (SV_MK / 4);
      const int b = b0 + r, c = c0 + 4 * q;
      bn[u] = (e < BQ && b < p && c < c_end) ? *(const f32x4v*)(R + (size_t)b * NM + c)
                                             : f32x4v{0.f, 0.f, 0.f, 0.f};
    }
  };
  if (c_begin < c_end) load_stage(c_begin);
  int stage = 0;
  for (int c0 = c_begin; c0 < c_end; c0 += SV_MK, ++stage) {
    float* const sb = sB[stage & 1];
    f32x4v ac[GR];
#pragma unroll
    for (int g = 0; g < GR; ++g) ac[g] = an[g];
    // right tile centred in FP64, rounded to FP32 (zero past the chunk and past p)
#pragma unroll
    for (int u = 0; u < BV; ++u) {
      const int e = tid + NT * u;
      if (e >= BQ) continue;
      const int r = e / (SV_MK / 4), q = e % (SV_MK / 4);
      f32x4v v = bn[u];  // zero past the chunk and past p already
      if constexpr (!CENTRED) {
        const int b = b0 + r, c = c0 + 4 * q;
        int x = c % m;
        const double* mu = muY + (size_t)(b < p ? b : 0) * m;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool live = b < p && c + j < c_end;
          v[j] = live ? (float)((double)bn[u][j] - mu[x]) : 0.f;
          x = (x + 1 == m) ? 0 : x + 1;
        }
      }
      *(f32x4v*)(sb + r * SV_CP + 4 * q) = v;
    }
    __syncthreads();  // this stage's right tile is in LDS; the other buffer is free again
    if (c0 + SV_MK < c_end) load_stage(c0 + SV_MK);  // the next stage's operands, in flight meanwhile
#pragma unroll
    for (int g = 0; g < GR; ++g)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const f32x4v b = *(const f32x4v*)(sb + (16 * nb + li) * SV_CP + 16 * g + 4 * lk);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[g][j], b[j], acc[nb], 0, 0, 0);
      }
    if ((stage & 1) == 1) {  // fold the FP32 sums of the last 256 columns into FP64
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) tot[nb][r] += (double)acc[nb][r];
        acc[nb] = f32x4v{0.f, 0.f, 0.f, 0.f};
      }
    }
  }
  double* out = part + (size_t)tz * Mtot * p;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = a0 + 16 * w + 4 * lk + r;
      const int b = b0 + nb * 16 + li;
      if (a < Mtot && b < p) out[(size_t)a * p + b] = tot[nb][r] + (double)acc[nb][r];
    }
}

// Split of FP32 values into BF16 pairs v ~ hi + lo (hi = v rounded to nearest BF16, lo =
// the rounded remainder v - hi, which FP32 holds exactly): the pair keeps 16 significant
// bits, and hi_a hi_b + hi_a lo_b + lo_a hi_b misses a product by about 2^-16 of it (the
// dropped lo_a lo_b and the remainders below lo).
typedef __bf16 bf16x8s __attribute__((ext_vector_type(8)));
typedef float f32x2s __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2s __attribute__((ext_vector_type(2)));
typedef unsigned u32x4s __attribute__((ext_vector_type(4)));
typedef unsigned u32x2s __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split2(float v0, float v1, unsigned& hi, unsigned& lo) {
  hi = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2s{v0, v1}, bf16x2s));
  const float h0 = __uint_as_float(hi << 16), h1 = __uint_as_float(hi & 0xffff0000u);
  lo = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2s{v0 - h0, v1 - h1}, bf16x2s));
}

// The FP32 statistics of the BF16 and FP8 modes with the products split into three BF16
// matrix-core products (v_mfma_f32_16x16x32_bf16: hi hi + hi lo + lo hi, FP32 accumulation,
// relative error about 2^-16 per product, far below those modes' rollout error), at a
// sixth of the FP32 matrix-core cycles.  Same tiling, XCD-aware order, FP64 fold every 256
// columns and split-K partials as k_stats_v4.  K steps of 32 columns: lane (i, g) reads
// columns 8g..8g+7 of its left row (two 16-byte loads) and splits them in registers; the
// centred right tile is split once while staged and sits in LDS as two BF16 planes (hi,
// lo), from which a lane reads the same 8 columns of a right row as one 16-byte load each.
constexpr int SB_CP = SV_MK + 8;  // right-plane row stride in LDS (BF16): 272 bytes
template <int NB>
__global__ __launch_bounds__(64 * SV_W) void k_stats_b3(Dims d, const float* __restrict__ traj, int Ma, int ny,
                                                        const float* __restrict__ Y, const float* __restrict__ Rc,
                                                        int p, int chunk, int xt, int ytiles, int tiles,
                                                        double* __restrict__ part, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(traj);
  OIC_GSH(Y);
  OIC_GSH(Rc);
  OIC_GSH(part);
  constexpr int RB = NB * 16, NT = 64 * SV_W;
  const int G = gridDim.x;
  const int L = (G & 7) ? (int)blockIdx.x : (int)(blockIdx.x & 7) * (G >> 3) + (int)(blockIdx.x >> 3);
  if (L >= tiles) return;
  const int ty = L % ytiles, tx = (L / ytiles) % xt, tz = L / (ytiles * xt);
  constexpr int GR = SV_MK / 32;             // 32-column K steps per stage
  constexpr int BQ = RB * SV_MK / 4;         // float4 of the right tile
  constexpr int BV = (BQ + NT - 1) / NT;
  __shared__ __attribute__((aligned(16))) __bf16 sB[2][2][RB * SB_CP];  // [stage][hi, lo]
  const int NM = (int)d.NM();
  const int Mtot = Ma + ny;
  const int a0 = tx * (16 * SV_W);
  const int b0 = ty * RB;
  const int c_begin = tz * chunk;
  const int c_end = min(c_begin + chunk, NM);
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int arow = a0 + 16 * w + li;
  const float* asrc = arow < Mtot ? (arow < Ma ? traj + (size_t)arow * NM : Y + (size_t)(arow - Ma) * NM) : nullptr;
  f32x4v acc[NB];
  f64x4 tot[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    acc[nb] = f32x4v{0.f, 0.f, 0.f, 0.f};
    tot[nb] = f64x4{0.0, 0.0, 0.0, 0.0};
  }
  f32x4v an[GR][2], bn[BV];
  auto load_stage = [&](int c0) {
#pragma unroll
    for (int g = 0; g < GR; ++g)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int c = c0 + 32 * g + 8 * lk + 4 * h;
        an[g][h] = (asrc && c < c_end) ? *(const f32x4v*)(asrc + c) : f32x4v{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
    for (int u = 0; u < BV; ++u) {
      const int e = tid + NT * u;
      const int r = e / (SV_MK / 4), q = e % (SV_MK / 4);
      const int b = b0 + r, c = c0 + 4 * q;
      bn[u] = (e < BQ && b < p && c < c_end) ? *(const f32x4v*)(Rc + (size_t)b * NM + c)
                                             : f32x4v{0.f, 0.f, 0.f, 0.f};
    }
  };
  if (c_begin < c_end) load_stage(c_begin);
  int stage = 0;
  for (int c0 = c_begin; c0 < c_end; c0 += SV_MK, ++stage) {
    __bf16* const sh = sB[stage & 1][0];
    __bf16* const sl = sB[stage & 1][1];
    // this stage's left fragments, split
    bf16x8s ah[GR], al[GR];
#pragma unroll
    for (int g = 0; g < GR; ++g) {
      unsigned h[4], lo[4];
      split2(an[g][0][0], an[g][0][1], h[0], lo[0]);
      split2(an[g][0][2], an[g][0][3], h[1], lo[1]);
      split2(an[g][1][0], an[g][1][1], h[2], lo[2]);
      split2(an[g][1][2], an[g][1][3], h[3], lo[3]);
      ah[g] = __builtin_bit_cast(bf16x8s, u32x4s{h[0], h[1], h[2], h[3]});
      al[g] = __builtin_bit_cast(bf16x8s, u32x4s{lo[0], lo[1], lo[2], lo[3]});
    }
    // the right tile, split into its two planes (zero past the chunk and past p already)
#pragma unroll
    for (int u = 0; u < BV; ++u) {
      const int e = tid + NT * u;
      if (e >= BQ) continue;
      const int r = e / (SV_MK / 4), q = e % (SV_MK / 4);
      unsigned h[2], lo[2];
      split2(bn[u][0], bn[u][1], h[0], lo[0]);
      split2(bn[u][2], bn[u][3], h[1], lo[1]);
      *(u32x2s*)(sh + r * SB_CP + 4 * q) = u32x2s{h[0], h[1]};
      *(u32x2s*)(sl + r * SB_CP + 4 * q) = u32x2s{lo[0], lo[1]};
    }
    __syncthreads();  // this stage's right planes are in LDS; the other buffer is free again
    if (c0 + SV_MK < c_end) load_stage(c0 + SV_MK);  // the next stage's operands, in flight meanwhile
#pragma unroll
    for (int g = 0; g < GR; ++g)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int off = (16 * nb + li) * SB_CP + 32 * g + 8 * lk;
        const bf16x8s bh = *(const bf16x8s*)(sh + off);
        const bf16x8s bl = *(const bf16x8s*)(sl + off);
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[g], bh, acc[nb], 0, 0, 0);
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[g], bl, acc[nb], 0, 0, 0);
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[g], bh, acc[nb], 0, 0, 0);
      }
    if ((stage & 1) == 1) {  // fold the FP32 sums of the last 256 columns into FP64
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) tot[nb][r] += (double)acc[nb][r];
        acc[nb] = f32x4v{0.f, 0.f, 0.f, 0.f};
      }
    }
  }
  double* out = part + (size_t)tz * Mtot * p;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = a0 + 16 * w + 4 * lk + r;
      const int b = b0 + nb * 16 + li;
      if (a < Mtot && b < p) out[(size_t)a * p + b] = tot[nb][r] + (double)acc[nb][r];
    }
}

// Rc[b][c] = R[b][c] - mu[b][c mod m], the subtraction in FP64, rounded to FP32: the
// centred right operand of the FP32 statistics, formed once per horizon step instead of
// in every workgroup's staging (there its FP64 mean loads sat between each stage's loads
// and its barrier).
__global__ __launch_bounds__(256) void k_center_rows(const float* __restrict__ R, int rows, int NM, int m,
                                                     const double* __restrict__ mu, float* __restrict__ Rc,
                                                     Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(R);
  OIC_GSH(mu);
  OIC_GSH(Rc);
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;  // float4 index
  const long long total = (long long)rows * NM / 4;
  if (q >= total) return;
  const long long e = 4 * q;
  const int b = (int)(e / NM), c = (int)(e - (long long)b * NM);
  const f32x4v v = *(const f32x4v*)(R + e);
  const double* mb = mu + (size_t)b * m;
  int x = c % m;
  f32x4v o;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    o[j] = (float)((double)v[j] - mb[x]);
    x = (x + 1 == m) ? 0 : x + 1;
  }
  *(f32x4v*)(Rc + e) = o;
}

// S[idx] = scale * sum_z part[z][idx].  Block (64, RG): lane x owns output idx, and the
// RG threads of a column sum interleaved subsets of the splits (z = y, y + RG, ...), which
// are then added in the order y = 0, 1, ..., RG - 1: a fixed order, so the result is
// the same on every run.
constexpr int RG = 8;
__global__ __launch_bounds__(64 * RG) void k_stats_reduce(const double* __restrict__ part, int splits,
                                                          long long count, double scale,
                                                          double* __restrict__ S, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(part);
  OIC_GSH(S);
  __shared__ double sub[RG][64];
  const long long idx = (long long)blockIdx.x * 64 + threadIdx.x;
  const int y = threadIdx.y;
  double s = 0.0;
  if (idx < count) {
    int z = y;
    for (; z + 3 * RG < splits; z += 4 * RG) {  // four loads in flight, summed in order
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = part[(size_t)(z + u * RG) * count + idx];
#pragma unroll
      for (int u = 0; u < 4; ++u) s += v[u];
    }
    for (; z < splits; z += RG) s += part[(size_t)z * count + idx];
  }
  sub[y][threadIdx.x] = s;
  __syncthreads();
  if (y == 0 && idx < count) {
    double tot = sub[0][threadIdx.x];
#pragma unroll
    for (int g = 1; g < RG; ++g) tot += sub[g][threadIdx.x];
    S[idx] = scale * tot;
  }
}

}  // namespace

static bool means_v4_ok(int N, int m) { return m % 4 == 0 && 1024 % m == 0 && ((long long)N * m) % 4 == 0; }

void launch_means(hipStream_t s, Timer& t, const float* A, int rows, int N, int m, float* mean) {
  const long long total = (long long)rows * m;
  if (!total) return;
  if (means_v4_ok(N, m)) {
    OIC_GLAUNCH(t, KC_MEANS, s, k_means_rows_v4<float>, dim3((unsigned)rows), dim3(256), 0, A, N, m, mean);
    return;
  }
  if (m <= 256 && 256 % m == 0) {
    OIC_GLAUNCH(t, KC_MEANS, s, k_means_rows, dim3((unsigned)rows), dim3(256), 0, A, N, m, mean);
    return;
  }
  OIC_GLAUNCH(t, KC_MEANS, s, k_means, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, A, rows,
             N, m, mean);
}

void launch_means_f64(hipStream_t s, Timer& t, const float* A, int rows, int N, int m, double* mean) {
  const long long total = (long long)rows * m;
  if (!total) return;
  if (means_v4_ok(N, m)) {
    OIC_GLAUNCH(t, KC_MEANS, s, k_means_rows_v4<double>, dim3((unsigned)rows), dim3(256), 0, A, N, m, mean);
    return;
  }
  if (m <= 256 && 256 % m == 0) {
    OIC_GLAUNCH(t, KC_MEANS, s, k_means_rows_f64, dim3((unsigned)rows), dim3(256), 0, A, N, m, mean);
    return;
  }
  OIC_GLAUNCH(t, KC_MEANS, s, k_means_f64, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, A,
             rows, N, m, mean);
}

void launch_center(hipStream_t s, Timer& t, const float* R, int rows, int NM, int m, const double* mu,
                   float* Rc) {
  const long long total = (long long)rows * NM / 4;
  OIC_GLAUNCH(t, KC_MEANS, s, k_center_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, R, rows, NM, m,
             mu, Rc);
}

// Compute units of the current device, read once per device.
int device_cus() {
  static std::atomic<int> cus[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int v = cus[dev].load(std::memory_order_relaxed);
  if (v > 0) return v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) return 256;
  cus[dev].store(v, std::memory_order_relaxed);
  return v;
}

void launch_cross(hipStream_t s, Timer& t, const Dims& d, const float* traj, int Ma, int ny,
                  const float* Y, const float* R, int p, const double* muR, double* part, size_t part_cap,
                  double* S, double scale, bool f32, const float* Rc, bool b3) {
  const int Mtot = Ma + ny;
  const int NM = (int)d.NM();
  if (f32 && NM % 4 == 0) {
    // right rows per block: NB*16 with NB <= 7, balanced over grid.y tiles
    const int nbk = (p + 15) / 16;
    const int ytiles = (nbk + 6) / 7;
    const int NBv = (nbk + ytiles - 1) / ytiles;
    const int xt = (Mtot + 16 * SV_W - 1) / (16 * SV_W);
    const int tiles = xt * ytiles;
    // K split: a workgroup's time is set by its chunk of K, and one eight-wave workgroup fits
    // a CU (its LDS), so the launch takes ceil(tiles * splits / CUs) rounds of one chunk each.
    // Choose the split count that minimises rounds x (chunk + two stages of fixed cost per
    // workgroup); chunks are whole SV_MK-column stages and the partials must fit the split
    // buffer.  (At 256x256, N = 512: 12 to 220 tiles over the horizon; "enough splits for
    // two rounds" left a third round of a few workgroups on most steps.)
    const int slots = device_cus();
    int max_splits = (NM + SV_MK - 1) / SV_MK;
    const size_t by_cap = part_cap / ((size_t)Mtot * p);
    if ((size_t)max_splits > by_cap) max_splits = (int)by_cap;
    if (max_splits > 64) max_splits = 64;
    int splits = 1, chunk = (NM + SV_MK - 1) / SV_MK * SV_MK;
    long long best = -1;
    for (int sp = 1; sp <= max_splits; ++sp) {
      const int ch = ((NM + sp - 1) / sp + SV_MK - 1) / SV_MK * SV_MK;
      const int eff = (NM + ch - 1) / ch;
      const long long rounds = ((long long)tiles * eff + slots - 1) / slots;
      const long long cost = rounds * (ch + 2 * SV_MK);
      if (best < 0 || cost < best) {
        best = cost;
        splits = eff;
        chunk = ch;
      }
    }
    const int all = tiles * splits;
    const dim3 grid((unsigned)((all + 7) / 8 * 8));  // whole groups of eight for the XCD order
    switch (NBv) {
#define OIC_SV_CASE(NBV)                                                                                 \
  case NBV:                                                                                              \
    if (Rc && b3)                                                                                        \
      OIC_GLAUNCH(t, KC_STATS, s, k_stats_b3<NBV>, grid, dim3(64 * SV_W), 0, d, traj, Ma, ny, Y, Rc, p, chunk, \
                 xt, ytiles, all, part);                                                                 \
    else if (Rc)                                                                                         \
      OIC_LAUNCH(t, KC_STATS, s, (k_stats_v4<NBV, true>), grid, dim3(64 * SV_W), 0, d, traj, Ma, ny, Y, Rc, p, \
                 muR, chunk, xt, ytiles, all, part);                                                     \
    else                                                                                                 \
      OIC_LAUNCH(t, KC_STATS, s, (k_stats_v4<NBV, false>), grid, dim3(64 * SV_W), 0, d, traj, Ma, ny, Y, R, p, \
                 muR, chunk, xt, ytiles, all, part);                                                     \
    break;
      OIC_SV_CASE(1) OIC_SV_CASE(2) OIC_SV_CASE(3) OIC_SV_CASE(4) OIC_SV_CASE(5) OIC_SV_CASE(6)
      OIC_SV_CASE(7)
#undef OIC_SV_CASE
    }
    const long long count = (long long)Mtot * p;
    OIC_GLAUNCH(t, KC_STATS_REDUCE, s, k_stats_reduce, dim3((unsigned)((count + 63) / 64)), dim3(64, RG), 0,
               part, splits, count, scale, S);
    return;
  }
  // right rows per block: NB*16 with NB <= 8, balanced over grid.y tiles
  const int nbk = (p + 15) / 16;
  const int ytiles = (nbk + 7) / 8;
  const int NB = (nbk + ytiles - 1) / ytiles;
  // eight waves (128 left rows) share each staged right tile once the left side is tall
  const bool tall = Mtot >= kStatsTall;
  const int ma = tall ? 128 : 64;
  const int tiles = ((Mtot + ma - 1) / ma) * ytiles;
  // Split K so that about two workgroups per CU (their LDS allows two) are in flight
  // even for the few output tiles of the early horizon steps: a workgroup's time is set
  // by its chunk of K, not by the size of the output.  Chunks are whole 64-column
  // stages; the partials must fit the split buffer.
  // Eight-wave blocks: 256 of them (the same waves in flight as 512 four-wave blocks) while
  // the one-workgroup Cholesky of Sigma^Y (p <= 90) runs beside this product, leaving it
  // room on the CUs; 384 otherwise (128x128 BF16: statistics 3.20 -> 2.75 ms per solve;
  // at 64x64 FP32, 384 or 512 cost 0.5-2% per step).
  const int target = tall ? (chol_blocked(p) ? 384 : 256) : 512;
  int splits = (target + tiles - 1) / tiles;
  const int max_by_len = (NM + MK - 1) / MK;
  if (splits > max_by_len) splits = max_by_len;
  const size_t by_cap = part_cap / ((size_t)Mtot * p);
  if ((size_t)splits > by_cap) splits = (int)by_cap;
  if (splits < 1) splits = 1;
  int chunk = (NM + splits - 1) / splits;
  chunk = (chunk + MK - 1) / MK * MK;
  splits = (NM + chunk - 1) / chunk;
  if (tall) {
    // one eight-wave workgroup per CU (its LDS): as for the FP32 product above, the split
    // count that minimises rounds x (chunk + two stages of fixed cost) over the CUs
    const int slots = device_cus();
    int max_splits = max_by_len;
    if ((size_t)max_splits > by_cap) max_splits = (int)by_cap;
    if (max_splits > 64) max_splits = 64;
    long long best = -1;
    for (int sp = 1; sp <= max_splits; ++sp) {
      const int ch = ((NM + sp - 1) / sp + MK - 1) / MK * MK;
      const int eff = (NM + ch - 1) / ch;
      const long long cost = (((long long)tiles * eff + slots - 1) / slots) * (ch + 2 * MK);
      if (best < 0 || cost < best) {
        best = cost;
        splits = eff;
        chunk = ch;
      }
    }
  }
  const dim3 grid((unsigned)((Mtot + ma - 1) / ma), (unsigned)ytiles, (unsigned)splits);
  const bool vec = NM % 4 == 0;
#define OIC_STATS_LAUNCH(KERN, NBV, WLV)                                                        \
  OIC_LAUNCH(t, KC_STATS, s, (KERN<NBV, true, WLV>), grid, dim3(64 * WLV), 0, d, traj, Ma, ny, Y, R, p, \
             muR, chunk, part)
#define OIC_STATS_LAUNCH_NV(KERN, NBV, WLV)                                                     \
  OIC_LAUNCH(t, KC_STATS, s, (KERN<NBV, false, WLV>), grid, dim3(64 * WLV), 0, d, traj, Ma, ny, Y, R, \
             p, muR, chunk, part)
#define OIC_STATS_CASE(NBV)                                                                     \
  case NBV:                                                                                     \
    if (f32) {                                                                                  \
      if (vec) {                                                                                \
        if (tall) OIC_STATS_LAUNCH(k_stats_mfma32, NBV, 8); else OIC_STATS_LAUNCH(k_stats_mfma32, NBV, 4); \
      } else {                                                                                  \
        if (tall) OIC_STATS_LAUNCH_NV(k_stats_mfma32, NBV, 8); else OIC_STATS_LAUNCH_NV(k_stats_mfma32, NBV, 4); \
      }                                                                                         \
    } else {                                                                                    \
      if (vec) {                                                                                \
        if (tall) OIC_STATS_LAUNCH(k_stats_mfma, NBV, 8); else OIC_STATS_LAUNCH(k_stats_mfma, NBV, 4); \
      } else {                                                                                  \
        if (tall) OIC_STATS_LAUNCH_NV(k_stats_mfma, NBV, 8); else OIC_STATS_LAUNCH_NV(k_stats_mfma, NBV, 4); \
      }                                                                                         \
    }                                                                                           \
    break;
  switch (NB) {
    OIC_STATS_CASE(1) OIC_STATS_CASE(2) OIC_STATS_CASE(3) OIC_STATS_CASE(4)
    OIC_STATS_CASE(5) OIC_STATS_CASE(6) OIC_STATS_CASE(7) OIC_STATS_CASE(8)
  }
#undef OIC_STATS_CASE
#undef OIC_STATS_LAUNCH
#undef OIC_STATS_LAUNCH_NV
  const long long count = (long long)Mtot * p;
  OIC_GLAUNCH(t, KC_STATS_REDUCE, s, k_stats_reduce, dim3((unsigned)((count + 63) / 64)), dim3(64, RG), 0,
             part, splits, count, scale, S);
}

void launch_stats(hipStream_t s, Timer& t, const Dims& d, const float* traj, int Ma, int ny,
                  const float* Y, const double* muY, double* part, size_t part_cap, double* S, bool f32,
                  const float* Yc, bool b3) {
  launch_cross(s, t, d, traj, Ma, ny, Y, Y, d.p(), muY, part, part_cap, S, 1.0, f32, Yc, b3);
}

}  // namespace oic
