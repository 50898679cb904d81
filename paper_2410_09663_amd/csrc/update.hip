// Ensemble analysis over the whole stored trajectory, Eq. (14b) with Eq. (15c):
//   Xcal^i <- Xcal^i + K (Ybar_t - Ybar^i)   for every member i and every slice k..t,
// which is the lag update that turns the forward pass into a smoother (Eq. (7)).
// As a matrix product: (rows x p) times (p x N*m), added in place.  The innovation
// has mean Ybar_t - mean(Ybar^i), so the updated members' mean moves by K times that
// (Eq. (14a)); the means are recomputed once at the end of the solve.
#include "oic_internal.h"

namespace oic {
namespace {

typedef float f32x4u __attribute__((ext_vector_type(4)));

constexpr int UC = 64;  // columns per tile (4 N-blocks of 16)
constexpr int PB = 80;  // observation rows per LDS stage
constexpr int kUpdWavesRows = 8;  // waves (16 rows each) of the persistent update's row tiles
constexpr int kUpdWaves = 8;      // waves of the general update's row tiles

// traj[a][c] += sum_b K[a][b] (Ybar[b][c mod m] - Y[b][c]),  Ybar = [X^ref_t; 0],
// on the FP32 matrix cores (v_mfma_f32_16x16x4_f32).  Wave w owns trajectory rows
// 16w..16w+15 of the tile and all 64 columns.  The gain tile, the innovation tile and
// the lane's own 16 trajectory values are all requested before the first LDS store.
// Lane layout: A[i][k] from lane i + 16k, B[k][j] from lane j + 16k, element r of
// lane j + 16g holds D[4g + r][j].
template <int WR>  // waves along the rows: tiles of 16 WR rows x 64 columns
__global__ __launch_bounds__(64 * WR) void k_update_mfma(Dims d, float* __restrict__ traj, int Ma,
                                                     const float* __restrict__ K,
                                                     const float* __restrict__ Y,
                                                     const float* __restrict__ xref) {
  constexpr int NT = 64 * WR, TR_ = 16 * WR;
  __shared__ float sK[TR_][PB + 1];
  __shared__ float sE[PB][UC + 1];
  const int NM = (int)d.NM();
  const int m = d.m, n = d.n, p = d.p();
  const int r0 = blockIdx.y * TR_;
  const int c0 = blockIdx.x * UC;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // the lane's trajectory values (read-modify-write), fetched first
  float old[4][4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = r0 + w * 16 + 4 * lk + r, c = c0 + nb * 16 + li;
      old[nb][r] = (a < Ma && c < NM) ? traj[(size_t)a * NM + c] : 0.f;
    }
  f32x4u acc[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4u{0.f, 0.f, 0.f, 0.f};
  for (int b0 = 0; b0 < p; b0 += PB) {
    constexpr int KS = TR_ * PB / NT;  // 20 gain values per thread
    constexpr int ES = PB * UC / NT;   // 20 innovation values per thread (10 with 8 waves)
    float kv[KS], ev[ES];
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      const int e = tid + NT * u;
      const int rl = e / PB, bl = e % PB;
      const int a = r0 + rl, b = b0 + bl;
      kv[u] = (a < Ma && b < p) ? K[(size_t)a * p + b] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < ES; ++u) {
      const int e = tid + NT * u;
      const int bl = e / UC, cl = e % UC;
      const int b = b0 + bl, c = c0 + cl;
      float v = 0.f;
      if (b < p && c < NM) {
        const float ybar = b < n ? xref[(size_t)b * m + c % m] : 0.f;
        v = ybar - Y[(size_t)b * NM + c];
      }
      ev[u] = v;
    }
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      const int e = tid + NT * u;
      sK[e / PB][e % PB] = kv[u];
    }
#pragma unroll
    for (int u = 0; u < ES; ++u) {
      const int e = tid + NT * u;
      sE[e / UC][e % UC] = ev[u];
    }
    __syncthreads();
    const int kmax = min(PB, p - b0);
    for (int ks = 0; ks < kmax; ks += 4) {
      const float av = sK[w * 16 + li][ks + lk];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, sE[ks + lk][nb * 16 + li], acc[nb], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int nb = 0; nb < 4; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = r0 + w * 16 + 4 * lk + r, c = c0 + nb * 16 + li;
      if (a < Ma && c < NM) traj[(size_t)a * NM + c] = old[nb][r] + acc[nb][r];
    }
}

// The same update for p <= PB as a persistent kernel over row tiles: block (x, y) owns
// columns 64x .. 64x + 63 and row tiles y, y + gridDim.y, ...  The innovation tile is
// formed in LDS once per block; the gain rows and the trajectory values of the next row
// tile are loaded into registers while the current tile is on the matrix cores.
template <int WR>  // waves along the rows: tiles of 16 WR rows
__global__ __launch_bounds__(64 * WR) void k_update_rows(Dims d, float* __restrict__ traj, int Ma,
                                                     const float* __restrict__ K,
                                                     const float* __restrict__ Y,
                                                     const float* __restrict__ xref, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(traj);
  OIC_GSH(K);
  OIC_GSH(Y);
  OIC_GSH(xref);
  constexpr int NT = 64 * WR, TR_ = 16 * WR;
  __shared__ float sK[TR_][PB + 1];
  __shared__ float sE[PB][UC + 1];
  const int NM = (int)d.NM();
  const int m = d.m, n = d.n, p = d.p();
  const int c0 = blockIdx.x * UC;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int row_tiles = (Ma + TR_ - 1) / TR_;
  constexpr int KS = TR_ * PB / NT;  // 20 gain values per thread
  constexpr int ES = PB * UC / NT;   // innovation values per thread
#pragma unroll
  for (int u = 0; u < ES; ++u) {
    const int e = tid + NT * u;
    const int b = e / UC, cl = e % UC;
    const int c = c0 + cl;
    float v = 0.f;
    if (b < p && c < NM) {
      const float ybar = b < n ? xref[(size_t)b * m + c % m] : 0.f;
      v = ybar - Y[(size_t)b * NM + c];
    }
    sE[b][cl] = v;
  }
  float kv[KS], old[4][4];
  auto load_rows = [&](int rt) {
    const int r0 = rt * TR_;
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      const int e = tid + NT * u;
      const int rl = e / PB, b = e % PB;
      const int a = r0 + rl;
      kv[u] = (a < Ma && b < p) ? K[(size_t)a * p + b] : 0.f;
    }
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = r0 + w * 16 + 4 * lk + r, c = c0 + nb * 16 + li;
        old[nb][r] = (a < Ma && c < NM) ? traj[(size_t)a * NM + c] : 0.f;
      }
  };
  int rt = blockIdx.y;
  if (rt < row_tiles) load_rows(rt);
  for (; rt < row_tiles; rt += gridDim.y) {
    const int r0 = rt * TR_;
    __syncthreads();  // the previous tile's products are done with sK (and sE is complete)
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      const int e = tid + NT * u;
      sK[e / PB][e % PB] = kv[u];
    }
    float cur[4][4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) cur[nb][r] = old[nb][r];
    __syncthreads();
    if (rt + (int)gridDim.y < row_tiles) load_rows(rt + gridDim.y);  // in flight meanwhile
    f32x4u acc[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4u{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < p; ks += 4) {
      const float av = sK[w * 16 + li][ks + lk];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, sE[ks + lk][nb * 16 + li], acc[nb], 0, 0, 0);
    }
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = r0 + w * 16 + 4 * lk + r, c = c0 + nb * 16 + li;
        if (a < Ma && c < NM) traj[(size_t)a * NM + c] = cur[nb][r] + acc[nb][r];
      }
  }
}

// The same update for larger p, persistent over 64-column strips: a workgroup forms the
// strip's innovation tile E[b][c] = Ybar_t[b][c mod m] - Y[b][c] once, transposed in LDS
// (E^T[c][b], pixel stride P16 + 4 floats), and its eight waves then walk 16-row blocks
// of the trajectory independently (no barrier until the next strip): a wave reads its
// block's gain rows straight into registers (they are shared by every strip, so they
// come from L2) and, per 16 observation rows b, lane (i, g) takes K[a0 + i][b0 + 4g + j]
// for the j-th of four MFMAs against E^T rows read as one 16-byte LDS load, the pairs
// (g, j) covering the 16 rows once.  The trajectory tile is read and written once per
// step.  P16 is p rounded up to the instantiated size (gain and innovation are zero
// beyond p).
constexpr int kStripWaves = 8;
template <int P16>
__global__ __launch_bounds__(64 * kStripWaves) void k_update_strip(Dims d, float* __restrict__ traj, int Ma,
                                                               const float* __restrict__ K,
                                                               const float* __restrict__ Y,
                                                               const float* __restrict__ xref) {
  constexpr int NT = 64 * kStripWaves;
  constexpr int EP = P16;  // a multiple of 32 floats: E^T[c][b] sits at c*EP + (b ^ 4 (c mod 8))
  constexpr int S = P16 / 16;
  static_assert(P16 % 32 == 0, "row stride a multiple of the 32 banks");
  __shared__ __attribute__((aligned(16))) float sE[UC * EP];
  const int NM = (int)d.NM();
  const int m = d.m, n = d.n, p = d.p();
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int strips = (NM + UC - 1) / UC;
  const int row_blocks = (Ma + 15) / 16;
  for (int strip = blockIdx.x; strip < strips; strip += gridDim.x) {
    const int c0 = strip * UC;
    __syncthreads();  // every wave is done with the previous strip's tile
    for (int e = tid; e < P16 * UC; e += NT) {
      const int b = e / UC, cl = e % UC;
      const int c = c0 + cl;
      float v = 0.f;
      if (b < p && c < NM) v = (b < n ? xref[(size_t)b * m + c % m] : 0.f) - Y[(size_t)b * NM + c];
      // the XOR moves whole 4-float groups, so a lane's 16-byte read stays in one piece,
      // and puts the eight 16-byte reads of one LDS phase (8 consecutive c) in 8 bank groups
      sE[cl * EP + (b ^ (4 * (cl & 7)))] = v;
    }
    __syncthreads();
    for (int rb = w; rb < row_blocks; rb += kStripWaves) {
      const int a0 = rb * 16;
      // this lane's gain values: row a0 + li, columns 16s + 4lk + j
      float kr[S][4];
      const int ka = a0 + li;
      if ((p & 3) == 0) {  // 16-byte aligned gain rows: one vector load per step
#pragma unroll
        for (int st = 0; st < S; ++st) {
          const int b = 16 * st + 4 * lk;
          f32x4u v = f32x4u{0.f, 0.f, 0.f, 0.f};
          if (ka < Ma && b < p) v = *(const f32x4u*)(K + (size_t)ka * p + b);
#pragma unroll
          for (int j = 0; j < 4; ++j) kr[st][j] = v[j];
        }
      } else {
#pragma unroll
        for (int st = 0; st < S; ++st)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int b = 16 * st + 4 * lk + j;
            kr[st][j] = (ka < Ma && b < p) ? K[(size_t)ka * p + b] : 0.f;
          }
      }
      float old[4][4];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = a0 + 4 * lk + r, c = c0 + 16 * nb + li;
          old[nb][r] = (a < Ma && c < NM) ? traj[(size_t)a * NM + c] : 0.f;
        }
      f32x4u acc[4];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4u{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int st = 0; st < S; ++st)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          const int cl = 16 * nb + li;
          const f32x4u e = *(const f32x4u*)(sE + cl * EP + ((16 * st + 4 * lk) ^ (4 * (cl & 7))));
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(kr[st][j], e[j], acc[nb], 0, 0, 0);
          // one step's LDS reads at a time beside its MFMAs (hoisting them all would
          // need more registers than the gain rows leave)
          if (nb == 3) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = a0 + 4 * lk + r, c = c0 + 16 * nb + li;
          if (a < Ma && c < NM) traj[(size_t)a * NM + c] = old[nb][r] + acc[nb][r];
        }
    }
  }
}

// Split of FP32 values into BF16 pairs v ~ hi + lo (hi = v rounded to nearest BF16, lo =
// the rounded remainder, which FP32 holds exactly): 16 significant bits per pair.
typedef __bf16 bf16x8u __attribute__((ext_vector_type(8)));
typedef float f32x2u __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2u __attribute__((ext_vector_type(2)));
typedef unsigned u32x4u __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void split2u(float v0, float v1, unsigned& hi, unsigned& lo) {
  hi = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2u{v0, v1}, bf16x2u));
  const float h0 = __uint_as_float(hi << 16), h1 = __uint_as_float(hi & 0xffff0000u);
  lo = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2u{v0 - h0, v1 - h1}, bf16x2u));
}

// The gain split once per horizon step for k_update_strip_b3: planes hi and lo of
// rows16 x P16 BF16 values (rows16 = Ma rounded up to 16), zeros past Ma and p.  One
// thread per 8 consecutive values of a row.
__global__ void k_split_gain(const float* __restrict__ K, int Ma, int p, int rows16, int P16,
                             __bf16* __restrict__ Khl, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(K);
  OIC_GSH(Khl);
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int groups = P16 / 8;
  if (e >= (long long)rows16 * groups) return;
  const int a = (int)(e / groups), b = (int)(e % groups) * 8;
  float v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = (a < Ma && b + j < p) ? K[(size_t)a * p + b + j] : 0.f;
  unsigned h[4], lo[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) split2u(v[2 * q], v[2 * q + 1], h[q], lo[q]);
  *(u32x4u*)(Khl + (size_t)a * P16 + b) = u32x4u{h[0], h[1], h[2], h[3]};
  *(u32x4u*)(Khl + (size_t)rows16 * P16 + (size_t)a * P16 + b) = u32x4u{lo[0], lo[1], lo[2], lo[3]};
}

// k_update_strip for the BF16 and FP8 modes: the products K E as three BF16 matrix-core
// products of split operands (v_mfma_f32_16x16x32_bf16: hi hi + hi lo + lo hi, relative
// error about 2^-16 per product, FP32 accumulation), at a sixth of the FP32 matrix-core
// cycles.  The strip's innovation tile is split once into two BF16 planes E^T[c][b] (hi,
// lo; row stride P16 + 8 so that the 16-byte reads of 16 consecutive columns fall in
// distinct bank groups); a wave splits its block's gain rows in registers, lane (i, g)
// taking K[a0 + i][32 s + 8 g .. + 7] for K step s against the 16-byte reads of the same
// eight rows b of E^T.  Trajectory tile read once, written once, as in k_update_strip.
// Khl: the gain already split (k_split_gain: planes hi and lo, rows padded to whole 16-row
// blocks and P16 columns, zeros past Ma and p), or null to split each block's rows here.
template <int P16>
__global__ __launch_bounds__(64 * kStripWaves) void k_update_strip_b3(Dims d, float* __restrict__ traj, int Ma,
                                                                  const float* __restrict__ K,
                                                                  const __bf16* __restrict__ Khl,
                                                                  const float* __restrict__ Y,
                                                                  const float* __restrict__ xref, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(traj);
  OIC_GSH(K);
  OIC_GSH(Khl);
  OIC_GSH(Y);
  OIC_GSH(xref);
  constexpr int NT = 64 * kStripWaves;
  constexpr int EP = P16 + 8;  // BF16 elements per column of a plane
  constexpr int S = P16 / 32;
  static_assert(P16 % 32 == 0, "32-row K steps");
  __shared__ __attribute__((aligned(16))) __bf16 sE[2][UC * EP];  // [hi, lo]
  const int NM = (int)d.NM();
  const int m = d.m, n = d.n, p = d.p();
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int strips = (NM + UC - 1) / UC;
  const int row_blocks = (Ma + 15) / 16;
  for (int strip = blockIdx.x; strip < strips; strip += gridDim.x) {
    const int c0 = strip * UC;
    __syncthreads();  // every wave is done with the previous strip's tile
    for (int e = tid; e < (P16 / 2) * UC; e += NT) {
      const int b = 2 * (e / UC), cl = e % UC;
      const int c = c0 + cl;
      float v[2] = {0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 2; ++k)
        if (b + k < p && c < NM)
          v[k] = (b + k < n ? xref[(size_t)(b + k) * m + c % m] : 0.f) - Y[(size_t)(b + k) * NM + c];
      unsigned hi, lo;
      split2u(v[0], v[1], hi, lo);
      *(unsigned*)(sE[0] + cl * EP + b) = hi;
      *(unsigned*)(sE[1] + cl * EP + b) = lo;
    }
    __syncthreads();
    for (int rb = w; rb < row_blocks; rb += kStripWaves) {
      const int a0 = rb * 16;
      // this lane's gain values, split: row a0 + li, columns 32 s + 8 lk .. + 7
      bf16x8u kh[S], kl[S];
      const int ka = a0 + li;
      if (Khl) {
        const size_t plane = (size_t)row_blocks * 16 * P16;
#pragma unroll
        for (int st = 0; st < S; ++st) {
          kh[st] = *(const bf16x8u*)(Khl + (size_t)ka * P16 + 32 * st + 8 * lk);
          kl[st] = *(const bf16x8u*)(Khl + plane + (size_t)ka * P16 + 32 * st + 8 * lk);
        }
      } else {
#pragma unroll
      for (int st = 0; st < S; ++st) {
        float kv[8];
        const int b = 32 * st + 8 * lk;
        if ((p & 3) == 0) {  // 16-byte aligned gain rows
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            f32x4u v = f32x4u{0.f, 0.f, 0.f, 0.f};
            if (ka < Ma && b + 4 * h < p) v = *(const f32x4u*)(K + (size_t)ka * p + b + 4 * h);
#pragma unroll
            for (int j = 0; j < 4; ++j) kv[4 * h + j] = v[j];
          }
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) kv[j] = (ka < Ma && b + j < p) ? K[(size_t)ka * p + b + j] : 0.f;
        }
        unsigned h[4], lo[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) split2u(kv[2 * q], kv[2 * q + 1], h[q], lo[q]);
        kh[st] = __builtin_bit_cast(bf16x8u, u32x4u{h[0], h[1], h[2], h[3]});
        kl[st] = __builtin_bit_cast(bf16x8u, u32x4u{lo[0], lo[1], lo[2], lo[3]});
      }
      }
      float old[4][4];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = a0 + 4 * lk + r, c = c0 + 16 * nb + li;
          old[nb][r] = (a < Ma && c < NM) ? traj[(size_t)a * NM + c] : 0.f;
        }
      f32x4u acc[4];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4u{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int st = 0; st < S; ++st)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          const int off = (16 * nb + li) * EP + 32 * st + 8 * lk;
          const bf16x8u eh = *(const bf16x8u*)(sE[0] + off);
          const bf16x8u el = *(const bf16x8u*)(sE[1] + off);
          acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kl[st], eh, acc[nb], 0, 0, 0);
          acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kh[st], el, acc[nb], 0, 0, 0);
          acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kh[st], eh, acc[nb], 0, 0, 0);
          // one step's LDS reads at a time beside its MFMAs
          if (nb == 3) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = a0 + 4 * lk + r, c = c0 + 16 * nb + li;
          if (a < Ma && c < NM) traj[(size_t)a * NM + c] = old[nb][r] + acc[nb][r];
        }
    }
  }
}

// Smoothed means of every slice -> U_out (H+1, l, m), X_out (H+1, n, m) and U_hat_k.
__global__ void k_extract(Dims d, const float* __restrict__ mu, float* __restrict__ Uout,
                          float* __restrict__ Xout, float* __restrict__ Uprev, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(mu);
  OIC_GSH(Uout);
  OIC_GSH(Xout);
  OIC_GSH(Uprev);
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
                   const float* Y, const float* xref_t, bool b3, void* scratch, size_t scratch_bytes) {
  const unsigned col_tiles = (unsigned)((d.NM() + UC - 1) / UC);
  if (d.p() <= PB) {
    constexpr int WR = kUpdWavesRows;
    const unsigned row_tiles = (unsigned)((Ma + 16 * WR - 1) / (16 * WR));
    // about two workgroups per CU (the register budget allows two) on 256 CUs
    const unsigned want = (512 + col_tiles - 1) / col_tiles;
    const unsigned groups = row_tiles < want ? row_tiles : want;
    OIC_GLAUNCH(t, KC_UPDATE, s, k_update_rows<WR>, dim3(col_tiles, groups), dim3(64 * WR), 0, d, traj, Ma, K, Y,
               xref_t);
    return;
  }
  // strips: one workgroup per CU (the transposed innovation tile fills most of its LDS)
  const unsigned strips = col_tiles < 256 ? col_tiles : 256;
#define OIC_STRIP_CASE(P16V)                                                                            \
  if (d.p() <= P16V) {                                                                                  \
    if constexpr (P16V <= 448) { /* beyond, the split gain rows would not fit the registers */     \
      if (b3) {                                                                                         \
        const int rows16 = (Ma + 15) / 16 * 16;                                                         \
        __bf16* khl = nullptr;                                                                          \
        if (scratch && (size_t)2 * rows16 * P16V * 2 <= scratch_bytes) {                                \
          khl = reinterpret_cast<__bf16*>(scratch);                                                     \
          const long long items = (long long)rows16 * (P16V / 8);                                      \
          OIC_GLAUNCH(t, KC_UPDATE, s, k_split_gain, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, K, Ma, \
                     d.p(), rows16, P16V, khl);                                                         \
        }                                                                                               \
        OIC_GLAUNCH(t, KC_UPDATE, s, k_update_strip_b3<P16V>, dim3(strips), dim3(64 * kStripWaves), 0, d, \
                   traj, Ma, K, khl, Y, xref_t);                                                        \
        return;                                                                                         \
      }                                                                                                 \
    }                                                                                                   \
    OIC_LAUNCH(t, KC_UPDATE, s, k_update_strip<P16V>, dim3(strips), dim3(64 * kStripWaves), 0, d, traj, Ma, K, \
               Y, xref_t);                                                                              \
    return;                                                                                             \
  }
  OIC_STRIP_CASE(128)
  OIC_STRIP_CASE(192)
  OIC_STRIP_CASE(256)
  OIC_STRIP_CASE(320)
  OIC_STRIP_CASE(384)
  OIC_STRIP_CASE(448)
  OIC_STRIP_CASE(512)
#undef OIC_STRIP_CASE
  constexpr int WR = kUpdWaves;
  const unsigned tall_tiles = (unsigned)((Ma + 16 * WR - 1) / (16 * WR));
  OIC_LAUNCH(t, KC_UPDATE, s, k_update_mfma<WR>, dim3(col_tiles, tall_tiles), dim3(64 * WR), 0, d, traj, Ma, K,
             Y, xref_t);
}

void launch_extract(hipStream_t s, Timer& t, const Dims& d, const float* mu_traj, float* Uout,
                    float* Xout, float* Uprev) {
  const long long total = (long long)(d.H + 1) * d.rr() * d.m;
  OIC_GLAUNCH(t, KC_EXTRACT, s, k_extract, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, d,
             mu_traj, Uout, Xout, Uprev);
}

}  // namespace oic
