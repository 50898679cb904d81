// Gain of the matrix-normal Kalman update, Eq. (10a) / Eq. (14b):
//   K = Sigma^{XY} (Sigma^Y)^{-1},
// in FP64.  The matrix inverted is p x p with p = n + l (the rows of the virtual
// observation).  For p <= 90 one workgroup factors Sigma^Y = L L^T (Cholesky) in LDS,
// inverts L and forms (Sigma^Y)^{-1} = L^{-T} L^{-1}; a second, wide kernel
// multiplies Sigma^{XY} by it.  Larger p use a blocked factorisation spread over the
// chip and two blocked triangular solves for the gain.
#include <algorithm>

#include "oic_internal.h"

namespace oic {
namespace {

constexpr int kCholThreads = 512;                  // 8 waves
constexpr int kLdsMaxP = 90;                       // two p8 x (p8+1) FP64 arrays (p8 <= 96) in the 160 KiB LDS
constexpr int NBK = 8;                             // panel width
constexpr int kMaxPanelsLds = (kLdsMaxP + NBK - 1) / NBK;  // 12

typedef double f64x4 __attribute__((ext_vector_type(4)));

// 1/sqrt(d) for d > 0: the hardware estimate refined by two Newton-Raphson steps,
// y <- y + y (1 - d y^2) / 2, each of which doubles the number of correct bits.
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-d * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  union {
    double d;
    int i[2];
  } u;
  u.d = v;
  u.i[0] = __builtin_amdgcn_readlane(u.i[0], lane);
  u.i[1] = __builtin_amdgcn_readlane(u.i[1], lane);
  return u.d;
}

// store(e, load(e)) for e = 0 .. count - 1 across the NT threads of a block, sixteen
// loads per thread in flight before their stores (global -> LDS staging without one
// memory latency per element).
template <int NT, typename Load, typename Store>
__device__ __forceinline__ void staged_copy(int count, Load load, Store store) {
  for (int base = 0; base < count; base += NT * 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = base + (int)threadIdx.x + NT * u;
      v[u] = e < count ? load(e) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = base + (int)threadIdx.x + NT * u;
      if (e < count) store(e, v[u]);
    }
  }
}

// D(16x16 tile at rows i0, cols j0 of M, leading dimension ld) += sum_k Aop[i][k] Bop[k][j]
// over k = 0..K-1 on the FP64 matrix cores, where the operands are read through the
// functors a(i, k) and b(k, j).  Reads are clamped into range and never skipped (a load
// under a branch costs a full LDS round trip): outside rows/cols the tile holds values
// that are never stored, since each output element depends only on its own row of A,
// column of B and accumulator; only the k >= K terms must be zeroed.  Lane layout (16x16x4 f64):
// A[i][k] from lane i + 16g (k = 4s + g), B[k][j] from lane j + 16g, element r of lane
// j + 16g holds D[g + 4r][j].
template <typename FA, typename FB>
__device__ __forceinline__ void mfma_tile_update(double* M, int ld, int rows, int cols, int i0, int j0,
                                                 int K, FA a, FB b, double sign) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  f64x4 acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + lk + 4 * r, j = j0 + li;
    acc[r] = M[min(i, rows - 1) * ld + min(j, cols - 1)];
  }
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int k = k0 + lk;
    const int kc = min(k, K - 1);  // clamped operand reads, zeroed past K
    const double a_ = a(i0 + li, kc), b_ = b(kc, j0 + li);
    const double av = (k < K) ? a_ : 0.0;
    const double bv = (k < K) ? sign * b_ : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + lk + 4 * r, j = j0 + li;
    if (i < rows && j < cols) M[i * ld + j] = acc[r];
  }
}

// Factor, invert and square the p x p SPD matrix in A (row-major, leading dimension
// ld = p + 1; LDS or global), with W (same shape and memory kind) as workspace; writes
// (Sigma^Y)^{-1} to Sinv (p x p) and sets *flag when a pivot is not positive and finite.
//
// Blocked right-looking Cholesky with 8-wide panels.  Per panel: wave 0 factors the
// 8 x 8 diagonal block with one row per lane (pivots broadcast by readlane) and also
// forms its inverse; the rows below become A21 L11^{-T} (eight independent dot
// products per row); the trailing lower triangle takes the rank-8 update on the FP64
// matrix cores.  W = L^{-1} follows by panels of rows (L11^{-1} times the panel, then
// a rank-8 update of the rows below, on the matrix cores), and (Sigma^Y)^{-1} = W^T W
// is one more matrix-core product.  The odd leading dimension spreads the rows read by
// the 16 lanes of an operand fragment over distinct LDS banks.
template <int MAXPAN, bool SQUARE, bool PAD8 = false>
__device__ __forceinline__ bool chol_inverse(int p, double* A, double* W, double* __restrict__ Sinv, int pout,
                                             int* __restrict__ flag) {
  const int ld = p + 1;
  __shared__ int bad;
  __shared__ double sLinv[MAXPAN][NBK][NBK];  // inverse of every diagonal block
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  constexpr int NW = kCholThreads / 64;
  const int npan = (p + NBK - 1) / NBK;
  if (tid == 0) bad = 0;
  // W = L^{-1} is built alongside the factor: it starts as the identity and takes, per
  // panel, the same two steps as the rows below (L11^{-1} times the panel rows, then a
  // rank-8 update of the rows below), in the same phases as the factorisation.
  for (int e = tid; e < p * ld; e += kCholThreads) {
    const int i = e / ld, j = e - i * ld;
    W[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  // Factor the pb-th 8 x 8 diagonal block (wave 0 only; every update it receives is done).
  auto factor_diag = [&](int pb) {
    const int kb = pb * NBK;
    const int nb = PAD8 ? NBK : min(NBK, p - kb);
    // Every lane factors the whole 8 x 8 diagonal block in its own registers (no
    // cross-lane traffic; identity rows pad a short last panel), keeping the
    // reciprocal square roots for the block inverse.
    double a[NBK][NBK], rs[NBK];
#pragma unroll
    for (int r = 0; r < NBK; ++r)
#pragma unroll
      for (int c = 0; c < NBK; ++c)
        a[r][c] = c > r ? 0.0
                        : ((r < nb) ? A[min(kb + r, p - 1) * ld + min(kb + c, p - 1)]  // clamped: no branch
                                    : (r == c ? 1.0 : 0.0));
    bool ok = true;
#pragma unroll
    for (int k = 0; k < NBK; ++k) {
      const double d = a[k][k];
      if (!(d > 0.0 && isfinite(d))) ok = false;
      const double rk = rsqrt_nr(d);  // computed unconditionally, selected below (no branch)
      rs[k] = (d > 0.0 && isfinite(d)) ? rk : 1.0;
      a[k][k] = d * rs[k];
#pragma unroll
      for (int r = k + 1; r < NBK; ++r) a[r][k] *= rs[k];
#pragma unroll
      for (int c = k + 1; c < NBK; ++c)
#pragma unroll
        for (int r = c; r < NBK; ++r) a[r][c] -= a[r][k] * a[c][k];
    }
    // lane c < 8 forms column c of L11^{-1}: x_r = (delta_rc - sum_{q<r} L_rq x_q) / L_rr
    if (lane < NBK) {
      double x[NBK];
#pragma unroll
      for (int r = 0; r < NBK; ++r) {
        double v = (r == lane) ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < r; ++q) v -= a[r][q] * x[q];
        x[r] = v * rs[r];
      }
#pragma unroll
      for (int r = 0; r < NBK; ++r) sLinv[pb][r][lane] = (r >= lane) ? x[r] : 0.0;
      if (lane < nb) {
#pragma unroll
        for (int c = 0; c < NBK; ++c) {
          double v = 0.0;
#pragma unroll
          for (int r = 0; r < NBK; ++r) v = (r == lane) ? a[r][c] : v;  // row `lane`, static indices
          // zeros above the diagonal (that triangle is never read); a short last panel
          // stops at column p - 1
          if (PAD8 || c < nb) A[(kb + lane) * ld + kb + c] = v;
        }
      }
    }
    if (lane == 0 && !ok) bad = 1;
  };
  if (wave == 0) factor_diag(0);
  __syncthreads();
  for (int pb = 0; pb < npan; ++pb) {
    const int kb = pb * NBK;
    const int nb = PAD8 ? NBK : min(NBK, p - kb);
    const int r0 = kb + nb, rem = p - r0;
    // rows below: L21 = A21 L11^{-T}
    for (int i = r0 + tid; i < p; i += kCholThreads) {
      double a21[NBK], l21[NBK];
#pragma unroll
      for (int q = 0; q < NBK; ++q) a21[q] = A[i * ld + kb + q];
#pragma unroll
      for (int c = 0; c < NBK; ++c) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q <= c; ++q) v = fma(a21[q], sLinv[pb][c][q], v);
        l21[c] = v;
      }
#pragma unroll
      for (int c = 0; c < NBK; ++c) A[i * ld + kb + c] = l21[c];
    }
    const int cols = kb + nb;
    // W[kb:kb+nb, j] = L11^{-1} B[kb:kb+nb, j] for every column j < cols
    for (int j = tid; j < cols; j += kCholThreads) {
      double bcol[NBK], w[NBK];
#pragma unroll
      for (int q = 0; q < NBK; ++q) bcol[q] = (q < nb) ? W[(kb + q) * ld + j] : 0.0;
#pragma unroll
      for (int r = 0; r < NBK; ++r) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q <= r; ++q) v = fma(sLinv[pb][r][q], bcol[q], v);
        w[r] = v;
      }
#pragma unroll
      for (int r = 0; r < NBK; ++r)
        if (r < nb) W[(kb + r) * ld + j] = w[r];
    }
    __syncthreads();
    // trailing lower triangle: A22 -= L21 L21^T, and W rows below: B[i][j] -= L21[i] W[kb:, j]
    // (i >= cols, j < cols), as 16 x 16 tiles on the matrix cores.  Look-ahead: wave 0
    // takes the tile holding the next diagonal block first and then factors that block,
    // while the other waves update the remaining tiles.
    if (rem > 0) {
      const int nt = (rem + 15) / 16;
      const int ntri = nt * (nt + 1) / 2;
      const int ntj = (cols + 15) / 16;
      auto a22_tile = [&](int t) {
        int ti = 0;
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        const int tj = t - ti * (ti + 1) / 2;
        mfma_tile_update(
            A, ld, p, p, r0 + 16 * ti, r0 + 16 * tj, NBK,
            [&](int i, int k) { return A[min(i, p - 1) * ld + kb + k]; },
            [&](int k, int j) { return A[min(j, p - 1) * ld + kb + k]; }, -1.0);
      };
      if (wave == 0) {
        a22_tile(0);
        factor_diag(pb + 1);
      } else {
        for (int t = wave; t < ntri + nt * ntj; t += NW - 1) {
          if (t < ntri) {
            a22_tile(t);
          } else {
            const int u = t - ntri;
            const int ti = u / ntj, tj = u - ti * ntj;
            mfma_tile_update(
                W, ld, p, cols, cols + 16 * ti, 16 * tj, nb,
                [&](int i, int k) { return A[min(i, p - 1) * ld + kb + k]; },
                [&](int k, int j) { return W[(kb + k) * ld + min(j, cols - 1)]; }, -1.0);
          }
        }
      }
    }
    __syncthreads();
  }
  if (bad) {
    if (tid == 0) *flag = 1;
    return false;
  }
  if (!SQUARE) return true;
  // (Sigma^Y)^{-1} = W^T W: lower 16 x 16 tiles, mirrored.
  {
    const int nt = (p + 15) / 16;
    const int li = lane & 15, lk = lane >> 4;
    for (int t = wave; t < nt * (nt + 1) / 2; t += NW) {
      int ti = 0;
      while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
      const int tj = t - ti * (ti + 1) / 2;
      const int i0 = 16 * ti, j0 = 16 * tj;
      f64x4 acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
      const int kmin = i0;  // W is lower triangular: rows k < i0 contribute nothing
      for (int k0 = kmin; k0 < p; k0 += 8) {
        const int k = k0 + lk, k2 = k + 4;
        const double av = (k < p && i0 + li < p) ? W[k * ld + i0 + li] : 0.0;
        const double bv = (k < p && j0 + li < p) ? W[k * ld + j0 + li] : 0.0;
        const double av2 = (k2 < p && i0 + li < p) ? W[k2 * ld + i0 + li] : 0.0;
        const double bv2 = (k2 < p && j0 + li < p) ? W[k2 * ld + j0 + li] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av2, bv2, acc2, 0, 0, 0);
      }
      acc += acc2;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + lk + 4 * r, j = j0 + li;
        if (i < pout && j < pout) {
          Sinv[i * pout + j] = acc[r];
          Sinv[j * pout + i] = acc[r];
        }
      }
    }
  }
  return true;
}

__global__ __launch_bounds__(kCholThreads) void k_chol_inv_lds(int p, const double* __restrict__ Syy,
                                                               double* __restrict__ Sinv,
                                                               int* __restrict__ flag, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(Syy);
  OIC_GSH(Sinv);
  OIC_GSH(flag);
  // Sigma^Y padded to p8 = p rounded up to a multiple of the panel width, with an identity
  // block: the factor of the padded matrix is diag(L, I), and every panel is full (no
  // branches on a short last panel).
  extern __shared__ double lds[];
  const int p8 = (p + NBK - 1) / NBK * NBK;
  {
    // every load of Sigma^Y in flight at once (p8 * p8 <= kLoadSlots * kCholThreads), then into LDS
    constexpr int kMaxP8 = (kLdsMaxP + NBK - 1) / NBK * NBK;
    constexpr int kLoadSlots = (kMaxP8 * kMaxP8 + kCholThreads - 1) / kCholThreads;
    double v[kLoadSlots];
#pragma unroll
    for (int u = 0; u < kLoadSlots; ++u) {
      const int idx = threadIdx.x + kCholThreads * u;
      const int r = idx / p8, c = idx - r * p8;
      v[u] = (r < p && c < p) ? Syy[r * p + c] : (r == c ? 1.0 : 0.0);
    }
#pragma unroll
    for (int u = 0; u < kLoadSlots; ++u) {
      const int idx = threadIdx.x + kCholThreads * u;
      const int r = idx / p8, c = idx - r * p8;
      if (idx < p8 * p8) lds[r * (p8 + 1) + c] = v[u];
    }
  }
  __syncthreads();
  chol_inverse<kMaxPanelsLds, true, true>(p8, lds, lds + p8 * (p8 + 1), Sinv, p, flag);
}

// K[a][b] = sum_c Sxy[a][c] Sinv[c][b], FP64, rounded to FP32 (any p).  Block (64, 4).
__global__ __launch_bounds__(256) void k_gain_product(int p, int Ma, const double* __restrict__ Sxy,
                                                      const double* __restrict__ Sinv,
                                                      float* __restrict__ K,
                                                      const int* __restrict__ flag, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(Sxy);
  OIC_GSH(Sinv);
  OIC_GSH(K);
  OIC_GSH(flag);
  if (*flag) return;
  const int b = blockIdx.y * 64 + threadIdx.x;
  const int a = blockIdx.x * 4 + threadIdx.y;
  if (a >= Ma || b >= p) return;
  const double* row = Sxy + (size_t)a * p;
  double s = 0.0;
  for (int c = 0; c < p; ++c) s = fma(row[c], Sinv[(size_t)c * p + b], s);
  K[(size_t)a * p + b] = (float)s;
}



// K = Sxy Sinv on the FP64 matrix cores.  A block of 4 waves owns 64 gain rows; wave w
// computes rows 16w..16w+15 against every 16-column block of Sinv (staged in LDS,
// zero-padded to a multiple of 16).  Lane layout as in the statistics kernel.
template <int NB>
__global__ __launch_bounds__(256) void k_gain_mfma(int p, int Ma, const double* __restrict__ Sxy,
                                                   const double* __restrict__ Sinv,
                                                   float* __restrict__ K,
                                                   const int* __restrict__ flag, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(Sxy);
  OIC_GSH(Sinv);
  OIC_GSH(K);
  OIC_GSH(flag);
  constexpr int P16 = NB * 16;
  __shared__ double sS[P16 * (P16 + 1)];
  if (*flag) return;
  {
    // every load of the inverse in flight at once, then into LDS
    constexpr int SV = P16 * P16 / 256;
    double v[SV];
#pragma unroll
    for (int u = 0; u < SV; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int r = e / P16, c = e % P16;
      v[u] = (r < p && c < p) ? Sinv[r * p + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < SV; ++u) {
      const int e = threadIdx.x + 256 * u;
      sS[(e / P16) * (P16 + 1) + e % P16] = v[u];
    }
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


// ---- Blocked factorisation for p > kLdsMaxP ----
//
// Right-looking blocked Cholesky with kPB-wide panels, one kernel per phase so that
// every phase spreads over the whole chip: per panel, (1) one workgroup factors the
// diagonal block in LDS and forms its inverse (the code above, without the final
// product), (2) the rows below become L21 = A21 L11^{-T}, (3) the trailing lower
// triangle takes A22 -= L21 L21^T.  The factor overwrites the lower triangle of
// Sigma^Y in place; the inverses of the diagonal blocks go to a side buffer.  The gain
// then follows from two blocked triangular solves per row of Sigma^{XY} (no explicit
// inverse): z L^T = s, then k L = z, i.e. k = s L^{-T} L^{-1} = s (Sigma^Y)^{-1}.
constexpr int kPB = 64;
constexpr int kPBP = kPB + 1;  // padded LDS leading dimension

__global__ __launch_bounds__(kCholThreads) void k_potrf_diag(int p, double* __restrict__ A, int kb,
                                                             double* __restrict__ Linv,
                                                             int* __restrict__ flag, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(A);
  OIC_GSH(Linv);
  OIC_GSH(flag);
  extern __shared__ double lds[];  // 2 x kPB x (kPB + 1)
  if (*flag) return;  // an earlier step failed; the solve reports it
  const int nb = min(kPB, p - kb);
  const int ld = nb + 1;
  double* sA = lds;
  double* sW = lds + nb * ld;
  staged_copy<kCholThreads>(
      nb * nb, [&](int e) { return A[(size_t)(kb + e / nb) * p + kb + e % nb]; },
      [&](int e, double v) { sA[(e / nb) * ld + e % nb] = v; });
  __syncthreads();
  if (!chol_inverse<kPB / NBK, false>(nb, sA, sW, nullptr, 0, flag)) return;
  __syncthreads();
  double* out = Linv + (size_t)(kb / kPB) * kPB * kPB;
  for (int e = threadIdx.x; e < kPB * kPB; e += kCholThreads) {
    const int r = e / kPB, c = e - r * kPB;
    const bool in = r < nb && c <= r;
    out[e] = in ? sW[r * ld + c] : 0.0;
    if (r < nb && c < nb) A[(size_t)(kb + r) * p + kb + c] = in ? sA[r * ld + c] : 0.0;
  }
}

// Rows r0 + 64*blockIdx.x .. +63 (r0 = kb + nb): L21 = A21 L11^{-T}.  Wave w owns 16
// rows against the panel's four 16-column blocks.
__global__ __launch_bounds__(256) void k_potrf_trsm(int p, double* __restrict__ A, int kb,
                                                    const double* __restrict__ Linv,
                                                    const int* __restrict__ flag, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(A);
  OIC_GSH(Linv);
  OIC_GSH(flag);
  __shared__ double sL[kPB * kPBP];
  __shared__ double sR[64 * kPBP];
  if (*flag) return;
  const int nb = min(kPB, p - kb);
  const int i0 = kb + nb + blockIdx.x * 64;
  const double* Li = Linv + (size_t)(kb / kPB) * kPB * kPB;
  staged_copy<256>(
      kPB * kPB, [&](int e) { return Li[e]; }, [&](int e, double v) { sL[(e / kPB) * kPBP + e % kPB] = v; });
  staged_copy<256>(
      kPB * kPB,
      [&](int e) {
        const int r = e / kPB, c = e - r * kPB;
        return (i0 + r < p && c < nb) ? A[(size_t)(i0 + r) * p + kb + c] : 0.0;
      },
      [&](int e, double v) { sR[(e / kPB) * kPBP + e % kPB] = v; });
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  f64x4 acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k0 = 0; k0 < kPB; k0 += 4) {
    const double av = sR[(16 * w + li) * kPBP + k0 + lk];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)  // B[k][j] = L11^{-1}[j][k]
      acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, sL[(16 * cb + li) * kPBP + k0 + lk], acc[cb],
                                                     0, 0, 0);
  }
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = i0 + 16 * w + lk + 4 * r, col = 16 * cb + li;
      if (row < p && col < nb) A[(size_t)row * p + kb + col] = acc[cb][r];
    }
}

// Trailing update of the lower triangle: 64 x 64 tile (ti, tj), ti >= tj, of the
// rows/columns from r0 = kb + nb: A22 -= L21[ti] L21[tj]^T.
__global__ __launch_bounds__(256) void k_potrf_syrk(int p, double* __restrict__ A, int kb,
                                                    const int* __restrict__ flag, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(A);
  OIC_GSH(flag);
  __shared__ double sI[64 * kPBP];
  __shared__ double sJ[64 * kPBP];
  if (*flag) return;
  const int nb = min(kPB, p - kb);
  const int r0 = kb + nb;
  int ti = 0;
  const int t = blockIdx.x;
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  const int tj = t - ti * (ti + 1) / 2;
  const int i0 = r0 + 64 * ti, j0 = r0 + 64 * tj;
  staged_copy<256>(
      64 * kPB,
      [&](int e) {
        const int r = e / kPB, c = e - r * kPB;
        return (i0 + r < p && c < nb) ? A[(size_t)(i0 + r) * p + kb + c] : 0.0;
      },
      [&](int e, double v) { sI[(e / kPB) * kPBP + e % kPB] = v; });
  staged_copy<256>(
      64 * kPB,
      [&](int e) {
        const int r = e / kPB, c = e - r * kPB;
        return (j0 + r < p && c < nb) ? A[(size_t)(j0 + r) * p + kb + c] : 0.0;
      },
      [&](int e, double v) { sJ[(e / kPB) * kPBP + e % kPB] = v; });
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  f64x4 acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = i0 + 16 * w + lk + 4 * r, col = j0 + 16 * cb + li;
      acc[cb][r] = (row < p && col < p) ? A[(size_t)row * p + col] : 0.0;
    }
#pragma unroll 4
  for (int k0 = 0; k0 < kPB; k0 += 4) {
    const double av = sI[(16 * w + li) * kPBP + k0 + lk];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
      acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, -sJ[(16 * cb + li) * kPBP + k0 + lk], acc[cb],
                                                     0, 0, 0);
  }
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = i0 + 16 * w + lk + 4 * r, col = j0 + 16 * cb + li;
      if (row < p && col < p) A[(size_t)row * p + col] = acc[cb][r];
    }
}

// K rows a0 .. a0 + RB - 1 (a0 = RB*blockIdx.x) from the factor L (lower triangle of
// A) and the diagonal-block inverses: forward z_i = (s_i - sum_{k<i} z_k L_ik^T)
// L_ii^{-T}, then backward k_i = (z_i - sum_{j>i} k_j L_ji) L_ii^{-1}, panel by panel,
// in FP64 on the matrix cores; the RB x p row block stays in LDS throughout and each
// 64 x 64 block of L passes through LDS once per use.  Tiles: RB/16 row tiles x 4
// column tiles of the current panel, spread over the 4 waves.
template <int RB>
__global__ __launch_bounds__(256) void k_gain_trsm(int p, int Ma, const double* __restrict__ Sxy,
                                                   const double* __restrict__ A,
                                                   const double* __restrict__ Linv,
                                                   float* __restrict__ K, const int* __restrict__ flag, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(Sxy);
  OIC_GSH(A);
  OIC_GSH(Linv);
  OIC_GSH(K);
  OIC_GSH(flag);
  extern __shared__ double lds[];
  constexpr int RT = RB / 16;       // row tiles
  constexpr int TPW = RT * 4 / 4;   // tiles per wave
  if (*flag) return;
  const int npan = (p + kPB - 1) / kPB;
  const int PP = npan * kPB + 1;    // z leading dimension
  double* z = lds;                  // RB x PP
  double* tmp = z + RB * PP;        // RB x kPBP
  double* sL = tmp + RB * kPBP;     // kPB x kPBP
  const int a0 = blockIdx.x * RB;
  const int tid = threadIdx.x;
  staged_copy<256>(
      RB * npan * kPB,
      [&](int e) {
        const int r = e / (npan * kPB), c = e - r * (npan * kPB);
        return (a0 + r < Ma && c < p) ? Sxy[(size_t)(a0 + r) * p + c] : 0.0;
      },
      [&](int e, double v) { z[(e / (npan * kPB)) * PP + e % (npan * kPB)] = v; });
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // tile u of this wave: row tile rt = (w*TPW + u) / 4, column tile ct = (w*TPW + u) % 4
  auto stage_block = [&](int bi, int bj) {  // sL[r][c] = L[64 bi + r][64 bj + c]
    staged_copy<256>(
        kPB * kPB,
        [&](int e) {
          const int gr = bi * kPB + e / kPB, gc = bj * kPB + e % kPB;
          return (gr < p && gc < p) ? A[(size_t)gr * p + gc] : 0.0;
        },
        [&](int e, double v) { sL[(e / kPB) * kPBP + e % kPB] = v; });
  };
  auto stage_inv = [&](int bi) {
    const double* Li = Linv + (size_t)bi * kPB * kPB;
    staged_copy<256>(
        kPB * kPB, [&](int e) { return Li[e]; }, [&](int e, double v) { sL[(e / kPB) * kPBP + e % kPB] = v; });
  };
  for (int pass = 0; pass < 2; ++pass) {
    const bool fwd = pass == 0;
    for (int q = 0; q < npan; ++q) {
      const int i = fwd ? q : npan - 1 - q;
      f64x4 acc[TPW];
#pragma unroll
      for (int u = 0; u < TPW; ++u) {
        const int rt = (w * TPW + u) / 4, ct = (w * TPW + u) % 4;
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[u][r] = z[(16 * rt + lk + 4 * r) * PP + i * kPB + 16 * ct + li];
      }
      // the other panels' contributions: forward k < i uses L_ik^T, backward j > i uses L_ji
      const int kb0 = fwd ? 0 : i + 1, kb1 = fwd ? i : npan;
      for (int kbk = kb0; kbk < kb1; ++kbk) {
        __syncthreads();
        if (fwd)
          stage_block(i, kbk);
        else
          stage_block(kbk, i);
        __syncthreads();
#pragma unroll 4
        for (int k0 = 0; k0 < kPB; k0 += 4) {
#pragma unroll
          for (int u = 0; u < TPW; ++u) {
            const int rt = (w * TPW + u) / 4, ct = (w * TPW + u) % 4;
            const double av = z[(16 * rt + li) * PP + kbk * kPB + k0 + lk];
            // forward: B[k][j] = L_ik[j][k]; backward: B[k][j] = L_ji[k][j]
            const double bv = fwd ? sL[(16 * ct + li) * kPBP + k0 + lk] : sL[(k0 + lk) * kPBP + 16 * ct + li];
            acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, -bv, acc[u], 0, 0, 0);
          }
        }
      }
      __syncthreads();  // every wave is done with sL and with tmp of the previous panel
#pragma unroll
      for (int u = 0; u < TPW; ++u) {
        const int rt = (w * TPW + u) / 4, ct = (w * TPW + u) % 4;
#pragma unroll
        for (int r = 0; r < 4; ++r) tmp[(16 * rt + lk + 4 * r) * kPBP + 16 * ct + li] = acc[u][r];
      }
      stage_inv(i);
      __syncthreads();
#pragma unroll
      for (int u = 0; u < TPW; ++u) acc[u] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
      for (int k0 = 0; k0 < kPB; k0 += 4) {
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
          const int rt = (w * TPW + u) / 4, ct = (w * TPW + u) % 4;
          const double av = tmp[(16 * rt + li) * kPBP + k0 + lk];
          // forward: times L_ii^{-T} (B[k][j] = Linv[j][k]); backward: times L_ii^{-1}
          const double bv = fwd ? sL[(16 * ct + li) * kPBP + k0 + lk] : sL[(k0 + lk) * kPBP + 16 * ct + li];
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[u], 0, 0, 0);
        }
      }
#pragma unroll
      for (int u = 0; u < TPW; ++u) {
        const int rt = (w * TPW + u) / 4, ct = (w * TPW + u) % 4;
#pragma unroll
        for (int r = 0; r < 4; ++r) z[(16 * rt + lk + 4 * r) * PP + i * kPB + 16 * ct + li] = acc[u][r];
      }
      __syncthreads();  // z_i is complete before any later panel reads it
    }
  }
  for (int e = tid; e < RB * p; e += 256) {
    const int r = e / p, c = e - r * p;
    if (a0 + r < Ma) K[(size_t)(a0 + r) * p + c] = (float)z[r * PP + c];
  }
}

size_t gain_trsm_lds(int p, int RB) {
  const int npan = (p + kPB - 1) / kPB;
  return sizeof(double) * ((size_t)RB * (npan * kPB + 1) + (size_t)RB * kPBP + (size_t)kPB * kPBP);
}

}  // namespace

void launch_chol(hipStream_t s, Timer& t, int p, double* Syy, double* Lwork, double* Sinv, int* flag) {
  if (p <= kLdsMaxP) {
    static const bool attr_set = [] {  // thread-safe one-time set-up
      constexpr int kMaxP8 = (kLdsMaxP + NBK - 1) / NBK * NBK;
      hipFuncSetAttribute((const void*)k_chol_inv_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                          2 * kMaxP8 * (kMaxP8 + 1) * (int)sizeof(double));
      return true;
    }();
    (void)attr_set;
    const int p8 = (p + NBK - 1) / NBK * NBK;  // padded order (identity block)
    OIC_GLAUNCH(t, KC_CHOL, s, k_chol_inv_lds, dim3(1), dim3(kCholThreads),
               2 * (size_t)p8 * (p8 + 1) * sizeof(double), p, Syy, Sinv, flag);
    return;
  }
  // blocked: Syy is factored in place, the diagonal-block inverses go to Lwork
  const size_t diag_lds = 2 * (size_t)kPB * kPBP * sizeof(double);
  static const bool diag_attr = [&] {
    hipFuncSetAttribute((const void*)k_potrf_diag, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)diag_lds);
    return true;
  }();
  (void)diag_attr;
  for (int kb = 0; kb < p; kb += kPB) {
    OIC_GLAUNCH(t, KC_CHOL, s, k_potrf_diag, dim3(1), dim3(kCholThreads), diag_lds, p, Syy, kb, Lwork,
               flag);
    const int rem = p - kb - std::min(kPB, p - kb);
    if (rem <= 0) break;
    const int nt = (rem + 63) / 64;
    OIC_GLAUNCH(t, KC_CHOL, s, k_potrf_trsm, dim3((unsigned)nt), dim3(256), 0, p, Syy, kb, Lwork, flag);
    OIC_GLAUNCH(t, KC_CHOL, s, k_potrf_syrk, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, p, Syy, kb,
               flag);
  }
}

bool chol_blocked(int p) { return p > kLdsMaxP; }

void launch_gain(hipStream_t s, Timer& t, int p, int Ma, const double* Sxy, const double* Sinv,
                 const double* L, const double* Linv, float* K, const int* flag) {
  if (p > kLdsMaxP) {
    // rows per block: 32 while the row block and its staging fit the LDS, else 16
    const bool big = gain_trsm_lds(p, 32) <= 160 * 1024;
    const int RB = big ? 32 : 16;
    const size_t bytes = gain_trsm_lds(p, RB);
    static const bool attr_set = [] {
      hipFuncSetAttribute((const void*)k_gain_trsm<32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          160 * 1024);
      hipFuncSetAttribute((const void*)k_gain_trsm<16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          160 * 1024);
      return true;
    }();
    (void)attr_set;
    const dim3 g((unsigned)((Ma + RB - 1) / RB));
    if (big)
      OIC_GLAUNCH(t, KC_GAIN, s, k_gain_trsm<32>, g, dim3(256), bytes, p, Ma, Sxy, L, Linv, K, flag);
    else
      OIC_GLAUNCH(t, KC_GAIN, s, k_gain_trsm<16>, g, dim3(256), bytes, p, Ma, Sxy, L, Linv, K, flag);
    return;
  }
  const int nbk = (p + 15) / 16;
  const dim3 g((unsigned)((Ma + 63) / 64));
  switch (nbk) {
#define OIC_GAIN_CASE(NBV) \
  case NBV: OIC_GLAUNCH(t, KC_GAIN, s, k_gain_mfma<NBV>, g, dim3(256), 0, p, Ma, Sxy, Sinv, K, flag); return;
    OIC_GAIN_CASE(1) OIC_GAIN_CASE(2) OIC_GAIN_CASE(3) OIC_GAIN_CASE(4)
    OIC_GAIN_CASE(5) OIC_GAIN_CASE(6)
#undef OIC_GAIN_CASE
    default:
      OIC_GLAUNCH(t, KC_GAIN, s, k_gain_product, dim3((unsigned)((Ma + 3) / 4), (unsigned)((p + 63) / 64)),
                 dim3(64, 4), 0, p, Ma, Sxy, Sinv, K, flag);
  }
}

}  // namespace oic
