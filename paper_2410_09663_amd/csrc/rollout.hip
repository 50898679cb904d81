// Ensemble rollout through the CNN surrogate, Eq. (1) / Eq. (15b):
// x0 = [X, B U] (two channels), then zero-padded 3x3 cross-correlation layers
// with the activation between them and none after the last.
//
// Activations are NHWC [member][row][col][channel].  The first kernel ("lift")
// builds the two input channels straight from the trajectory buffer; the last
// layer writes its single channel straight back into the trajectory (or any
// strided field), so no extra pass touches the next state.
#include "oic_internal.h"

namespace oic {
namespace {

__device__ __forceinline__ float activate(float v, int act) {
  if (act == OIC_ACT_TANH) return tanhf(v);
  return 0.5f * v * (1.0f + erff(v * 0.70710678118654752f));  // exact GELU
}

// BF16 storage: round to nearest even (activations are finite), and back by shifting.
typedef unsigned short bf16_t;
__device__ __forceinline__ bf16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(bf16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ void store_act(float* p, float v) { *p = v; }
__device__ __forceinline__ void store_act(bf16_t* p, float v) { *p = to_bf16(v); }

// x0[i][y][x] = (X^i[y][x], sum_a B[y][a] U^i[a][x]).
__global__ void k_lift(int N, int n, int m, int l, FieldRef X, FieldRef U,
                       const float* __restrict__ B, float* __restrict__ out) {
  const long long total = (long long)N * n * m;
  const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= total) return;
  const int x = (int)(pix % m);
  const long long r = pix / m;
  const int y = (int)(r % n);
  const int i = (int)(r / n);
  const float xv = X.base[i * X.si + y * X.sy + x];
  const float* Bq = B + (size_t)y * l;
  const float* Ui = U.base + i * U.si + x;
  float bu = 0.f;
  for (int a = 0; a < l; ++a) bu = fmaf(Bq[a], Ui[a * U.sy], bu);
  out[pix * 2 + 0] = xv;
  out[pix * 2 + 1] = bu;
}

// Direct FP32 3x3 convolution: one thread per output pixel and a block of
// CO_BLK output channels (blockIdx.y).  Weights [C_out][C_in][3][3].
template <int CO_BLK>
__global__ void k_conv_direct(int N, int n, int m, int cin, int cout,
                              const float* __restrict__ in, const float* __restrict__ w,
                              const float* __restrict__ bias, int act, float* __restrict__ out,
                              FieldOut fo) {
  const long long total = (long long)N * n * m;
  const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= total) return;
  const int co0 = blockIdx.y * CO_BLK;
  const int x = (int)(pix % m);
  const long long r = pix / m;
  const int y = (int)(r % n);
  const int i = (int)(r / n);
  float acc[CO_BLK];
#pragma unroll
  for (int o = 0; o < CO_BLK; ++o) acc[o] = (bias && co0 + o < cout) ? bias[co0 + o] : 0.f;
  for (int dy = 0; dy < 3; ++dy) {
    const int yy = y + dy - 1;
    if (yy < 0 || yy >= n) continue;
    for (int dx = 0; dx < 3; ++dx) {
      const int xx = x + dx - 1;
      if (xx < 0 || xx >= m) continue;
      const float* ip = in + (((size_t)i * n + yy) * m + xx) * cin;
      const int tap = dy * 3 + dx;
      for (int c = 0; c < cin; ++c) {
        const float v = ip[c];
#pragma unroll
        for (int o = 0; o < CO_BLK; ++o) {
          if (co0 + o < cout) acc[o] = fmaf(w[((size_t)(co0 + o) * cin + c) * 9 + tap], v, acc[o]);
        }
      }
    }
  }
  if (fo.base) {  // last layer: one channel, written to the strided field
    fo.base[i * fo.si + y * fo.sy + x] = acc[0];
    return;
  }
#pragma unroll
  for (int o = 0; o < CO_BLK; ++o)
    if (co0 + o < cout) out[pix * cout + co0 + o] = activate(acc[o], act);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Stage the HR x HC halo (rows y0-1.., columns x0-1..) of member i of an NHWC
// [N][n][m][CIN] tensor into s_in[(yy*HC + xx)*CP + c], zero outside the field.
// Every float4 load of a thread is issued before its first LDS store, so a tile
// costs one memory round trip instead of one per element.
template <int CIN, int HR, int HC, int CP, int NT>
__device__ __forceinline__ void stage_halo(const float* __restrict__ in, int i, int n, int m, int y0,
                                           int x0, float* s_in) {
  constexpr int Q = CIN / 4;
  constexpr int TOTAL = HR * HC * Q;
  constexpr int SLOTS = (TOTAL + NT - 1) / NT;
  f32x4 v[SLOTS];
#pragma unroll
  for (int u = 0; u < SLOTS; ++u) {
    const int e = threadIdx.x + u * NT;
    v[u] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (e < TOTAL) {
      const int q = e % Q, pix = e / Q;
      const int xx = pix % HC, yy = pix / HC;
      const int gy = y0 + yy - 1, gx = x0 + xx - 1;
      if (gy >= 0 && gy < n && gx >= 0 && gx < m)
        v[u] = *(const f32x4*)(in + (((size_t)i * n + gy) * m + gx) * CIN + 4 * q);
    }
  }
#pragma unroll
  for (int u = 0; u < SLOTS; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e < TOTAL) {
      const int q = e % Q, pix = e / Q;
      float* dst = s_in + pix * CP + 4 * q;
      dst[0] = v[u][0];
      dst[1] = v[u][1];
      dst[2] = v[u][2];
      dst[3] = v[u][3];
    }
  }
}

typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// The same staging for a BF16 NHWC input, widened to FP32 in LDS (16-byte loads of
// 8 channels).
template <int CIN, int HR, int HC, int CP, int NT>
__device__ __forceinline__ void stage_halo(const bf16_t* __restrict__ in, int i, int n, int m, int y0,
                                           int x0, float* s_in) {
  constexpr int Q = CIN / 8;
  constexpr int TOTAL = HR * HC * Q;
  constexpr int SLOTS = (TOTAL + NT - 1) / NT;
  u16x8 v[SLOTS];
#pragma unroll
  for (int u = 0; u < SLOTS; ++u) {
    const int e = threadIdx.x + u * NT;
    v[u] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
    if (e < TOTAL) {
      const int q = e % Q, pix = e / Q;
      const int xx = pix % HC, yy = pix / HC;
      const int gy = y0 + yy - 1, gx = x0 + xx - 1;
      if (gy >= 0 && gy < n && gx >= 0 && gx < m)
        v[u] = *(const u16x8*)(in + (((size_t)i * n + gy) * m + gx) * CIN + 8 * q);
    }
  }
#pragma unroll
  for (int u = 0; u < SLOTS; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e < TOTAL) {
      const int q = e % Q, pix = e / Q;
      float* dst = s_in + pix * CP + 8 * q;
#pragma unroll
      for (int j = 0; j < 8; ++j) dst[j] = from_bf16(v[u][j]);
    }
  }
}

// Hidden layer as an implicit GEMM on MFMA (v_mfma_f32_16x16x4_f32): rows = output
// pixels, columns = output channels, K = 9*CIN ordered (channel chunk, tap, channel).
// A block owns TR output rows x 64 output columns of one member; wave w computes rows
// w, w+4, ... as 16-pixel M-blocks against all COUT/16 N-blocks.  The input channels
// are taken CCH at a time: per chunk the halo tile ((TR+2) x 66 x CCH, zero-padded)
// and the weight rows Wk[tap*CIN + c][o] of those channels sit in LDS (so 64-channel
// layers fit), and the accumulators carry over the chunks.  The pixel stride in LDS
// is CCH+1 floats so the 16 pixels of an A fragment fall in distinct banks.  Lane
// layout (16x16x4 f32): A[i][k] from lane i + 16k, B[k][j] from lane j + 16k, and
// element r of lane j + 16g holds D[4g + r][j].
template <int CIN, int COUT, int TR, int CCH>
__global__ __launch_bounds__(256) void k_conv_mfma_f32(int N, int n, int m,
                                                       const float* __restrict__ in,
                                                       const float* __restrict__ wk,
                                                       const float* __restrict__ bias, int act,
                                                       float* __restrict__ out) {
  static_assert(CIN % CCH == 0 && CCH % 4 == 0, "channel chunks");
  constexpr int TC = 64;
  constexpr int HR = TR + 2, HC = TC + 2;
  constexpr int CP = CCH + 1;
  constexpr int KC = 9 * CCH;  // K-indices per chunk
  constexpr int NB = COUT / 16;
  constexpr int RPW = TR / 4;  // output rows per wave
  __shared__ __attribute__((aligned(16))) float s_in[HR * HC * CP];
  __shared__ __attribute__((aligned(16))) float s_w[KC * COUT];
  const int col_tiles = (m + TC - 1) / TC;
  const int row_tiles = (n + TR - 1) / TR;
  int bid = blockIdx.x;
  const int ct = bid % col_tiles;
  bid /= col_tiles;
  const int rt = bid % row_tiles;
  const int i = bid / row_tiles;
  const int y0 = rt * TR, x0 = ct * TC;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  f32x4 acc[RPW][4][NB];
#pragma unroll
  for (int rw = 0; rw < RPW; ++rw)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[rw][mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int c0 = 0; c0 < CIN; c0 += CCH) {
    if (c0 > 0) __syncthreads();  // the previous chunk's reads are done
    {
      // weight rows (tap, c0..c0+CCH) -> s_w[(tap*CCH + cc)*COUT + o]; every global
      // load of the thread is issued before its first LDS store
      constexpr int WQ = CCH * COUT / 4;  // float4 per tap
      constexpr int WV = 9 * WQ;
      constexpr int WS = (WV + 255) / 256;
      constexpr int Q = CCH / 4;
      constexpr int TOTAL = HR * HC * Q;
      constexpr int SLOTS = (TOTAL + 255) / 256;
      f32x4 wv[WS], v[SLOTS];
#pragma unroll
      for (int u = 0; u < WS; ++u) {
        const int e = tid + 256 * u;
        const int tap = e / WQ, r = e - tap * WQ;
        wv[u] = e < WV ? *(const f32x4*)(wk + ((size_t)tap * CIN + c0) * COUT + 4 * r)
                       : f32x4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int u = 0; u < SLOTS; ++u) {
        const int e = tid + u * 256;
        v[u] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (e < TOTAL) {
          const int q = e % Q, pix = e / Q;
          const int xx = pix % HC, yy = pix / HC;
          const int gy = y0 + yy - 1, gx = x0 + xx - 1;
          if (gy >= 0 && gy < n && gx >= 0 && gx < m)
            v[u] = *(const f32x4*)(in + (((size_t)i * n + gy) * m + gx) * CIN + c0 + 4 * q);
        }
      }
#pragma unroll
      for (int u = 0; u < WS; ++u) {
        const int e = tid + 256 * u;
        if (e < WV) *(f32x4*)(s_w + 4 * e) = wv[u];
      }
#pragma unroll
      for (int u = 0; u < SLOTS; ++u) {
        const int e = tid + u * 256;
        if (e < TOTAL) {
          const int q = e % Q, pix = e / Q;
          float* dst = s_in + pix * CP + 4 * q;
          dst[0] = v[u][0];
          dst[1] = v[u][1];
          dst[2] = v[u][2];
          dst[3] = v[u][3];
        }
      }
    }
    __syncthreads();
#pragma unroll 2
    for (int kb = 0; kb < KC / 4; ++kb) {
      const int k = kb * 4 + lk;
      const int tap = k / CCH, c = k - tap * CCH;
      const int dy = tap / 3, dx = tap - dy * 3;
      float b[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) b[nb] = s_w[k * COUT + nb * 16 + li];
#pragma unroll
      for (int rw = 0; rw < RPW; ++rw) {
        const int ry = w + 4 * rw;
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          const float a = s_in[((ry + dy) * HC + mb * 16 + li + dx) * CP + c];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[rw][mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[nb], acc[rw][mb][nb], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int rw = 0; rw < RPW; ++rw) {
    const int y = y0 + w + 4 * rw;
    if (y >= n) continue;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int o = nb * 16 + li;
        const float bo = bias ? bias[o] : 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int x = x0 + mb * 16 + 4 * lk + r;
          if (x < m)
            out[(((size_t)i * n + y) * m + x) * COUT + o] = activate(acc[rw][mb][nb][r] + bo, act);
        }
      }
  }
}

// First layer with the lift fused: the block stages the 6 x 66 halo of X, the l rows
// of U over the same columns and the 6 rows of B in LDS (all loads issued before the
// stores), forms B U per halo cell from LDS, computes 4 x 64 output pixels x COUT
// channels on the VALU (18 taps each), and writes the NHWC rows out through LDS so
// that the global stores are contiguous.
template <int COUT, typename TOUT>
__global__ __launch_bounds__(256) void k_conv_first(int N, int n, int m, int l, FieldRef X,
                                                    FieldRef U, const float* __restrict__ B,
                                                    const float* __restrict__ w,
                                                    const float* __restrict__ bias, int act,
                                                    TOUT* __restrict__ out) {
  constexpr int TR = 4, TC = 64, HR = TR + 2, HC = TC + 2;
  constexpr int LMAX = 64;
  __shared__ float s_x[HR * HC];
  __shared__ float s_bu[HR * HC];
  __shared__ float s_u[LMAX * HC];
  __shared__ float s_b[HR * LMAX];
  __shared__ float s_w[COUT * 18 + COUT];
  __shared__ float s_out[TR * TC * (COUT + 1)];
  const int col_tiles = (m + TC - 1) / TC;
  const int row_tiles = (n + TR - 1) / TR;
  int bid = blockIdx.x;
  const int ct = bid % col_tiles;
  bid /= col_tiles;
  const int rt = bid % row_tiles;
  const int i = bid / row_tiles;
  const int y0 = rt * TR, x0 = ct * TC;
  const int tid = threadIdx.x;
  {
    // X halo: 396 cells; U rows: l x 66; B rows: 6 x l  (l <= 64)
    constexpr int XS = (HR * HC + 255) / 256;
    constexpr int US = (LMAX * HC + 255) / 256;
    float xv[XS], uv[US], bv[2];
#pragma unroll
    for (int u = 0; u < XS; ++u) {
      const int e = tid + 256 * u;
      const int yy = e / HC, xx = e % HC;
      const int gy = y0 + yy - 1, gx = x0 + xx - 1;
      xv[u] = (e < HR * HC && gy >= 0 && gy < n && gx >= 0 && gx < m) ? X.base[i * X.si + gy * X.sy + gx]
                                                                       : 0.f;
    }
#pragma unroll
    for (int u = 0; u < US; ++u) {
      const int e = tid + 256 * u;
      const int a = e / HC, xx = e % HC;
      const int gx = x0 + xx - 1;
      uv[u] = (a < l && gx >= 0 && gx < m) ? U.base[i * U.si + a * U.sy + gx] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = tid + 256 * u;
      const int yy = e / LMAX, a = e % LMAX;
      const int gy = y0 + yy - 1;
      bv[u] = (yy < HR && a < l && gy >= 0 && gy < n) ? B[(size_t)gy * l + a] : 0.f;
    }
    for (int e = tid; e < COUT * 18; e += 256) s_w[e] = w[e];
    if (tid < COUT) s_w[COUT * 18 + tid] = bias ? bias[tid] : 0.f;
#pragma unroll
    for (int u = 0; u < XS; ++u)
      if (tid + 256 * u < HR * HC) s_x[tid + 256 * u] = xv[u];
#pragma unroll
    for (int u = 0; u < US; ++u)
      if (tid + 256 * u < LMAX * HC) s_u[tid + 256 * u] = uv[u];
#pragma unroll
    for (int u = 0; u < 2; ++u)
      if (tid + 256 * u < HR * LMAX) s_b[tid + 256 * u] = bv[u];
  }
  __syncthreads();
  for (int e = tid; e < HR * HC; e += 256) {
    const int yy = e / HC, xx = e % HC;
    float bu = 0.f;
    for (int a = 0; a < l; ++a) bu = fmaf(s_b[yy * LMAX + a], s_u[a * HC + xx], bu);
    s_bu[e] = bu;
  }
  __syncthreads();
  const int ty = tid / TC, tx = tid % TC;
  float inx[18];
#pragma unroll
  for (int dy = 0; dy < 3; ++dy)
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      inx[dy * 3 + dx] = s_x[(ty + dy) * HC + tx + dx];
      inx[9 + dy * 3 + dx] = s_bu[(ty + dy) * HC + tx + dx];
    }
#pragma unroll 4
  for (int o = 0; o < COUT; ++o) {
    float acc = s_w[COUT * 18 + o];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc = fmaf(s_w[o * 18 + q], inx[q], acc);          // channel X
#pragma unroll
    for (int q = 0; q < 9; ++q) acc = fmaf(s_w[o * 18 + 9 + q], inx[9 + q], acc);  // channel B U
    s_out[tid * (COUT + 1) + o] = activate(acc, act);
  }
  __syncthreads();
  for (int r = 0; r < TR; ++r) {
    const int y = y0 + r;
    if (y >= n) break;
    const int valid = min(TC, m - x0);
    TOUT* dst = out + (((size_t)i * n + y) * m + x0) * COUT;
    for (int e = tid; e < valid * COUT; e += 256) {
      const int px = e / COUT, o = e % COUT;
      store_act(dst + e, s_out[(r * TC + px) * (COUT + 1) + o]);
    }
  }
}

// Last layer (one output channel) from an LDS halo tile of the NHWC input; each
// thread computes one pixel (9*CIN taps) and the store to the strided field is
// contiguous along x.
template <int CIN, typename TIN>
__global__ __launch_bounds__(256) void k_conv_last(int N, int n, int m, const TIN* __restrict__ in,
                                                   const float* __restrict__ w,
                                                   const float* __restrict__ bias, FieldOut fo) {
  constexpr int TR = 4, TC = 64, HR = TR + 2, HC = TC + 2, CP = CIN + 1;
  __shared__ __attribute__((aligned(16))) float s_in[HR * HC * CP];
  __shared__ float s_w[9 * CIN];
  const int col_tiles = (m + TC - 1) / TC;
  const int row_tiles = (n + TR - 1) / TR;
  int bid = blockIdx.x;
  const int ct = bid % col_tiles;
  bid /= col_tiles;
  const int rt = bid % row_tiles;
  const int i = bid / row_tiles;
  const int y0 = rt * TR, x0 = ct * TC;
  const int tid = threadIdx.x;
  // weights [0][c][dy][dx] -> s_w[tap * CIN + c]
  for (int e = tid; e < 9 * CIN; e += 256) {
    const int c = e / 9, tap = e % 9;
    s_w[tap * CIN + c] = w[e];
  }
  stage_halo<CIN, HR, HC, CP, 256>(in, i, n, m, y0, x0, s_in);
  __syncthreads();
  const int ty = tid / TC, tx = tid % TC;
  const int y = y0 + ty, x = x0 + tx;
  float acc = bias ? bias[0] : 0.f;
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int dy = tap / 3, dx = tap % 3;
    const float* src = s_in + ((ty + dy) * HC + tx + dx) * CP;
#pragma unroll 8
    for (int c = 0; c < CIN; ++c) acc = fmaf(s_w[tap * CIN + c], src[c], acc);
  }
  if (y < n && x < m) fo.base[i * fo.si + y * fo.sy + x] = acc;
}

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// Hidden layer in BF16 on MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulation): the
// same tiling as the FP32 kernel, but each k-step covers 32 K-indices (tap, channel)
// and every lane supplies 8 consecutive channels of one tap for A and 8 consecutive
// K-indices of one output channel for B, each as one 16-byte LDS read.  Input and
// output activations are BF16 NHWC; the weights sit in LDS as [o][tap*CIN + c].
// Row strides in LDS are padded by 8 elements so the 16 lanes of a fragment hit
// distinct banks.  Lane layout (16x16x32): A[i][k] for k = 8g..8g+7 from lane i + 16g,
// B[k][j] for k = 8g..8g+7 from lane j + 16g, element r of lane j + 16g holds D[4g + r][j].
template <int CIN, int COUT, int TR>
__global__ __launch_bounds__(256) void k_conv_mfma_bf16(int N, int n, int m,
                                                        const bf16_t* __restrict__ in,
                                                        const bf16_t* __restrict__ wt,
                                                        const float* __restrict__ bias, int act,
                                                        bf16_t* __restrict__ out) {
  constexpr int TC = 64;
  constexpr int HR = TR + 2, HC = TC + 2;
  constexpr int CP = CIN + 8;
  constexpr int KD = 9 * CIN;
  constexpr int KD32 = (KD + 31) / 32 * 32;  // K rounded up to whole k-steps (zero weights past KD)
  constexpr int KDP = KD32 + 8;
  constexpr int NB = COUT / 16;
  constexpr int RPW = TR / 4;
  __shared__ __attribute__((aligned(16))) bf16_t s_in[HR * HC * CP];
  __shared__ __attribute__((aligned(16))) bf16_t s_w[COUT * KDP];
  const int col_tiles = (m + TC - 1) / TC;
  const int row_tiles = (n + TR - 1) / TR;
  int bid = blockIdx.x;
  const int ct = bid % col_tiles;
  bid /= col_tiles;
  const int rt = bid % row_tiles;
  const int i = bid / row_tiles;
  const int y0 = rt * TR, x0 = ct * TC;
  const int tid = threadIdx.x;
  {
    constexpr int WQ = KD / 8;              // 16-byte vectors per weight row
    constexpr int WV = COUT * WQ;
    constexpr int WS = (WV + 255) / 256;
    constexpr int IQ = CIN / 8;
    constexpr int IV = HR * HC * IQ;
    constexpr int IS = (IV + 255) / 256;
    u16x8 wv[WS], iv[IS];
#pragma unroll
    for (int u = 0; u < WS; ++u) {
      const int e = tid + 256 * u;
      wv[u] = e < WV ? *(const u16x8*)(wt + (size_t)8 * e) : u16x8{0, 0, 0, 0, 0, 0, 0, 0};
    }
#pragma unroll
    for (int u = 0; u < IS; ++u) {
      const int e = tid + 256 * u;
      iv[u] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      if (e < IV) {
        const int q = e % IQ, pix = e / IQ;
        const int xx = pix % HC, yy = pix / HC;
        const int gy = y0 + yy - 1, gx = x0 + xx - 1;
        if (gy >= 0 && gy < n && gx >= 0 && gx < m)
          iv[u] = *(const u16x8*)(in + (((size_t)i * n + gy) * m + gx) * CIN + 8 * q);
      }
    }
#pragma unroll
    for (int u = 0; u < WS; ++u) {
      const int e = tid + 256 * u;
      if (e < WV) *(u16x8*)(s_w + (e / WQ) * KDP + 8 * (e % WQ)) = wv[u];
    }
    if (KD32 > KD) {  // zero the K padding of every weight row
      constexpr int PQ = (KD32 - KD) / 8;
      for (int e = tid; e < COUT * PQ; e += 256)
        *(u16x8*)(s_w + (e / PQ) * KDP + KD + 8 * (e % PQ)) = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
    }
#pragma unroll
    for (int u = 0; u < IS; ++u) {
      const int e = tid + 256 * u;
      if (e < IV) *(u16x8*)(s_in + (e / IQ) * CP + 8 * (e % IQ)) = iv[u];
    }
  }
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  f32x4 acc[RPW][4][NB];
#pragma unroll
  for (int rw = 0; rw < RPW; ++rw)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[rw][mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 3
  for (int kb = 0; kb < KD32 / 32; ++kb) {
    const int k0 = kb * 32 + 8 * lk;
    // past KD the weights are zero; read any in-tile (finite) activations there
    const int kk = k0 < KD ? k0 : 0;
    const int tap = kk / CIN, c0 = kk - tap * CIN;
    const int dy = tap / 3, dx = tap - dy * 3;
    bf16x8_t b[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      b[nb] = __builtin_bit_cast(bf16x8_t, *(const u16x8*)(s_w + (nb * 16 + li) * KDP + k0));
#pragma unroll
    for (int rw = 0; rw < RPW; ++rw) {
      const int ry = w + 4 * rw;
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        const bf16x8_t a = __builtin_bit_cast(
            bf16x8_t, *(const u16x8*)(s_in + ((ry + dy) * HC + mb * 16 + li + dx) * CP + c0));
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[rw][mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[nb], acc[rw][mb][nb], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int rw = 0; rw < RPW; ++rw) {
    const int y = y0 + w + 4 * rw;
    if (y >= n) continue;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int o = nb * 16 + li;
        const float bo = bias ? bias[o] : 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int x = x0 + mb * 16 + 4 * lk + r;
          if (x < m)
            out[(((size_t)i * n + y) * m + x) * COUT + o] = to_bf16(activate(acc[rw][mb][nb][r] + bo, act));
        }
      }
  }
}

}  // namespace

bool conv_first_supported(int cout, int l) {
  return (cout == 8 || cout == 16 || cout == 32 || cout == 64) && l <= 64;
}
bool conv_last_supported(int cin) { return cin == 8 || cin == 16 || cin == 32 || cin == 64; }

void launch_conv_first(hipStream_t s, Timer& t, int N, int n, int m, int l, FieldRef X, FieldRef U,
                       const float* B, int cout, const float* w, const float* bias, int act,
                       void* out_nhwc, bool bf16) {
  const unsigned blocks = (unsigned)((long long)N * ((n + 3) / 4) * ((m + 63) / 64));
#define OIC_FIRST_CASE(CO)                                                                        \
  if (cout == CO) {                                                                               \
    if (bf16)                                                                                     \
      OIC_LAUNCH(t, KC_CONV_FIRST, s, (k_conv_first<CO, bf16_t>), dim3(blocks), dim3(256), 0, N, n, \
                 m, l, X, U, B, w, bias, act, (bf16_t*)out_nhwc);                                 \
    else                                                                                          \
      OIC_LAUNCH(t, KC_CONV_FIRST, s, (k_conv_first<CO, float>), dim3(blocks), dim3(256), 0, N, n,  \
                 m, l, X, U, B, w, bias, act, (float*)out_nhwc);                                  \
    return;                                                                                       \
  }
  OIC_FIRST_CASE(8)
  OIC_FIRST_CASE(16)
  OIC_FIRST_CASE(32)
  OIC_FIRST_CASE(64)
#undef OIC_FIRST_CASE
}

void launch_conv_last(hipStream_t s, Timer& t, int N, int n, int m, int cin, const void* in_nhwc,
                      const float* w, const float* bias, FieldOut fo, bool bf16) {
  const unsigned blocks = (unsigned)((long long)N * ((n + 3) / 4) * ((m + 63) / 64));
#define OIC_LAST_CASE(CI)                                                                         \
  if (cin == CI) {                                                                                \
    if (bf16)                                                                                     \
      OIC_LAUNCH(t, KC_CONV_LAST, s, (k_conv_last<CI, bf16_t>), dim3(blocks), dim3(256), 0, N, n, m, \
                 (const bf16_t*)in_nhwc, w, bias, fo);                                            \
    else                                                                                          \
      OIC_LAUNCH(t, KC_CONV_LAST, s, (k_conv_last<CI, float>), dim3(blocks), dim3(256), 0, N, n, m,  \
                 (const float*)in_nhwc, w, bias, fo);                                             \
    return;                                                                                       \
  }
  OIC_LAST_CASE(8)
  OIC_LAST_CASE(16)
  OIC_LAST_CASE(32)
  OIC_LAST_CASE(64)
#undef OIC_LAST_CASE
}

bool conv_mfma_bf16_supported(int cin, int cout) {
  return (cin == 16 && cout == 16) || (cin == 32 && cout == 32) || (cin == 64 && cout == 64) ||
         (cin == 16 && cout == 32) || (cin == 32 && cout == 16) || (cin == 32 && cout == 64) ||
         (cin == 64 && cout == 32);
}

void launch_conv_mfma_bf16(hipStream_t s, Timer& t, int kclass, int N, int n, int m, int cin, int cout,
                           const void* in_nhwc, const void* wt, const float* bias, int act,
                           void* out_nhwc) {
#define OIC_BF_CASE(CI, CO)                                                                      \
  if (cin == CI && cout == CO) {                                                                 \
    constexpr int TRV = CI <= 32 ? 8 : 4;                                                        \
    const unsigned blocks = (unsigned)((long long)N * ((n + TRV - 1) / TRV) * ((m + 63) / 64));  \
    OIC_LAUNCH(t, kclass, s, (k_conv_mfma_bf16<CI, CO, TRV>), dim3(blocks), dim3(256), 0, N, n, m, \
               (const bf16_t*)in_nhwc, (const bf16_t*)wt, bias, act, (bf16_t*)out_nhwc);         \
    return;                                                                                      \
  }
  OIC_BF_CASE(16, 16)
  OIC_BF_CASE(32, 32)
  OIC_BF_CASE(64, 64)
  OIC_BF_CASE(16, 32)
  OIC_BF_CASE(32, 16)
  OIC_BF_CASE(32, 64)
  OIC_BF_CASE(64, 32)
#undef OIC_BF_CASE
}

bool conv_mfma_supported(int cin, int cout) {
  return (cin == 16 || cin == 32 || cin == 64) && (cout == 16 || cout == 32 || cout == 64);
}

void launch_conv_mfma(hipStream_t s, Timer& t, int kclass, int N, int n, int m, int cin, int cout,
                      const float* in_nhwc, const float* wk, const float* bias, int act,
                      float* out_nhwc) {
#define OIC_CONV_CASE(CI, CO)                                                                   \
  if (cin == CI && cout == CO) {                                                                \
    constexpr int TRV = (CI <= 16 && CO <= 32) ? 8 : 4;                                         \
    constexpr int CCH = CI <= 32 ? CI : 32;                                                     \
    const unsigned blocks = (unsigned)((long long)N * ((n + TRV - 1) / TRV) * ((m + 63) / 64)); \
    OIC_LAUNCH(t, kclass, s, (k_conv_mfma_f32<CI, CO, TRV, CCH>), dim3(blocks), dim3(256), 0, N, n, \
               m, in_nhwc, wk, bias, act, out_nhwc);                                            \
    return;                                                                                     \
  }
  OIC_CONV_CASE(16, 16)
  OIC_CONV_CASE(32, 32)
  OIC_CONV_CASE(16, 32)
  OIC_CONV_CASE(32, 16)
  OIC_CONV_CASE(64, 64)
  OIC_CONV_CASE(16, 64)
  OIC_CONV_CASE(64, 16)
  OIC_CONV_CASE(32, 64)
  OIC_CONV_CASE(64, 32)
#undef OIC_CONV_CASE
}

void launch_lift(hipStream_t s, Timer& t, int N, int n, int m, int l, FieldRef X, FieldRef U,
                 const float* B, float* out_nhwc) {
  const long long total = (long long)N * n * m;
  OIC_LAUNCH(t, KC_LIFT, s, k_lift, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, N, n, m,
             l, X, U, B, out_nhwc);
}

void launch_conv(hipStream_t s, Timer& t, int kclass, int N, int n, int m, int cin, int cout,
                 const float* in_nhwc, const float* w_oihw, const float* bias, int act,
                 float* out_nhwc, FieldOut final_out) {
  const long long total = (long long)N * n * m;
  const unsigned gx = (unsigned)((total + 255) / 256);
  if (cout == 1) {
    OIC_LAUNCH(t, kclass, s, k_conv_direct<1>, dim3(gx, 1), dim3(256), 0, N, n, m, cin, cout,
               in_nhwc, w_oihw, bias, act, out_nhwc, final_out);
    return;
  }
  constexpr int CB = 16;
  const unsigned gy = (unsigned)((cout + CB - 1) / CB);
  OIC_LAUNCH(t, kclass, s, k_conv_direct<CB>, dim3(gx, gy), dim3(256), 0, N, n, m, cin, cout,
             in_nhwc, w_oihw, bias, act, out_nhwc, final_out);
}

}  // namespace oic
