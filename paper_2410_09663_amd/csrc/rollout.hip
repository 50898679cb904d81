// Ensemble rollout through the CNN surrogate, Eq. (1) / Eq. (15b):
// x0 = [X, B U] (two channels), then zero-padded 3x3 cross-correlation layers
// with the activation between them and none after the last.
//
// Activations are NHWC [member][row][col][channel].  The first kernel ("lift")
// builds the two input channels straight from the trajectory buffer; the last
// layer writes its single channel straight back into the trajectory (or any
// strided field), so no extra pass touches the next state.
#include "noise_value.h"
#include "oic_internal.h"

namespace oic {
namespace {

// tanh from the hardware exp2 and reciprocal: tanh|x| = 1 - 2 / (exp(2|x|) + 1) for
// |x| >= 1/8, and its odd Taylor series to x^7 below (truncation < 2e-9 there, where
// the closed form would lose relative accuracy to cancellation).  Absolute error a few
// 1e-8, relative error below 1e-6 everywhere.
__device__ __forceinline__ float fast_tanh(float x) {
  const float a = fabsf(x);
  const float e = __builtin_amdgcn_exp2f(a * 2.8853900817779268f);  // exp(2a) = 2^(2a log2 e)
  float big = 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
  big = a > 44.0f ? 1.0f : big;
  const float a2 = a * a;
  const float small = a * fmaf(a2, fmaf(a2, fmaf(a2, -17.0f / 315.0f, 2.0f / 15.0f), -1.0f / 3.0f), 1.0f);
  return copysignf(a < 0.125f ? small : big, x);
}

// erf by Abramowitz & Stegun 7.1.26 (Hastings' rational approximation), absolute error
// below 1.5e-7: erf|x| = 1 - (a1 t + ... + a5 t^5) exp(-x^2), t = 1 / (1 + p|x|).
__device__ __forceinline__ float fast_erf(float x) {
  const float a = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, a, 1.0f));
  const float poly =
      t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f),
               0.254829592f);
  const float ex = __builtin_amdgcn_exp2f(-a * a * 1.4426950408889634f);  // exp(-a^2)
  return copysignf(1.0f - poly * ex, x);
}

__device__ __forceinline__ float activate(float v, int act) {
  if (act == OIC_ACT_TANH) return fast_tanh(v);
  return 0.5f * v * (1.0f + fast_erf(v * 0.70710678118654752f));  // GELU, erf form
}

// GELU from a polynomial erf with no transcendental instructions: erf(z) on [0, 3.5] is
// fitted by z (c0 + ... + c8 z^8) (absolute error below 5e-5; erf = 1 beyond 3.5, where
// 1 - erf(3.5) = 7.4e-7), and since erf is odd, GELU(x) = x/2 + |x| erf(|x|/sqrt2)/2 =
// fma(|x| a, Q(a), x/2) with a = min(|x|, 3.5 sqrt2) and q_k = c_k / (2 sqrt2^(k+1)).
// Coefficients written by gen_erf_poly.py; twelve instructions per value.
constexpr float kGeluPoly[9] = {3.990201056e-01f, -2.460608492e-03f, -5.473593995e-02f, -2.319048159e-02f,
                                3.365044296e-02f, -1.329257339e-02f, 2.602266148e-03f, -2.602511959e-04f,
                                1.064957814e-05f};
__device__ __forceinline__ float poly_gelu(float x) {
  const float a = fabsf(x);
  const float ac = fminf(a, 4.94974746830583f);
  float p = kGeluPoly[8];
#pragma unroll
  for (int k = 7; k >= 0; --k) p = fmaf(p, ac, kGeluPoly[k]);
  return fmaf(a * ac, p, 0.5f * x);
}

// The activation of the layers whose outputs are stored in BF16 (the BF16 and FP8
// rollouts): GELU through poly_gelu, whose error (|x|/2 times the erf fit's, plus the FP32
// rounding of the Horner sum: at most 3.5e-5 relative) is far below BF16's rounding of the
// stored value (2^-9 relative); tanh as in activate.
__device__ __forceinline__ float activate_lp(float v, int act) {
  if (act == OIC_ACT_TANH) return fast_tanh(v);
  return poly_gelu(v);
}

// The activation as a compile-time choice: epilogues that evaluate it for every output
// element branch on the runtime code once per tile and run a straight-line body for it.
template <int A>
struct ActC {
  static constexpr int value = A;
};
template <int ACT>
__device__ __forceinline__ float activate_c(float v) {
  if constexpr (ACT == OIC_ACT_TANH)
    return fast_tanh(v);
  else
    return 0.5f * v * (1.0f + fast_erf(v * 0.70710678118654752f));  // GELU, erf form
}
template <int ACT>
__device__ __forceinline__ float activate_lp_c(float v) {
  if constexpr (ACT == OIC_ACT_TANH) {
    return fast_tanh(v);
  } else {
    return poly_gelu(v);
  }
}
// Runs f(ActC<act>{}) for the runtime activation code.
template <typename F>
__device__ __forceinline__ void with_activation(int act, F&& f) {
  if (act == OIC_ACT_TANH)
    f(ActC<OIC_ACT_TANH>{});
  else
    f(ActC<OIC_ACT_GELU>{});
}

// BF16 storage: round to nearest even (the hardware conversion; activations are finite),
// and back by shifting.
typedef unsigned short bf16_t;
__device__ __forceinline__ bf16_t to_bf16(float f) { return __builtin_bit_cast(bf16_t, (__bf16)f); }
// Two values as one 32-bit word of BF16s (lo in the low half): one v_cvt_pk_bf16_f32.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned pack_bf16x2(float lo, float hi) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2_t{lo, hi}, bf16x2_t));
}
__device__ __forceinline__ float from_bf16(bf16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ void store_act(float* p, float v) { *p = v; }
__device__ __forceinline__ void store_act(bf16_t* p, float v) { *p = to_bf16(v); }

// Largest |value| written by a wave, folded into *amax (the bit pattern of a
// non-negative float orders like the float, so an integer max is exact and the
// result does not depend on the order of the atomics).
// The wave's maximum goes to one of the layer's kAmaxSlots slots, chosen by workgroup and
// wave so that the atomics of a launch spread over all of them.  A slot only grows during
// a launch, so a wave whose maximum does not exceed the value it reads there (current or
// older) has nothing to add and skips its atomic: once the slots hold the layer's typical
// maxima, few of the hundreds of thousands of waves of a first layer still queue on them.
__device__ __forceinline__ void amax_publish(float v, unsigned* amax) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  const unsigned slot = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % kAmaxSlots;
  const unsigned u = __float_as_uint(v);
  if ((threadIdx.x & 63) == 0 && u > amax[slot]) atomicMax(amax + slot, u);
}

// The layer's largest |activation|: the maximum over its slots.
__device__ __forceinline__ float amax_read(const unsigned* __restrict__ amax) {
  unsigned mx = 0u;
#pragma unroll 8
  for (int s = 0; s < kAmaxSlots; ++s) mx = max(mx, amax[s]);
  return __uint_as_float(mx);
}

__global__ void k_zero_u32(unsigned* __restrict__ p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0u;
}

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
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

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
// Eight BF16 activations from floats as one 16-byte store (p 16-byte aligned).
__device__ __forceinline__ void store_vec16(bf16_t* p, const float* v) {
  u16x8 h;
#pragma unroll
  for (int q = 0; q < 8; ++q) h[q] = to_bf16(v[q]);
  *(u16x8*)p = h;
}

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

// The same layer for CIN <= 32 (one channel chunk) as a persistent kernel: a block
// keeps the weights in LDS and walks over tiles tile, tile + gridDim.x, ...; the next
// tile's halo is loaded into registers while the current one is on the matrix cores,
// so the global-load latency of a tile hides behind the previous tile's MFMAs.
template <int CIN, int COUT, int TR, int WGM>
__global__ __launch_bounds__(256 * WGM) void k_conv_mfma_f32p(int N, int n, int m,
                                                        const float* __restrict__ in,
                                                        const float* __restrict__ wk,
                                                        const float* __restrict__ bias, int act,
                                                        float* __restrict__ out) {
  constexpr int TC = 64;
  constexpr int HR = TR + 2, HC = TC + 2;
  constexpr int CP = CIN + 1;
  constexpr int KD = 9 * CIN;
  constexpr int NB = COUT / 16;
  constexpr int NW = 4 * WGM, NT = 64 * NW;  // waves: one output row each per pass
  static_assert(TR % NW == 0, "whole rows per wave");
  constexpr int RPW = TR / NW;
  constexpr int Q = CIN / 4;
  constexpr int TOTAL = HR * HC * Q;
  constexpr int SLOTS = (TOTAL + NT - 1) / NT;
  __shared__ __attribute__((aligned(16))) float s_in[HR * HC * CP];
  __shared__ __attribute__((aligned(16))) float s_w[KD * COUT];
  const int col_tiles = (m + TC - 1) / TC;
  const int row_tiles = (n + TR - 1) / TR;
  const int tiles = N * row_tiles * col_tiles;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  {
    constexpr int WV = KD * COUT / 4;
    constexpr int WS = (WV + NT - 1) / NT;
#pragma unroll
    for (int u = 0; u < WS; ++u) {
      const int e = tid + NT * u;
      if (e < WV) *(f32x4*)(s_w + 4 * e) = *(const f32x4*)(wk + 4 * e);
    }
  }
  f32x4 v[SLOTS];
  auto load_halo = [&](int tile) {
    const int ct = tile % col_tiles, rest = tile / col_tiles;
    const int rt = rest % row_tiles, i = rest / row_tiles;
    const int y0 = rt * TR, x0 = ct * TC;
#pragma unroll
    for (int u = 0; u < SLOTS; ++u) {
      const int e = tid + u * NT;
      v[u] = f32x4{0.f, 0.f, 0.f, 0.f};
      if (e < TOTAL) {
        const int q = e % Q, pix = e / Q;
        const int xx = pix % HC, yy = pix / HC;
        const int gy = y0 + yy - 1, gx = x0 + xx - 1;
        if (gy >= 0 && gy < n && gx >= 0 && gx < m)
          v[u] = *(const f32x4*)(in + (((size_t)i * n + gy) * m + gx) * CIN + 4 * q);
      }
    }
  };
  int tile = blockIdx.x;
  if (tile < tiles) load_halo(tile);
  for (; tile < tiles; tile += gridDim.x) {
    const int ct = tile % col_tiles, rest = tile / col_tiles;
    const int rt = rest % row_tiles, i = rest / row_tiles;
    const int y0 = rt * TR, x0 = ct * TC;
    __syncthreads();  // the previous tile's MFMAs are done with s_in (and s_w is staged)
#pragma unroll
    for (int u = 0; u < SLOTS; ++u) {
      const int e = tid + u * NT;
      if (e < TOTAL) {
        const int q = e % Q, pix = e / Q;
        float* dst = s_in + pix * CP + 4 * q;
        dst[0] = v[u][0];
        dst[1] = v[u][1];
        dst[2] = v[u][2];
        dst[3] = v[u][3];
      }
    }
    __syncthreads();
    if (tile + (int)gridDim.x < tiles) load_halo(tile + gridDim.x);  // in flight meanwhile
    f32x4 acc[RPW][4][NB];
#pragma unroll
    for (int rw = 0; rw < RPW; ++rw)
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[rw][mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the matrix-core phase at raised wave priority, as in k_conv_f32r (64 x 64 FP32 solve:
    // 1.75 -> 1.73 ms; the BF16 and FP8 hidden layers with weights in LDS gain nothing)
    __builtin_amdgcn_s_setprio(1);
#pragma unroll 2
    for (int kb = 0; kb < KD / 4; ++kb) {
      const int k = kb * 4 + lk;
      const int tap = k / CIN, c = k - tap * CIN;
      const int dy = tap / 3, dx = tap - dy * 3;
      float b[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) b[nb] = s_w[k * COUT + nb * 16 + li];
#pragma unroll
      for (int rw = 0; rw < RPW; ++rw) {
        const int ry = w + NW * rw;
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          const float a = s_in[((ry + dy) * HC + mb * 16 + li + dx) * CP + c];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[rw][mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[nb], acc[rw][mb][nb], 0, 0, 0);
        }
      }
    }
    __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int rw = 0; rw < RPW; ++rw) {
      const int y = y0 + w + NW * rw;
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
}

// Persistent walk of `tiles` tiles by gridDim.x workgroups, aware of the eight XCDs:
// workgroup b runs on XCD b mod 8, so the tiles are cut into eight contiguous ranges and
// the workgroups of one XCD walk theirs side by side (tile = range start + b / 8,
// then + gridDim.x / 8, ...).  Neighbouring tiles share halo rows; this keeps the
// workgroups that read them at the same time behind the same L2.  When the grid is not
// a multiple of eight, or exceeds the tiles, a plain stride is used.
struct TileWalk {
  int first, step, end;
  __device__ TileWalk(int tiles) {
    const int G = gridDim.x;
    if ((G & 7) == 0 && tiles >= G) {
      const int x = blockIdx.x & 7;
      first = (int)((long long)tiles * x / 8) + (blockIdx.x >> 3);
      step = G >> 3;
      end = (int)((long long)tiles * (x + 1) / 8);
    } else {
      first = blockIdx.x;
      step = G;
      end = tiles;
    }
  }
};

// FP32 hidden layer CIN -> 64 on v_mfma_f32_16x16x4f32 with the weights held in
// registers.  Wave w of the four-wave workgroup owns output channels 16w..16w+15 for
// every pixel of a TR x 64 tile: its B fragments for all K = 9*CIN indices stay in
// registers for the whole (persistent) kernel, so the LDS holds only the halo tile and
// two workgroups fit on a CU (one stages its next tile while the other is on the matrix
// cores).  K is walked in steps of 16 channels of one tap: lane (i, g) reads channels
// c0+4g..c0+4g+3 of its pixel as one 16-byte LDS load and feeds them to four MFMAs, the
// j-th taking channel c0+4g+j in k-slot g, with the weights permuted the same way (each
// four-MFMA group then covers the 16 channels once).  The pixel stride in LDS is CIN+4
// floats: the eight lanes of a 128-byte LDS phase read 8 consecutive pixels at a
// 16-byte offset each, covering all banks.  Lane layout (16x16x4 f32): A[i][k] from lane
// i + 16k, B[k][j] from lane j + 16k, element r of lane j + 16g holds D[4g + r][j].
//
// LASTQ: this is the last hidden layer and the network's last layer (64 -> 1) is folded
// into the epilogue.  The activated tile goes to LDS instead of HBM and the last layer's
// per-tap partial sums P_tap(p) = sum_c wl[c][tap] h(p)[c] are formed on the matrix cores
// (K = 64 channels, the 9 taps as the N side); they leave as nine FP32 planes
// qout[tap][i][y][x] (plane stride N n m), and k_conv_last_sum adds the nine shifted
// taps: out(y, x) = sum over (dy, dx) of P_(dy,dx)(y + dy - 1, x + dx - 1).  Per pixel the
// hidden layer then writes 36 bytes instead of 256, and the last layer reads them once.
template <int CIN, int TR, bool LASTQ>
__global__ __launch_bounds__(256, 2) void k_conv_f32r(int N, int n, int m, const float* __restrict__ in,
                                                      const float* __restrict__ wk,
                                                      const float* __restrict__ bias, int act,
                                                      float* __restrict__ out, const float* __restrict__ wl) {
  constexpr int COUT = 64, TC = 64;
  constexpr int HR = TR + 2, HC = TC + 2;
  constexpr int CP = CIN + 4;
  constexpr int CG = CIN / 16;  // 16-channel groups per tap
  constexpr int S = 9 * CG;     // K steps of 16 indices
  // The halo arrives by LDS-direct buffer loads: 16-byte slot s of the tile (pixel s / SLOT,
  // channels 4 (s mod SLOT) ..; the last slot of a pixel is its padding) is loaded by lane
  // s mod 64 of wave-instruction s / 64, which writes 64 consecutive slots.  Slots outside
  // the field (and the padding) take an offset past the end of the buffer, which the
  // hardware returns as zeros.  No registers hold the halo and a tile costs one memory
  // round trip.
  constexpr int SLOT = CIN / 4 + 1;
  constexpr int TOTAL_SLOTS = HR * HC * SLOT;
  constexpr int INSTR = (TOTAL_SLOTS + 63) / 64;
  static_assert(CIN % 16 == 0, "16-channel K steps");
  static_assert(CP == 4 * SLOT, "pixel stride = whole slots");
  constexpr int HP = COUT + 4;  // pixel stride of the activated tile (LASTQ)
  static_assert(!LASTQ || TR * TC * HP <= HR * HC * CP, "the activated tile reuses the halo's LDS");
  __shared__ __attribute__((aligned(16))) float s_in[INSTR * 64 * 4];
  __shared__ float s_wl[LASTQ ? COUT * 16 : 1];  // last layer [c][tap], taps 9..15 zero
  const int col_tiles = (m + TC - 1) / TC;
  const int row_tiles = (n + TR - 1) / TR;
  const int tiles = N * row_tiles * col_tiles;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int o = 16 * w + li;
  if constexpr (LASTQ) {
    for (int e = tid; e < COUT * 16; e += 256) {
      const int c = e >> 4, tap = e & 15;
      s_wl[e] = tap < 9 ? wl[c * 9 + tap] : 0.f;
    }
  }
  // this lane's weights: step s, MFMA j -> W[tap][c0 + 4 lk + j][o]
  float wr[S][4];
#pragma unroll
  for (int st = 0; st < S; ++st) {
    const int tap = st / CG, c0 = (st % CG) * 16 + 4 * lk;
#pragma unroll
    for (int j = 0; j < 4; ++j) wr[st][j] = wk[((size_t)tap * CIN + c0 + j) * COUT + o];
  }
  const float bo = bias ? bias[o] : 0.f;
  const TileWalk walk(tiles);
  for (int tile = walk.first; tile < walk.end; tile += walk.step) {
    const int ct = tile % col_tiles, rest = tile / col_tiles;
    const int rt = rest % row_tiles, i = rest / row_tiles;
    const int y0 = rt * TR, x0 = ct * TC;
    __syncthreads();  // every wave is done with the previous tile
    {
      // member i's image as the buffer (its byte size fits the 32-bit record count: the
      // launcher checks), the halo's zero padding from out-of-range offsets
      const unsigned nrec = (unsigned)n * m * CIN * 4;
      const __amdgpu_buffer_rsrc_t rsrc =
          __builtin_amdgcn_make_buffer_rsrc((void*)(in + (size_t)i * n * m * CIN), (short)0, (int)nrec, 0x00020000);
#pragma unroll
      for (int u = 0; u < (INSTR + 3) / 4; ++u) {
        const int ins = w + 4 * u;  // wave-uniform
        if (ins < INSTR) {
          int slot = ins * 64 + lane;
          // recompute the slot's coordinates for every tile: hoisted out of the tile loop
          // they would not fit the registers beside the weights
          asm volatile("" : "+v"(slot));
          const int pix = slot / SLOT, q = slot - pix * SLOT;
          const int yy = pix / HC, xx = pix - yy * HC;
          const int gy = y0 + yy - 1, gx = x0 + xx - 1;
          const bool live = slot < TOTAL_SLOTS && q < CIN / 4 && gy >= 0 && gy < n && gx >= 0 && gx < m;
          const unsigned voff = live ? (unsigned)(((gy * m + gx) * CIN + 4 * q) * 4) : nrec;
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (__attribute__((address_space(3))) void*)(s_in + ins * 256),
                                                   16, (int)voff, 0, 0, 0);
        }
      }
      __builtin_amdgcn_s_waitcnt(0);  // the LDS-direct loads have landed (vmcnt)
    }
    __syncthreads();
    f32x4 acc[TR][4];
#pragma unroll
    for (int r = 0; r < TR; ++r)
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) acc[r][mb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the matrix-core phase at raised wave priority, as in k_conv_bf16r: the other
    // workgroup's epilogue and halo staging fill the matrix core's busy cycles (256 x 256
    // FP32 solve: 1429 -> 1407 ms)
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int st = 0; st < S; ++st) {
      const int tap = st / CG, c0 = (st % CG) * 16 + 4 * lk;
      const int dy = tap / 3, dx = tap % 3;
#pragma unroll
      for (int r = 0; r < TR; ++r)
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          const f32x4 a = *(const f32x4*)(s_in + ((r + dy) * HC + 16 * mb + li + dx) * CP + c0);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[r][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], wr[st][j], acc[r][mb], 0, 0, 0);
        }
      // keep each step's LDS reads beside its MFMAs: hoisting later steps' reads ahead
      // would hold more A fragments live than the registers beside the weights allow
      __builtin_amdgcn_sched_barrier(0);
    }
    __builtin_amdgcn_s_setprio(0);
    if constexpr (!LASTQ) {
#pragma unroll
      for (int r = 0; r < TR; ++r) {
        const int y = y0 + r;
        if (y >= n) continue;
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int x = x0 + 16 * mb + 4 * lk + q;
            if (x < m) out[(((size_t)i * n + y) * m + x) * COUT + o] = activate(acc[r][mb][q] + bo, act);
          }
      }
    } else {
      __syncthreads();  // every wave is done with the halo tile
      float* const s_h = s_in;  // activated tile [pixel][channel], pixel = r * 64 + x
#pragma unroll
      for (int r = 0; r < TR; ++r)
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            s_h[(r * TC + 16 * mb + 4 * lk + q) * HP + o] = activate(acc[r][mb][q] + bo, act);
      __syncthreads();
      // wave w: pixels 32w .. 32w+31 of the tile as two M-blocks, K = 64 channels in the
      // same 16-channel steps as above, N = the 9 taps (padded to 16)
      constexpr int MB2 = TR * TC / 64;  // M-blocks per wave
#pragma unroll
      for (int mb = 0; mb < MB2; ++mb) {
        const int pb = (w * MB2 + mb) * 16;
        f32x4 qa = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c0 = 0; c0 < COUT; c0 += 16) {
          const f32x4 a = *(const f32x4*)(s_h + (pb + li) * HP + c0 + 4 * lk);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            qa = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], s_wl[(c0 + 4 * lk + j) * 16 + li], qa, 0, 0, 0);
        }
        if (li < 9) {
          const long long plane = (long long)N * n * m;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int px = pb + 4 * lk + q;
            const int y = y0 + px / TC, x = x0 + px % TC;
            if (y < n && x < m) out[li * plane + ((long long)i * n + y) * m + x] = qa[q];
          }
        }
      }
    }
  }
}

// The last layer from the nine tap planes of k_conv_f32r<..., true>: out(y, x) = bias +
// the sum over the 3 x 3 taps of P_tap at (y + dy - 1, x + dx - 1), zero outside the
// field; writes the strided field and, with obs.Y, the X rows of Ybar (Eq. (12)).
__global__ __launch_bounds__(256) void k_conv_last_sum(int N, int n, int m, const float* __restrict__ q,
                                                       const float* __restrict__ bias, FieldOut fo,
                                                       ObserveArgs obs, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(q);
  OIC_GSH(bias);
  OIC_GSH(fo);
  OIC_GSH(obs);
  const long long plane = (long long)N * n * m;
  const int x = blockIdx.y * 256 + threadIdx.x;
  const int y = blockIdx.x % n, i = blockIdx.x / n;
  if (x >= m) return;
  float acc = bias ? bias[0] : 0.f;
#pragma unroll
  for (int dy = 0; dy < 3; ++dy) {
    const int yy = y + dy - 1;
    if (yy < 0 || yy >= n) continue;
    const float* row = q + ((long long)i * n + yy) * m;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      const int xx = x + dx - 1;
      if (xx >= 0 && xx < m) acc += row[(3 * dy + dx) * plane + xx];
    }
  }
  fo.base[i * fo.si + y * fo.sy + x] = acc;
  if (obs.Y) obs.Y[y * obs.NM + (long long)i * m + x] = acc + noise_value(obs.vx, y, i, x, m);
}

// The lift channel of the first layer as a field of its own: bu[i][y][x] = sum_a B[y][a]
// U_i[a][x], FP32 fused multiply-adds in ascending a from zero (the order k_conv_first
// uses when it forms the lift itself).  One thread per column, YB rows per block: the
// thread keeps its column of U in registers; the block's YB rows of B sit in LDS (zero
// past l), read as broadcasts.
template <int YB>
__global__ __launch_bounds__(256) void k_lift_bu(int N, int n, int m, int l, FieldRef U, const float* __restrict__ B,
                                                 float* __restrict__ bu, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(U);
  OIC_GSH(B);
  OIC_GSH(bu);
  constexpr int LMAX = 64;
  __shared__ __attribute__((aligned(16))) float s_b[YB][LMAX];
  const int yblocks = (n + YB - 1) / YB;
  const int i = blockIdx.x / yblocks, y0 = (blockIdx.x % yblocks) * YB;
  const int y1 = min(n, y0 + YB);
  for (int e = threadIdx.x; e < YB * LMAX; e += 256) {
    const int r = e / LMAX, a = e % LMAX;
    s_b[r][a] = (y0 + r < y1 && a < l) ? B[(size_t)(y0 + r) * l + a] : 0.f;
  }
  __syncthreads();
  const int x = blockIdx.y * 256 + threadIdx.x;
  if (x >= m) return;
  // the column of U: every load issued before the first use (the address stops at row
  // l - 1, whose value the rows past l repeat unused)
  float u[LMAX];
  const float* up = U.base + i * U.si + x;
#pragma unroll
  for (int a = 0; a < LMAX; ++a) {
    u[a] = *up;
    if (a + 1 < l) up += U.sy;
  }
  for (int y = y0; y < y1; ++y) {
    const float* brow = s_b[y - y0];
    float acc = 0.f;
#pragma unroll
    for (int a = 0; a < LMAX; a += 4) {
      const f32x4 b4 = *(const f32x4*)(brow + a);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (a + q < l) acc = fmaf(b4[q], u[a + q], acc);
    }
    bu[((size_t)i * n + y) * m + x] = acc;
  }
}

// First layer with the lift fused: the block stages the 6 x 66 halo of X, the l rows
// of U over the same columns and the 6 rows of B in LDS (all loads issued before the
// stores), forms B U per halo cell from LDS, computes 4 x 64 output pixels x COUT
// channels on the matrix cores (K = 2 channels x 9 taps, padded to 20), and writes the
// NHWC rows out through LDS so that the global stores are contiguous.  With 64 output
// channels the lift comes precomputed (bu_in, from k_lift_bu) and its 6 x 66 halo is
// staged like X's: the block then loads neither U nor B, its LDS shrinks from 27 to 8.5
// KiB and, held to 128 registers, four workgroups share a CU instead of three (at
// 256 x 256, N = 512: 2.91 -> 2.15 ms per launch in FP32, plus 0.15 ms for the lift).
template <int COUT, typename TOUT>
__global__ __launch_bounds__(256, COUT >= 64 ? 4 : 1) void k_conv_first(int N, int n, int m, int l, FieldRef X,
                                                    FieldRef U, const float* __restrict__ B,
                                                    const float* __restrict__ w,
                                                    const float* __restrict__ bias, int act,
                                                    TOUT* __restrict__ out, unsigned* __restrict__ amax,
                                                    ObserveArgs obs, const float* __restrict__ bu_in, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(X);
  OIC_GSH(U);
  OIC_GSH(B);
  OIC_GSH(w);
  OIC_GSH(bias);
  OIC_GSH(out);
  OIC_GSH(amax);
  OIC_GSH(obs);
  OIC_GSH(bu_in);
  constexpr int TR = 4, TC = 64, HR = TR + 2, HC = TC + 2;
  constexpr int LMAX = 64;
  constexpr bool BUF = COUT >= 64;  // the lift precomputed
  __shared__ float s_x[HR * HC];
  __shared__ float s_bu[HR * HC];
  __shared__ float s_u[BUF ? 1 : LMAX * HC];
  __shared__ float s_b[BUF ? 1 : HR * LMAX];
  __shared__ float s_w[20 * COUT];  // [k = channel*9 + tap, zero-padded to 20][o]
  __shared__ float s_bias[COUT];
  // BF16 output with up to 32 channels leaves as 16-byte stores, so each pixel's channels
  // stay 16-byte aligned in LDS; FP32 output and 64 channels keep the odd stride and
  // scalar stores (measured faster there: 128x128 C=32 3.2 -> 2.7 ms per solve with
  // vectors, 256x256 C=64 141 -> 171 ms)
  constexpr bool VEC = sizeof(TOUT) == 2 && COUT <= 32;
  constexpr int OPAD = VEC ? COUT + 4 : COUT + 1;
  // 64 output channels leave straight from the accumulators (each 16-lane group stores
  // one pixel's 16 consecutive channels): without the output tile the LDS holds five
  // workgroups per CU instead of one
  constexpr bool DIRECT = COUT >= 64;
  __shared__ __attribute__((aligned(16))) float s_out[DIRECT ? 1 : TR * TC * OPAD];
  const int col_tiles = (m + TC - 1) / TC;
  const int row_tiles = (n + TR - 1) / TR;
  int bid = blockIdx.x;
  const int ct = bid % col_tiles;
  bid /= col_tiles;
  const int rt = bid % row_tiles;
  const int i = bid / row_tiles;
  const int y0 = rt * TR, x0 = ct * TC;
  const int tid = threadIdx.x;
  const int a0 = (rt * l) / row_tiles, a1 = ((rt + 1) * l) / row_tiles;
  const int ne = obs.U_cur ? (a1 - a0) * TC : 0;
  float pw = 0.f, pv = 0.f;
  {
    // X halo: 396 cells; U rows: l x 66; B rows: 6 x l  (l <= 64); or the lift's halo
    constexpr int XS = (HR * HC + 255) / 256;
    constexpr int US = BUF ? 1 : (LMAX * HC + 255) / 256;
    float xv[XS], uv[US], bv[2], qv[XS];
#pragma unroll
    for (int u = 0; u < XS; ++u) {
      const int e = tid + 256 * u;
      const int yy = e / HC, xx = e % HC;
      const int gy = y0 + yy - 1, gx = x0 + xx - 1;
      const bool in = e < HR * HC && gy >= 0 && gy < n && gx >= 0 && gx < m;
      xv[u] = in ? X.base[i * X.si + gy * X.sy + gx] : 0.f;
      if constexpr (BUF) qv[u] = in ? bu_in[((size_t)i * n + gy) * m + gx] : 0.f;
    }
    if constexpr (!BUF) {
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
    }
    constexpr int WS = (20 * COUT + 255) / 256;
    float wv[WS];
#pragma unroll
    for (int u = 0; u < WS; ++u) {
      const int e = tid + 256 * u;
      const int kk = e / COUT, o = e % COUT;
      wv[u] = (e < 20 * COUT && kk < 18) ? w[o * 18 + kk] : 0.f;
    }
    const float bias_v = (tid < COUT && bias) ? bias[tid] : 0.f;
    // the first noise pairs of the U rows, requested after the halo loads so that their
    // latency overlaps (each noise value waits for its own loads)
    if (tid < ne && x0 + tid % TC < m) {
      const int a = a0 + tid / TC, x = x0 + tid % TC;
      if (obs.w.diag && obs.vu.diag) {  // diagonal covariances: four loads, one wait
        const float dw = obs.w.diag[a], dv = obs.vu.diag[a];
        const float zw = obs.w.Z[((size_t)i * obs.w.rows + a) * m + x];
        const float zv = obs.vu.Z[((size_t)i * obs.vu.rows + a) * m + x];
        pw = dw * zw;
        pv = dv * zv;
      } else {
        pw = noise_value(obs.w, a, i, x, m);
        pv = noise_value(obs.vu, a, i, x, m);
      }
    }
#pragma unroll
    for (int u = 0; u < WS; ++u)
      if (tid + 256 * u < 20 * COUT) s_w[tid + 256 * u] = wv[u];
    if (tid < COUT) s_bias[tid] = bias_v;
#pragma unroll
    for (int u = 0; u < XS; ++u)
      if (tid + 256 * u < HR * HC) {
        s_x[tid + 256 * u] = xv[u];
        if constexpr (BUF) s_bu[tid + 256 * u] = qv[u];
      }
    if constexpr (!BUF) {
#pragma unroll
      for (int u = 0; u < US; ++u)
        if (tid + 256 * u < LMAX * HC) s_u[tid + 256 * u] = uv[u];
#pragma unroll
      for (int u = 0; u < 2; ++u)
        if (tid + 256 * u < HR * LMAX) s_b[tid + 256 * u] = bv[u];
    }
  }
  __syncthreads();
  if constexpr (!BUF) {
    for (int e = tid; e < HR * HC; e += 256) {
      const int yy = e / HC, xx = e % HC;
      float bu = 0.f;
      for (int a = 0; a < l; ++a) bu = fmaf(s_b[yy * LMAX + a], s_u[a * HC + xx], bu);
      s_bu[e] = bu;
    }
  }
  // the U rows of the new slice and their observations: the l rows of this column tile
  // are shared out over its row tiles; the first 256 noise pairs were requested with the halo
  for (int e = tid; e < ne; e += 256) {
    const int a = a0 + e / TC, xx = e % TC, x = x0 + xx;
    if (x < m) {
      const long long col = (long long)i * m + x;
      const float uprev = BUF ? U.base[i * U.si + a * U.sy + x] : s_u[a * HC + xx + 1];
      const float u = uprev + (e < 256 ? pw : noise_value(obs.w, a, i, x, m));
      obs.U_cur[a * obs.NM + col] = u;
      obs.Y[(n + a) * obs.NM + col] = u + (e < 256 ? pv : noise_value(obs.vu, a, i, x, m));
    }
  }
  __syncthreads();
  // 256 pixels x COUT channels x K = 18 (two channels x 9 taps, padded to 20) on the
  // matrix cores: wave w owns pixel blocks 4w..4w+3 (16 pixels each, one output row)
  {
    constexpr int NB = (COUT + 15) / 16;  // COUT = 8 uses half of one N-block
    const int lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    f32x4 acc[4][NB];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the matrix-core phase at raised wave priority, as in k_conv_f32r (256 x 256 FP32
    // solve: 1410.4 -> 1408.1 ms)
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int kb = 0; kb < 5; ++kb) {
      const int kq = kb * 4 + lk;
      const int kk = kq < 18 ? kq : 0;  // past 18 the weights are zero
      const float* src = kk < 9 ? s_x : s_bu;
      const int tap = kk % 9;
      const int off = (tap / 3) * HC + tap % 3;
      float b[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int o = DIRECT ? NB * li + nb : nb * 16 + li;  // DIRECT: a lane holds NB adjacent channels
        b[nb] = o < COUT ? s_w[kq * COUT + o] : 0.f;
      }
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        const int px = (4 * w + mb) * 16 + li;  // pixel (px / 64, px % 64) of the tile
        const float a = src[(px / TC) * HC + px % TC + off];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[nb], acc[mb][nb], 0, 0, 0);
      }
    }
    __builtin_amdgcn_s_setprio(0);
    if constexpr (DIRECT) {
      // wave w owns output row w of the tile; lane (li, lk) holds channels NB li .. NB li + NB-1
      // of pixels 16 mb + 4 lk + r and stores them as one vector (16 B FP32, 8 B BF16)
      static_assert(NB == 4, "four adjacent channels per lane");
      const int y = y0 + w;
      float vmax = 0.f;
      if (y < n) {
        float bo[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) bo[nb] = s_bias[NB * li + nb];
        TOUT* const orow = out + (((size_t)i * n + y) * m + x0) * COUT + NB * li;
        const bool full = x0 + TC <= m;
        with_activation(act, [&](auto actc) {
          constexpr int ACT = decltype(actc)::value;
#pragma unroll
          for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int px = mb * 16 + 4 * lk + r;
              if (full || x0 + px < m) {
                float v[NB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                  v[nb] = sizeof(TOUT) == 2 ? activate_lp_c<ACT>(acc[mb][nb][r] + bo[nb])
                                            : activate_c<ACT>(acc[mb][nb][r] + bo[nb]);
                  vmax = fmaxf(vmax, fabsf(v[nb]));
                }
                if constexpr (sizeof(TOUT) == 2)
                  *reinterpret_cast<u32x2*>(orow + (size_t)px * COUT) = u32x2{pack_bf16x2(v[0], v[1]),
                                                                              pack_bf16x2(v[2], v[3])};
                else
                  *reinterpret_cast<f32x4*>(orow + (size_t)px * COUT) = f32x4{v[0], v[1], v[2], v[3]};
              }
            }
        });
      }
      if (amax) amax_publish(vmax, amax);
      return;
    }
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int o = nb * 16 + li;
        if (o >= COUT) continue;
        const float bo = s_bias[o];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int px = (4 * w + mb) * 16 + 4 * lk + r;
          s_out[px * OPAD + o] = sizeof(TOUT) == 2 ? activate_lp(acc[mb][nb][r] + bo, act)
                                                   : activate(acc[mb][nb][r] + bo, act);
        }
      }
  }
  __syncthreads();
  constexpr int V = VEC ? 8 : 1;  // channels per store
  static_assert(COUT % V == 0, "a pixel's channels split into whole 16-byte vectors");
  float vmax = 0.f;
  for (int r = 0; r < TR; ++r) {
    const int y = y0 + r;
    if (y >= n) break;
    const int valid = min(TC, m - x0);
    TOUT* dst = out + (((size_t)i * n + y) * m + x0) * COUT;
    if constexpr (!VEC) {
      for (int e = tid; e < valid * COUT; e += 256) {
        const float v = s_out[(r * TC + e / COUT) * OPAD + e % COUT];
        store_act(dst + e, v);
        vmax = fmaxf(vmax, fabsf(v));
      }
    } else {
      for (int e = tid; e < valid * COUT / V; e += 256) {
        const int px = (e * V) / COUT, o = (e * V) % COUT;
        const float* src = s_out + (r * TC + px) * OPAD + o;  // 16-byte aligned: OPAD, o multiples of 4
        float v[V];
#pragma unroll
        for (int q = 0; q < V; q += 4) {
          const f32x4 f = *(const f32x4*)(src + q);
          v[q] = f[0];
          v[q + 1] = f[1];
          v[q + 2] = f[2];
          v[q + 3] = f[3];
        }
#pragma unroll
        for (int q = 0; q < V; ++q) vmax = fmaxf(vmax, fabsf(v[q]));
        store_vec16(dst + e * V, v);
      }
    }
  }
  if (amax) amax_publish(vmax, amax);
}

// Last layer (one output channel) from an LDS halo tile of the NHWC input; each
// thread computes one pixel (9*CIN taps) and the store to the strided field is
// contiguous along x.
template <int CIN, typename TIN>
__global__ __launch_bounds__(256) void k_conv_last(int N, int n, int m, const TIN* __restrict__ in,
                                                   const float* __restrict__ w,
                                                   const float* __restrict__ bias, FieldOut fo,
                                                   ObserveArgs obs, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(in);
  OIC_GSH(w);
  OIC_GSH(bias);
  OIC_GSH(fo);
  OIC_GSH(obs);
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
  // weights [0][c][dy][dx] -> s_w[tap * CIN + c], requested before the halo
  constexpr int WS = (9 * CIN + 255) / 256;
  float wv[WS];
#pragma unroll
  for (int u = 0; u < WS; ++u) wv[u] = tid + 256 * u < 9 * CIN ? w[tid + 256 * u] : 0.f;
  stage_halo<CIN, HR, HC, CP, 256>(in, i, n, m, y0, x0, s_in);
#pragma unroll
  for (int u = 0; u < WS; ++u) {
    const int e = tid + 256 * u;
    if (e < 9 * CIN) s_w[(e % 9) * CIN + e / 9] = wv[u];
  }
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
  if (y < n && x < m) {
    fo.base[i * fo.si + y * fo.sy + x] = acc;
    if (obs.Y) obs.Y[y * obs.NM + (long long)i * m + x] = acc + noise_value(obs.vx, y, i, x, m);
  }
}

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// Folded last layer (64 -> 1) from an activated BF16 tile in LDS, s_out[pixel][channel]
// with pixel stride OP (pixel = tile row * TC + column): the nine per-tap partial sums
// P_tap(p) = sum_c wl[c][tap] h(p)[c] on the BF16 matrix cores, K = the COUT channels in
// steps of 32, N = the taps (padded to 16), the weights as a BF16 pair wl2 = [hi, lo]
// [16 taps][COUT]; the sums leave as nine FP32 planes qout[tap][i][y][x] (plane stride
// N n m).  The NT threads' waves take whole 16-pixel M-blocks of the tile.
template <int COUT, int TR, int TC, int OP, int NT>
__device__ __forceinline__ void fold_last_epilogue(const bf16_t* s_out, const bf16_t* __restrict__ wl2,
                                                   float* __restrict__ qout, int N, int n, int m, int i, int y0,
                                                   int x0, int tid) {
  static_assert(COUT % 32 == 0, "whole 32-channel K steps");
  constexpr int NWV = NT / 64;       // waves
  constexpr int MBT = TR * TC / 16;  // M-blocks of the tile
  static_assert(MBT % NWV == 0, "whole M-blocks per wave");
  const int wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const long long plane = (long long)N * n * m;
#pragma unroll
  for (int u = 0; u < MBT / NWV; ++u) {
    const int pb = (wave * (MBT / NWV) + u) * 16;
    f32x4 qa = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < COUT / 32; ++ks) {
      const bf16x8_t a = __builtin_bit_cast(bf16x8_t, *(const u16x8*)(s_out + (pb + li) * OP + 32 * ks + 8 * lk));
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2) {
        const bf16x8_t b =
            __builtin_bit_cast(bf16x8_t, *(const u16x8*)(wl2 + ((size_t)h2 * 16 + li) * COUT + 32 * ks + 8 * lk));
        qa = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, qa, 0, 0, 0);
      }
    }
    if (li < 9) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int px = pb + 4 * lk + r;
        const int y = y0 + px / TC, x = x0 + px % TC;
        if (y < n && x < m) qout[li * plane + ((long long)i * n + y) * m + x] = qa[r];
      }
    }
  }
}

// Hidden layer in BF16 on MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulation): the
// same tiling as the FP32 kernel, but each k-step covers 32 K-indices (tap, channel)
// and every lane supplies 8 consecutive channels of one tap for A and 8 consecutive
// K-indices of one output channel for B, each as one 16-byte LDS read.  Input and
// output activations are BF16 NHWC; the weights sit in LDS as [o][tap*CIN + c].
// Row strides in LDS are padded by 8 elements so the 16 lanes of a fragment hit
// distinct banks.  Lane layout (16x16x32): A[i][k] for k = 8g..8g+7 from lane i + 16g,
// B[k][j] for k = 8g..8g+7 from lane j + 16g, element r of lane j + 16g holds D[4g + r][j].
//
// LASTQ (64 output channels): the network's last layer (64 -> 1) is folded into the
// epilogue as in k_conv_f32r: from the activated BF16 tile in LDS, the nine per-tap partial
// sums P_tap(p) = sum_c wl[c][tap] h(p)[c] are formed on the BF16 matrix cores with the
// last layer's weights as a BF16 pair wl = hi + lo (wl2[0] and wl2[1], [tap padded to
// 16][c], exact to about 16 bits) and leave as nine FP32 planes (out, plane stride N n m)
// for k_conv_last_sum.
template <int CIN, int COUT, int TR, int WG, bool LASTQ = false>
__global__ __launch_bounds__(256 * WG) void k_conv_mfma_bf16(int N, int n, int m,
                                                        const bf16_t* __restrict__ in,
                                                        const bf16_t* __restrict__ wt,
                                                        const float* __restrict__ bias, int act,
                                                        bf16_t* __restrict__ out,
                                                        const bf16_t* __restrict__ wl2, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(in);
  OIC_GSH(wt);
  OIC_GSH(bias);
  OIC_GSH(out);
  OIC_GSH(wl2);
  constexpr int TC = 64;
  constexpr int HR = TR + 2, HC = TC + 2;
  constexpr int CP = CIN + 8;
  constexpr int KD = 9 * CIN;
  constexpr int KD32 = (KD + 31) / 32 * 32;  // K rounded up to whole k-steps (zero weights past KD)
  constexpr int KDP = KD32 + 8;
  constexpr int NB = COUT / 16;
  constexpr int RPW = TR / 4;
  constexpr int OP = COUT + 8;
  constexpr int IQ = CIN / 8;
  constexpr int IV = HR * HC * IQ;
  constexpr int NT = 256 * WG;       // WG groups of 4 waves split the output channels
  constexpr int NBW = NB / WG;       // N-blocks per wave
  static_assert(NB % WG == 0, "whole N-blocks per wave group");
  constexpr int IS = (IV + NT - 1) / NT;
  // the weights stay resident; the halo tile and, after the MFMA loop, the output tile
  // share the rest
  constexpr int TILE = HR * HC * CP > TR * TC * OP ? HR * HC * CP : TR * TC * OP;
  __shared__ __attribute__((aligned(16))) bf16_t s_w[COUT * KDP];
  __shared__ __attribute__((aligned(16))) bf16_t s_tile[TILE];
  bf16_t* const s_in = s_tile;
  bf16_t* const s_out = s_tile;
  const int col_tiles = (m + TC - 1) / TC;
  const int row_tiles = (n + TR - 1) / TR;
  const int tiles = N * row_tiles * col_tiles;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = (tid >> 6) & 3, ng = tid >> 8;
  const int li = lane & 15, lk = lane >> 4;
  {
    constexpr int WQ = KD / 8;  // 16-byte vectors per weight row
    constexpr int WV = COUT * WQ;
    constexpr int WS = (WV + NT - 1) / NT;
#pragma unroll
    for (int u = 0; u < WS; ++u) {
      const int e = tid + NT * u;
      if (e < WV) *(u16x8*)(s_w + (e / WQ) * KDP + 8 * (e % WQ)) = *(const u16x8*)(wt + (size_t)8 * e);
    }
    if (KD32 > KD) {  // zero the K padding of every weight row
      constexpr int PQ = (KD32 - KD) / 8;
      for (int e = tid; e < COUT * PQ; e += NT)
        *(u16x8*)(s_w + (e / PQ) * KDP + KD + 8 * (e % PQ)) = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
    }
  }
  // Persistent over tiles tile, tile + gridDim.x, ...: the next tile's halo is loaded
  // into registers while the current one is on the matrix cores.
  u16x8 iv[IS];
  auto load_halo = [&](int tile) {
    const int ct = tile % col_tiles, rest = tile / col_tiles;
    const int rt = rest % row_tiles, i = rest / row_tiles;
    const int y0 = rt * TR, x0 = ct * TC;
#pragma unroll
    for (int u = 0; u < IS; ++u) {
      const int e = tid + NT * u;
      iv[u] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      if (e < IV) {
        const int q = e % IQ, pix = e / IQ;
        const int xx = pix % HC, yy = pix / HC;
        const int gy = y0 + yy - 1, gx = x0 + xx - 1;
        if (gy >= 0 && gy < n && gx >= 0 && gx < m)
          iv[u] = *(const u16x8*)(in + (((size_t)i * n + gy) * m + gx) * CIN + 8 * q);
      }
    }
  };
  int tile = blockIdx.x;
  if (tile < tiles) load_halo(tile);
  for (; tile < tiles; tile += gridDim.x) {
    const int ct = tile % col_tiles, rest = tile / col_tiles;
    const int rt = rest % row_tiles, i = rest / row_tiles;
    const int y0 = rt * TR, x0 = ct * TC;
    __syncthreads();  // the previous tile's output has left s_tile (and s_w is staged)
#pragma unroll
    for (int u = 0; u < IS; ++u) {
      const int e = tid + NT * u;
      if (e < IV) *(u16x8*)(s_in + (e / IQ) * CP + 8 * (e % IQ)) = iv[u];
    }
    __syncthreads();
    if (tile + (int)gridDim.x < tiles) load_halo(tile + gridDim.x);  // in flight meanwhile
    f32x4 acc[RPW][4][NBW];
#pragma unroll
    for (int rw = 0; rw < RPW; ++rw)
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb) acc[rw][mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 3
    for (int kb = 0; kb < KD32 / 32; ++kb) {
      const int k0 = kb * 32 + 8 * lk;
      // past KD the weights are zero; read any in-tile (finite) activations there
      const int kk = k0 < KD ? k0 : 0;
      const int tap = kk / CIN, c0 = kk - tap * CIN;
      const int dy = tap / 3, dx = tap - dy * 3;
      bf16x8_t b[NBW];
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb)
        b[nb] = __builtin_bit_cast(bf16x8_t, *(const u16x8*)(s_w + ((ng * NBW + nb) * 16 + li) * KDP + k0));
#pragma unroll
      for (int rw = 0; rw < RPW; ++rw) {
        const int ry = w + 4 * rw;
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          const bf16x8_t a = __builtin_bit_cast(
              bf16x8_t, *(const u16x8*)(s_in + ((ry + dy) * HC + mb * 16 + li + dx) * CP + c0));
#pragma unroll
          for (int nb = 0; nb < NBW; ++nb)
            acc[rw][mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[nb], acc[rw][mb][nb], 0, 0, 0);
        }
      }
    }
    // Epilogue through LDS: every lane writes its activated outputs into the tile
    // [pixel][channel] (BF16, rows padded by 8), then the tile leaves as 16-byte rows
    // of 8 channels, so the NHWC stores are full vector stores instead of 2-byte ones.
    __syncthreads();  // every wave is done with the halo tile
#pragma unroll
    for (int rw = 0; rw < RPW; ++rw) {
      const int ty = w + 4 * rw;
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb) {
          const int o = (ng * NBW + nb) * 16 + li;
          const float bo = bias ? bias[o] : 0.f;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int tx = mb * 16 + 4 * lk + r;
            s_out[(ty * TC + tx) * OP + o] = to_bf16(activate_lp(acc[rw][mb][nb][r] + bo, act));
          }
        }
    }
    __syncthreads();
    if constexpr (!LASTQ) {
      constexpr int QV = COUT / 8;  // 16-byte vectors per pixel
      for (int e = tid; e < TR * TC * QV; e += NT) {
        const int px = e / QV, q = e - px * QV;
        const int y = y0 + px / TC, x = x0 + px % TC;
        if (y < n && x < m)
          *(u16x8*)(out + (((size_t)i * n + y) * m + x) * COUT + 8 * q) = *(const u16x8*)(s_out + px * OP + 8 * q);
      }
    } else {
      fold_last_epilogue<COUT, TR, TC, OP, NT>(s_out, wl2, reinterpret_cast<float*>(out), N, n, m, i, y0, x0, tid);
    }
  }
}

// Hidden layer in BF16 with the weights held in registers (cin 32 or 64 -> cout 32 or 64),
// the BF16 counterpart of k_conv_f32r: each wave owns 32 output channels (two N-blocks)
// for TR/RG rows of a TR x 64 tile (RG = 4 waves / (cout / 32) channel groups), holds its
// B fragments for all K = 9 cin indices (8 consecutive channels of one tap per lane and
// k-step of 32), so the LDS holds only the BF16 halo tile and every 16-byte A fragment
// read feeds two MFMAs (v_mfma_f32_16x16x32_bf16).  The halo arrives by LDS-direct buffer
// loads (16-byte slots, one padding slot per pixel, out-of-field slots zero-filled by the
// buffer bounds); two persistent workgroups per CU walk the tiles in the XCD-aware order.
// LASTQ (cout 64): the network's last layer is folded into the epilogue
// (fold_last_epilogue); otherwise the BF16 outputs leave straight from the accumulators.
// Lane layout (16x16x32): A[i][k] for k = 8g..8g+7 from lane i + 16g, B[k][j] likewise
// from lane j + 16g, element r of lane j + 16g holds D[4g + r][j].
// GROUPED: the instance for grouped launches (the plain one leaves the group argument
// alone, so that its code is exactly the single-solve kernel's).
template <int CIN, int COUT, int TR, bool LASTQ, bool GROUPED>
__global__ __launch_bounds__(256, 2) void k_conv_bf16r(int N, int n, int m, const bf16_t* __restrict__ in,
                                                       const bf16_t* __restrict__ wt,
                                                       const float* __restrict__ bias, int act,
                                                       bf16_t* __restrict__ out, const bf16_t* __restrict__ wl2,
                                                       Grp grp) {
  if constexpr (GROUPED) {
    OIC_GROUP_ENTER(grp);
    OIC_GSH(in);
    OIC_GSH(wt);
    OIC_GSH(bias);
    OIC_GSH(out);
    OIC_GSH(wl2);
  }
  static_assert(CIN % 32 == 0 && COUT % 32 == 0, "32-channel K steps and channel groups");
  constexpr int TC = 64, HR = TR + 2, HC = TC + 2;
  constexpr int NG = COUT / 32;          // channel groups (one per wave of a row group)
  constexpr int RG = 4 / NG;             // row groups
  static_assert(TR % RG == 0, "whole rows per wave");
  constexpr int RW = TR / RG;            // rows per wave
  constexpr int CPB = CIN + 8;           // pixel stride in LDS (bf16): CIN / 8 data slots + 1 padding slot
  constexpr int SLOT = CPB / 8;
  constexpr int TOTAL_SLOTS = HR * HC * SLOT;
  constexpr int INSTR = (TOTAL_SLOTS + 63) / 64;
  constexpr int SPW = (INSTR + 3) / 4;   // halo load instructions per wave (at most)
  constexpr int KS = 9 * CIN / 32;       // k-steps
  constexpr int CG = CIN / 32;           // k-steps per tap
  constexpr int OP = COUT + 8;           // pixel stride of the activated tile (LASTQ)
  static_assert(!LASTQ || TR * TC * OP <= INSTR * 64 * 8, "the activated tile reuses the halo's LDS");
  __shared__ __attribute__((aligned(16))) bf16_t s_in[INSTR * 64 * 8];
  const int col_tiles = (m + TC - 1) / TC;
  const int row_tiles = (n + TR - 1) / TR;
  const int tiles = N * row_tiles * col_tiles;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ng = w % NG, rg = w / NG;
  // Output channel of column li in N-block nb: 32 ng + 2 li + nb, so that a lane holds two
  // adjacent channels of each of its pixels and stores them as one 32-bit word.
  // This lane's weights: k-step ks, N-block nb -> W[32 ng + 2 li + nb][32 ks + 8 lk .. +7].
  bf16x8_t wr[KS][2];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
      wr[ks][nb] = __builtin_bit_cast(
          bf16x8_t, *(const u16x8*)(wt + (size_t)(32 * ng + 2 * li + nb) * (9 * CIN) + 32 * ks + 8 * lk));
  float bo[2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) bo[nb] = bias ? bias[32 * ng + 2 * li + nb] : 0.f;
  // The halo slots this lane loads, fixed for every tile: byte offset from the tile's
  // origin pixel and column offset (-1..64); slots past the halo or on a padding slot get
  // a column offset that fails the column test.  Rows above or below the field need no
  // test: their offsets fall outside the member's buffer range, whose loads return zeros.
  // With the last layer folded in (LASTQ), or more than ten loads per lane, the registers
  // are needed elsewhere: the offsets are then recomputed for every tile.
  constexpr bool PRE = !LASTQ && SPW <= 10;
  auto slot_offsets = [&](int u, unsigned& rel, int& gxo) {
    int slot = (w + 4 * u) * 64 + lane;
    if constexpr (!PRE) asm volatile("" : "+v"(slot));  // keep the recomputation in the tile loop
    const int pix = slot / SLOT, q = slot - pix * SLOT;
    const int yy = pix / HC, xx = pix - yy * HC;
    const bool valid = w + 4 * u < INSTR && slot < TOTAL_SLOTS && q < CIN / 8;
    // modulo 2^32 (negative for the row above the tile)
    rel = ((unsigned)((yy - 1) * m + (xx - 1)) * CIN + 8u * q) * 2u;
    gxo = valid ? xx - 1 : -(1 << 24);
  };
  unsigned rel[SPW];
  int gxo[SPW];
  if constexpr (PRE)
#pragma unroll
    for (int u = 0; u < SPW; ++u) slot_offsets(u, rel[u], gxo[u]);
  const TileWalk walk(tiles);
  const unsigned nrec = (unsigned)n * m * CIN * 2;
  // LDS-direct loads of tile tl's (TR+2) x 66 x CIN halo into s_in; the caller has made sure
  // no wave still reads s_in
  auto issue_halo = [&](int tl) {
    const int ct = tl % col_tiles, rest = tl / col_tiles;
    const int rt = rest % row_tiles, i = rest / row_tiles;
    const int y0 = rt * TR, x0 = ct * TC;
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void*)(in + (size_t)i * n * m * CIN), (short)0, (int)nrec, 0x00020000);
    const unsigned tb = (unsigned)(y0 * m + x0) * CIN * 2;
#pragma unroll
    for (int u = 0; u < SPW; ++u) {
      const int ins = w + 4 * u;  // wave-uniform
      if (ins < INSTR) {
        if constexpr (!PRE) slot_offsets(u, rel[u], gxo[u]);
        // modulo 2^32: a row above the field wraps to a huge offset, one below lands past nrec
        const unsigned voff = (unsigned)(x0 + gxo[u]) < (unsigned)m ? tb + rel[u] : nrec;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (__attribute__((address_space(3))) void*)(s_in + ins * 512),
                                                 16, (int)voff, 0, 0, 0);
      }
    }
  };
  if (walk.first < walk.end) issue_halo(walk.first);
  for (int tile = walk.first; tile < walk.end; tile += walk.step) {
    const int ct = tile % col_tiles, rest = tile / col_tiles;
    const int rt = rest % row_tiles, i = rest / row_tiles;
    const int y0 = rt * TR, x0 = ct * TC;
    const int next = tile + walk.step;
    __builtin_amdgcn_s_waitcnt(0);  // this tile's LDS-direct loads have landed (vmcnt)
    __syncthreads();
    f32x4 acc[RW][4][2];  // start from the bias
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) acc[r][mb][nb] = f32x4{bo[nb], bo[nb], bo[nb], bo[nb]};
    // the matrix-core phase at raised wave priority: where the SIMD's other wave (of the
    // other workgroup on the CU) is in its epilogue, this wave's MFMAs issue first and the
    // epilogue's VALU work fills the matrix core's busy cycles (256 x 256 BF16 solve:
    // 317.3 -> 316.2 ms)
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int tap = ks / CG, c0 = (ks % CG) * 32 + 8 * lk;
      const int dy = tap / 3, dx = tap % 3;
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        const int ry = rg * RW + r;
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          const bf16x8_t a =
              __builtin_bit_cast(bf16x8_t, *(const u16x8*)(s_in + ((ry + dy) * HC + 16 * mb + li + dx) * CPB + c0));
#pragma unroll
          for (int nb = 0; nb < 2; ++nb)
            acc[r][mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wr[ks][nb], acc[r][mb][nb], 0, 0, 0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);  // one step's fragments live at a time
    }
    __builtin_amdgcn_s_setprio(0);
    if constexpr (!LASTQ) {
      // the next tile's halo lands while this tile's epilogue (no LDS) runs
      __syncthreads();  // every wave is done reading the halo
      if (next < walk.end) issue_halo(next);
      with_activation(act, [&](auto actc) {
        constexpr int ACT = decltype(actc)::value;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
          const int y = y0 + rg * RW + r;
          if (y >= n) continue;
          unsigned* const orow =
              reinterpret_cast<unsigned*>(out + (((size_t)i * n + y) * m + x0) * COUT + 32 * ng + 2 * li);
          if (x0 + TC <= m) {
#pragma unroll
            for (int mb = 0; mb < 4; ++mb)
#pragma unroll
              for (int q = 0; q < 4; ++q)
                orow[(16 * mb + 4 * lk + q) * (COUT / 2)] = pack_bf16x2(
                    activate_lp_c<ACT>(acc[r][mb][0][q]), activate_lp_c<ACT>(acc[r][mb][1][q]));
          } else {
#pragma unroll
            for (int mb = 0; mb < 4; ++mb)
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int px = 16 * mb + 4 * lk + q;
                if (x0 + px < m)
                  orow[px * (COUT / 2)] = pack_bf16x2(activate_lp_c<ACT>(acc[r][mb][0][q]),
                                                      activate_lp_c<ACT>(acc[r][mb][1][q]));
              }
          }
        }
      });
    } else {
      __syncthreads();  // every wave is done with the halo tile
      bf16_t* const s_out = s_in;
      with_activation(act, [&](auto actc) {
        constexpr int ACT = decltype(actc)::value;
#pragma unroll
        for (int r = 0; r < RW; ++r)
#pragma unroll
          for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              *reinterpret_cast<unsigned*>(s_out + ((rg * RW + r) * TC + 16 * mb + 4 * lk + q) * OP + 32 * ng +
                                           2 * li) =
                  pack_bf16x2(activate_lp_c<ACT>(acc[r][mb][0][q]), activate_lp_c<ACT>(acc[r][mb][1][q]));
      });
      __syncthreads();
      fold_last_epilogue<COUT, TR, TC, OP, 256>(s_out, wl2, reinterpret_cast<float*>(out), N, n, m, i, y0, x0, tid);
      __syncthreads();  // every wave is done with the activated tile
      if (next < walk.end) issue_halo(next);
    }
  }
}

// Hidden layer in FP8 (OCP e4m3) on the gfx950 matrix cores
// (v_mfma_scale_f32_16x16x128_f8f6f4 with unit block scales, FP32 accumulation).
// Weights arrive quantised per output channel, wq[o][k] = W[o][k] / ws[o], with K
// ordered (tap, channel) and zero-padded to a multiple of 128.  The BF16 input
// activations are quantised while the halo tile is staged, x / sa with sa = (largest
// |x| of the layer over the whole ensemble) / 448, that maximum having been folded in
// by the kernel that wrote them.  The epilogue rescales by sa * ws[o], adds the bias,
// applies the activation, stores BF16 and folds its own maximum into amax_out.
// Lane layout (16x16x128): A[i][k] for k = 32g..32g+31 from lane i + 16g (bytes in
// k order), B[k][j] likewise from lane j + 16g, element r of lane j + 16g holds
// D[4g + r][j].  CIN is a multiple of 32, so the 32 K-indices of a lane are 32
// consecutive channels of one tap.
//
// LASTQ (64 output channels): the network's last layer is folded into the epilogue as in
// the BF16 kernel (fold_last_epilogue): out then receives nine FP32 tap planes and no
// maximum is published (no FP8 layer follows).
template <int CIN, int COUT, int TR, int WG, bool LASTQ = false>
__global__ __launch_bounds__(256 * WG) void k_conv_mfma_fp8(int N, int n, int m,
                                                            const bf16_t* __restrict__ in,
                                                            const unsigned* __restrict__ amax_in,
                                                            const uint8_t* __restrict__ wq,
                                                            const float* __restrict__ ws,
                                                            const float* __restrict__ bias, int act,
                                                            bf16_t* __restrict__ out,
                                                            unsigned* __restrict__ amax_out,
                                                            const bf16_t* __restrict__ wl2) {
  static_assert(CIN % 32 == 0, "32 channels per lane fragment");
  constexpr int TC = 64;
  constexpr int HR = TR + 2, HC = TC + 2;
  constexpr int CP = CIN + 16;                      // bytes per halo pixel in LDS
  constexpr int KD = 9 * CIN;
  constexpr int KD128 = (KD + 127) / 128 * 128;      // zero weights past KD
  constexpr int KDP = KD128 + 16;
  constexpr int NB = COUT / 16;
  constexpr int RPW = TR / 4;
  constexpr int NT = 256 * WG;  // WG groups of 4 waves split the output channels
  constexpr int NBW = NB / WG;
  static_assert(NB % WG == 0, "whole N-blocks per wave group");
  constexpr int OP = COUT + 8;
  constexpr int IQ = CIN / 8;
  constexpr int IV = HR * HC * IQ;
  constexpr int IS = (IV + NT - 1) / NT;
  // the weights stay resident; the FP8 halo tile and, after the MFMA loop, the BF16
  // output tile share the rest
  constexpr int LDS_IN = HR * HC * CP, LDS_OUT = TR * TC * OP * 2;
  __shared__ __attribute__((aligned(16))) uint8_t s_w[COUT * KDP];
  __shared__ __attribute__((aligned(16))) uint8_t s_tile[LDS_IN > LDS_OUT ? LDS_IN : LDS_OUT];
  uint8_t* const s_in = s_tile;
  bf16_t* const s_out = reinterpret_cast<bf16_t*>(s_tile);
  const int col_tiles = (m + TC - 1) / TC;
  const int row_tiles = (n + TR - 1) / TR;
  const int tiles = N * row_tiles * col_tiles;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = (tid >> 6) & 3, ng = tid >> 8;
  const int li = lane & 15, lk = lane >> 4;
  const float amx = amax_read(amax_in);
  const float sa = amx > 0.f ? amx * (1.0f / 448.0f) : 1.0f;
  const float inv_sa = 1.0f / sa;
  {
    constexpr int WQ = KD128 / 16;  // 16-byte vectors per weight row
    constexpr int WV = COUT * WQ;
    constexpr int WS = (WV + NT - 1) / NT;
#pragma unroll
    for (int u = 0; u < WS; ++u) {
      const int e = tid + NT * u;
      if (e < WV) *(u32x4*)(s_w + (e / WQ) * KDP + 16 * (e % WQ)) = *(const u32x4*)(wq + (size_t)16 * e);
    }
  }
  // Persistent over tiles tile, tile + gridDim.x, ...: the next tile's BF16 halo is loaded
  // into registers while the current one is on the matrix cores.
  u16x8 iv[IS];
  auto load_halo = [&](int tile) {
    const int ct = tile % col_tiles, rest = tile / col_tiles;
    const int rt = rest % row_tiles, i = rest / row_tiles;
    const int y0 = rt * TR, x0 = ct * TC;
#pragma unroll
    for (int u = 0; u < IS; ++u) {
      const int e = tid + NT * u;
      iv[u] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      if (e < IV) {
        const int q = e % IQ, pix = e / IQ;
        const int xx = pix % HC, yy = pix / HC;
        const int gy = y0 + yy - 1, gx = x0 + xx - 1;
        if (gy >= 0 && gy < n && gx >= 0 && gx < m)
          iv[u] = *(const u16x8*)(in + (((size_t)i * n + gy) * m + gx) * CIN + 8 * q);
      }
    }
  };
  // Output channel of column li in N-block nb: with an even number of N-blocks per wave they
  // pair up (nb = 2h, 2h + 1) so that a lane holds two adjacent channels, 32 h + 2 li and
  // + 1, of each of its pixels (one 4-byte LDS write); otherwise 16 nb + li.
  constexpr bool PAIR = NBW % 2 == 0;
  auto out_channel = [&](int nb) {
    return PAIR ? ng * NBW * 16 + 32 * (nb >> 1) + 2 * li + (nb & 1) : (ng * NBW + nb) * 16 + li;
  };
  float vmax = 0.f;
  int tile = blockIdx.x;
  if (tile < tiles) load_halo(tile);
  for (; tile < tiles; tile += gridDim.x) {
    const int ct = tile % col_tiles, rest = tile / col_tiles;
    const int rt = rest % row_tiles, i = rest / row_tiles;
    const int y0 = rt * TR, x0 = ct * TC;
    __syncthreads();  // the previous tile's output has left s_tile (and s_w is staged)
    // quantise the halo to e4m3 (x / sa) on its way into LDS
#pragma unroll
    for (int u = 0; u < IS; ++u) {
      const int e = tid + NT * u;
      if (e < IV) {
        uint32_t lo = 0u, hi = 0u;
        lo = __builtin_amdgcn_cvt_pk_fp8_f32(from_bf16(iv[u][0]) * inv_sa, from_bf16(iv[u][1]) * inv_sa, lo, false);
        lo = __builtin_amdgcn_cvt_pk_fp8_f32(from_bf16(iv[u][2]) * inv_sa, from_bf16(iv[u][3]) * inv_sa, lo, true);
        hi = __builtin_amdgcn_cvt_pk_fp8_f32(from_bf16(iv[u][4]) * inv_sa, from_bf16(iv[u][5]) * inv_sa, hi, false);
        hi = __builtin_amdgcn_cvt_pk_fp8_f32(from_bf16(iv[u][6]) * inv_sa, from_bf16(iv[u][7]) * inv_sa, hi, true);
        *(u32x2*)(s_in + (e / IQ) * CP + 8 * (e % IQ)) = u32x2{lo, hi};
      }
    }
    __syncthreads();
    if (tile + (int)gridDim.x < tiles) load_halo(tile + gridDim.x);  // in flight meanwhile
    f32x4 acc[RPW][4][NBW];
#pragma unroll
    for (int rw = 0; rw < RPW; ++rw)
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb) acc[rw][mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int kb = 0; kb < KD128 / 128; ++kb) {
      const int k0 = kb * 128 + 32 * lk;
      // past KD the weights are zero; read any in-tile (finite) activations there
      const int kk = k0 < KD ? k0 : 0;
      const int tap = kk / CIN, c0 = kk - tap * CIN;
      const int dy = tap / 3, dx = tap - dy * 3;
      i32x8 b[NBW];
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) {
        const uint8_t* src = s_w + out_channel(nb) * KDP + k0;
        const u32x4 v0 = *(const u32x4*)src, v1 = *(const u32x4*)(src + 16);
        b[nb] = i32x8{(int)v0[0], (int)v0[1], (int)v0[2], (int)v0[3], (int)v1[0], (int)v1[1], (int)v1[2],
                      (int)v1[3]};
      }
#pragma unroll
      for (int rw = 0; rw < RPW; ++rw) {
        const int ry = w + 4 * rw;
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          const uint8_t* src = s_in + ((ry + dy) * HC + mb * 16 + li + dx) * CP + c0;
          const u32x4 v0 = *(const u32x4*)src, v1 = *(const u32x4*)(src + 16);
          const i32x8 a = {(int)v0[0], (int)v0[1], (int)v0[2], (int)v0[3],
                           (int)v1[0], (int)v1[1], (int)v1[2], (int)v1[3]};
#pragma unroll
          for (int nb = 0; nb < NBW; ++nb)
            acc[rw][mb][nb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b[nb], acc[rw][mb][nb], 0, 0,
                                                                               0, 127, 0, 127);
        }
      }
    }
    // Epilogue through LDS, as in the BF16 kernel: activated outputs into the BF16 tile
    // [pixel][channel], then 16-byte NHWC stores; the largest |output| of the valid
    // pixels goes to amax_out once the block is done.
    __syncthreads();  // every wave is done with the halo tile
    {
      float sc[NBW], bo[NBW];
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) {
        const int o = out_channel(nb);
        sc[nb] = sa * ws[o];
        bo[nb] = bias ? bias[o] : 0.f;
      }
      const bool full = y0 + TR <= n && x0 + TC <= m;
      with_activation(act, [&](auto actc) {
        constexpr int ACT = decltype(actc)::value;
#pragma unroll
        for (int rw = 0; rw < RPW; ++rw) {
          const int ty = w + 4 * rw;
#pragma unroll
          for (int mb = 0; mb < 4; ++mb) {
            if constexpr (PAIR) {
#pragma unroll
              for (int h = 0; h < NBW / 2; ++h)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                  const int tx = mb * 16 + 4 * lk + r;
                  const float v0 = activate_lp_c<ACT>(fmaf(acc[rw][mb][2 * h][r], sc[2 * h], bo[2 * h]));
                  const float v1 =
                      activate_lp_c<ACT>(fmaf(acc[rw][mb][2 * h + 1][r], sc[2 * h + 1], bo[2 * h + 1]));
                  *reinterpret_cast<unsigned*>(s_out + (ty * TC + tx) * OP + out_channel(2 * h)) =
                      pack_bf16x2(v0, v1);
                  if (full || (y0 + ty < n && x0 + tx < m)) vmax = fmaxf(vmax, fmaxf(fabsf(v0), fabsf(v1)));
                }
            } else {
#pragma unroll
              for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                  const int tx = mb * 16 + 4 * lk + r;
                  const float v = activate_lp_c<ACT>(fmaf(acc[rw][mb][nb][r], sc[nb], bo[nb]));
                  s_out[(ty * TC + tx) * OP + out_channel(nb)] = to_bf16(v);
                  if (full || (y0 + ty < n && x0 + tx < m)) vmax = fmaxf(vmax, fabsf(v));
                }
            }
          }
        }
      });
    }
    __syncthreads();
    if constexpr (LASTQ) {
      fold_last_epilogue<COUT, TR, TC, OP, NT>(s_out, wl2, reinterpret_cast<float*>(out), N, n, m, i, y0, x0, tid);
    } else {
      constexpr int QV = COUT / 8;
      for (int e = tid; e < TR * TC * QV; e += NT) {
        const int px = e / QV, q = e - px * QV;
        const int y = y0 + px / TC, x = x0 + px % TC;
        if (y < n && x < m)
          *(u16x8*)(out + (((size_t)i * n + y) * m + x) * COUT + 8 * q) = *(const u16x8*)(s_out + px * OP + 8 * q);
      }
    }
  }
  if constexpr (!LASTQ) amax_publish(vmax, amax_out);
}

}  // namespace

bool conv_first_supported(int cout, int l) {
  return (cout == 8 || cout == 16 || cout == 32 || cout == 64) && l <= 64;
}
bool conv_last_supported(int cin) { return cin == 8 || cin == 16 || cin == 32 || cin == 64; }

void launch_conv_first(hipStream_t s, Timer& t, int N, int n, int m, int l, FieldRef X, FieldRef U,
                       const float* B, int cout, const float* w, const float* bias, int act,
                       void* out_nhwc, bool bf16, float* lift, unsigned* amax, const ObserveArgs* obs) {
  const unsigned blocks = (unsigned)((long long)N * ((n + 3) / 4) * ((m + 63) / 64));
  const ObserveArgs oa = obs ? *obs : ObserveArgs{};
  if (cout >= 64) {  // the lift as a field of its own first (k_conv_first reads its halo)
    constexpr int YB = 16;
    OIC_GLAUNCH(t, KC_LIFT, s, k_lift_bu<YB>, dim3((unsigned)((long long)N * ((n + YB - 1) / YB)),
                                                   (unsigned)((m + 255) / 256)),
                dim3(256), 0, N, n, m, l, U, B, lift);
  }
#define OIC_FIRST_CASE(CO)                                                                        \
  if (cout == CO) {                                                                               \
    if (bf16)                                                                                     \
      OIC_GLAUNCH(t, KC_CONV_FIRST, s, (k_conv_first<CO, bf16_t>), dim3(blocks), dim3(256), 0, N, n, \
                 m, l, X, U, B, w, bias, act, (bf16_t*)out_nhwc, amax, oa, (const float*)lift);   \
    else                                                                                          \
      OIC_GLAUNCH(t, KC_CONV_FIRST, s, (k_conv_first<CO, float>), dim3(blocks), dim3(256), 0, N, n,  \
                 m, l, X, U, B, w, bias, act, (float*)out_nhwc, amax, oa, (const float*)lift);    \
    return;                                                                                       \
  }
  OIC_FIRST_CASE(8)
  OIC_FIRST_CASE(16)
  OIC_FIRST_CASE(32)
  OIC_FIRST_CASE(64)
#undef OIC_FIRST_CASE
}

void launch_conv_last(hipStream_t s, Timer& t, int N, int n, int m, int cin, const void* in_nhwc,
                      const float* w, const float* bias, FieldOut fo, bool bf16, const ObserveArgs* obs) {
  const unsigned blocks = (unsigned)((long long)N * ((n + 3) / 4) * ((m + 63) / 64));
  const ObserveArgs oa = obs ? *obs : ObserveArgs{};
#define OIC_LAST_CASE(CI)                                                                         \
  if (cin == CI) {                                                                                \
    if (bf16)                                                                                     \
      OIC_GLAUNCH(t, KC_CONV_LAST, s, (k_conv_last<CI, bf16_t>), dim3(blocks), dim3(256), 0, N, n, m, \
                 (const bf16_t*)in_nhwc, w, bias, fo, oa);                                        \
    else                                                                                          \
      OIC_GLAUNCH(t, KC_CONV_LAST, s, (k_conv_last<CI, float>), dim3(blocks), dim3(256), 0, N, n, m,  \
                 (const float*)in_nhwc, w, bias, fo, oa);                                         \
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

// Workgroups of `Kernel` (threads per workgroup as given) that one CU holds at once.
template <auto Kernel>
int resident_per_cu(int threads) {
  static const int nb = [threads] {
    int b = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, Kernel, threads, 0) != hipSuccess || b < 1) b = 1;
    return b;
  }();
  return nb;
}

// wave groups per workgroup of the BF16 hidden layers: two groups of four waves split
// the output channels once a layer has 32 or more of them
constexpr int kBf16GroupsWide = 2;  // 64 input or output channels
constexpr int kBf16Groups32 = 2;    // 32 output channels

// k_conv_bf16r addresses one member's input image through a buffer resource
static bool bf16r_fits(int n, int m, int cin) { return (long long)n * m * cin * 2 < (1LL << 31); }

// one output row per wave: 2 tile rows at 64 output channels (two channel groups), 4 at 32
template <int CI, int CO, bool LASTQ>
void launch_bf16r(hipStream_t s, Timer& t, int kclass, int N, int n, int m, const void* in_nhwc, const void* wt,
                  const float* bias, int act, void* out, const uint16_t* wl2) {
  constexpr int TRV = 4 / (CO / 32);
  const long long tiles = (long long)N * ((n + TRV - 1) / TRV) * ((m + 63) / 64);
  const long long cap = 2LL * 256;
  const unsigned blocks = (unsigned)(tiles < cap ? tiles : cap);
  if (launch_group().slots > 1)
    OIC_GLAUNCH(t, kclass, s, (k_conv_bf16r<CI, CO, TRV, LASTQ, true>), dim3(blocks), dim3(256), 0, N, n, m,
                (const bf16_t*)in_nhwc, (const bf16_t*)wt, bias, act, (bf16_t*)out, (const bf16_t*)wl2);
  else
    OIC_GLAUNCH(t, kclass, s, (k_conv_bf16r<CI, CO, TRV, LASTQ, false>), dim3(blocks), dim3(256), 0, N, n, m,
                (const bf16_t*)in_nhwc, (const bf16_t*)wt, bias, act, (bf16_t*)out, (const bf16_t*)wl2);
}

void launch_conv_mfma_bf16(hipStream_t s, Timer& t, int kclass, int N, int n, int m, int cin, int cout,
                           const void* in_nhwc, const void* wt, const float* bias, int act,
                           void* out_nhwc) {
  if ((cin == 32 || cin == 64) && (cout == 32 || cout == 64) && bf16r_fits(n, m, cin)) {
    if (cin == 32 && cout == 32) launch_bf16r<32, 32, false>(s, t, kclass, N, n, m, in_nhwc, wt, bias, act, out_nhwc, nullptr);
    if (cin == 32 && cout == 64) launch_bf16r<32, 64, false>(s, t, kclass, N, n, m, in_nhwc, wt, bias, act, out_nhwc, nullptr);
    if (cin == 64 && cout == 32) launch_bf16r<64, 32, false>(s, t, kclass, N, n, m, in_nhwc, wt, bias, act, out_nhwc, nullptr);
    if (cin == 64 && cout == 64) launch_bf16r<64, 64, false>(s, t, kclass, N, n, m, in_nhwc, wt, bias, act, out_nhwc, nullptr);
    return;
  }
  // pairs with 64 channels hold one workgroup per CU (their weights fill most of the LDS):
  // there two groups of four waves split the output channels of each tile
#define OIC_BF_CASE(CI, CO)                                                                      \
  if (cin == CI && cout == CO) {                                                                 \
    constexpr int TRV = CI <= 32 ? 8 : 4;                                                        \
    constexpr int WG = (CI == 64 || CO == 64) ? kBf16GroupsWide : (CO >= 32 ? kBf16Groups32 : 1);          \
    constexpr auto kern = k_conv_mfma_bf16<CI, CO, TRV, WG>;                                     \
    const long long tiles = (long long)N * ((n + TRV - 1) / TRV) * ((m + 63) / 64);             \
    const long long cap = 256LL * resident_per_cu<kern>(256 * WG); /* persistent */             \
    const unsigned blocks = (unsigned)(tiles < cap ? tiles : cap);                               \
    OIC_GLAUNCH(t, kclass, s, kern, dim3(blocks), dim3(256 * WG), 0, N, n, m,                    \
               (const bf16_t*)in_nhwc, (const bf16_t*)wt, bias, act, (bf16_t*)out_nhwc, nullptr); \
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

bool conv_last_folds_bf16(int cin, int cout) { return cout == 64 && (cin == 32 || cin == 64); }

void launch_conv_mfma_bf16_last(hipStream_t s, Timer& t, int N, int n, int m, int cin, const void* in_nhwc,
                                const void* wt, const float* bias, int act, const uint16_t* wl2,
                                const float* bias_last, float* qbuf, FieldOut fo, const ObserveArgs* obs) {
  if (bf16r_fits(n, m, cin)) {
    if (cin == 64) launch_bf16r<64, 64, true>(s, t, KC_CONV_MID, N, n, m, in_nhwc, wt, bias, act, qbuf, wl2);
    else launch_bf16r<32, 64, true>(s, t, KC_CONV_MID, N, n, m, in_nhwc, wt, bias, act, qbuf, wl2);
    const ObserveArgs oa = obs ? *obs : ObserveArgs{};
    OIC_GLAUNCH(t, KC_CONV_LAST, s, k_conv_last_sum, dim3((unsigned)(N * n), (unsigned)((m + 255) / 256)), dim3(256),
               0, N, n, m, qbuf, bias_last, fo, oa);
    return;
  }
#define OIC_BFL_CASE(CI)                                                                         \
  if (cin == CI) {                                                                               \
    constexpr int TRV = CI <= 32 ? 8 : 4;                                                        \
    constexpr auto kern = k_conv_mfma_bf16<CI, 64, TRV, kBf16GroupsWide, true>;                  \
    const long long tiles = (long long)N * ((n + TRV - 1) / TRV) * ((m + 63) / 64);             \
    const long long cap = 256LL * resident_per_cu<kern>(256 * kBf16GroupsWide);                  \
    const unsigned blocks = (unsigned)(tiles < cap ? tiles : cap);                               \
    OIC_GLAUNCH(t, KC_CONV_MID, s, kern, dim3(blocks), dim3(256 * kBf16GroupsWide), 0, N, n, m,   \
               (const bf16_t*)in_nhwc, (const bf16_t*)wt, bias, act, (bf16_t*)qbuf, (const bf16_t*)wl2); \
  }
  OIC_BFL_CASE(32)
  OIC_BFL_CASE(64)
#undef OIC_BFL_CASE
  const ObserveArgs oa = obs ? *obs : ObserveArgs{};
  OIC_GLAUNCH(t, KC_CONV_LAST, s, k_conv_last_sum, dim3((unsigned)(N * n), (unsigned)((m + 255) / 256)), dim3(256),
             0, N, n, m, qbuf, bias_last, fo, oa);
}

bool conv_mfma_fp8_supported(int cin, int cout) {
  return (cin == 32 || cin == 64) && (cout == 16 || cout == 32 || cout == 64);
}

constexpr int kFp8Groups = 2;  // wave groups of the FP8 hidden layers with 32+ output channels

void launch_conv_mfma_fp8(hipStream_t s, Timer& t, int kclass, int N, int n, int m, int cin, int cout,
                          const void* in_nhwc, const unsigned* amax_in, const uint8_t* wq, const float* ws,
                          const float* bias, int act, void* out_nhwc, unsigned* amax_out) {
  // 32+ output channels: two groups of four waves split each tile's output channels
  // (persistent kernel, 256x256: 330 ms per solve non-persistent, 301 persistent with
  // one group, 222 with two)
#define OIC_F8_CASE(CI, CO)                                                                        \
  if (cin == CI && cout == CO) {                                                                   \
    constexpr int TRV = 8;                                                                         \
    constexpr int WG = CO >= 32 ? kFp8Groups : 1;                                                      \
    constexpr auto kern = k_conv_mfma_fp8<CI, CO, TRV, WG>;                                        \
    const long long tiles = (long long)N * ((n + TRV - 1) / TRV) * ((m + 63) / 64);               \
    const long long cap = 256LL * resident_per_cu<kern>(256 * WG); /* persistent */               \
    const unsigned blocks = (unsigned)(tiles < cap ? tiles : cap);                                 \
    OIC_LAUNCH(t, kclass, s, kern, dim3(blocks), dim3(256 * WG), 0, N, n, m, (const bf16_t*)in_nhwc, \
               amax_in, wq, ws, bias, act, (bf16_t*)out_nhwc, amax_out, nullptr);                  \
    return;                                                                                        \
  }
  OIC_F8_CASE(32, 16)
  OIC_F8_CASE(32, 32)
  OIC_F8_CASE(32, 64)
  OIC_F8_CASE(64, 16)
  OIC_F8_CASE(64, 32)
  OIC_F8_CASE(64, 64)
#undef OIC_F8_CASE
}

void launch_conv_mfma_fp8_last(hipStream_t s, Timer& t, int N, int n, int m, int cin, const void* in_nhwc,
                               const unsigned* amax_in, const uint8_t* wq, const float* ws, const float* bias,
                               int act, const uint16_t* wl2, const float* bias_last, float* qbuf, FieldOut fo,
                               const ObserveArgs* obs) {
#define OIC_F8L_CASE(CI)                                                                            \
  if (cin == CI) {                                                                                  \
    constexpr int TRV = 8;                                                                          \
    constexpr auto kern = k_conv_mfma_fp8<CI, 64, TRV, kFp8Groups, true>;                           \
    const long long tiles = (long long)N * ((n + TRV - 1) / TRV) * ((m + 63) / 64);                \
    const long long cap = 256LL * resident_per_cu<kern>(256 * kFp8Groups);                          \
    const unsigned blocks = (unsigned)(tiles < cap ? tiles : cap);                                  \
    OIC_LAUNCH(t, KC_CONV_MID, s, kern, dim3(blocks), dim3(256 * kFp8Groups), 0, N, n, m,            \
               (const bf16_t*)in_nhwc, amax_in, wq, ws, bias, act, (bf16_t*)qbuf, (unsigned*)nullptr, \
               (const bf16_t*)wl2);                                                                 \
  }
  OIC_F8L_CASE(32)
  OIC_F8L_CASE(64)
#undef OIC_F8L_CASE
  const ObserveArgs oa = obs ? *obs : ObserveArgs{};
  OIC_GLAUNCH(t, KC_CONV_LAST, s, k_conv_last_sum, dim3((unsigned)(N * n), (unsigned)((m + 255) / 256)), dim3(256),
             0, N, n, m, qbuf, bias_last, fo, oa);
}

void launch_zero_u32(hipStream_t s, Timer& t, unsigned* p, int count) {
  OIC_LAUNCH(t, KC_ASSEMBLE, s, k_zero_u32, dim3((unsigned)((count + 63) / 64)), dim3(64), 0, p, count);
}

bool conv_mfma_supported(int cin, int cout) {
  return (cin == 16 || cin == 32 || cin == 64) && (cout == 16 || cout == 32 || cout == 64);
}

// k_conv_f32r addresses one member's input image through a buffer resource: its byte
// size must fit the 32-bit record count and offsets
static bool f32r_fits(int n, int m, int cin) { return (long long)n * m * cin * 4 < (1LL << 31); }

void launch_conv_mfma(hipStream_t s, Timer& t, int kclass, int N, int n, int m, int cin, int cout,
                      const float* in_nhwc, const float* wk, const float* bias, int act,
                      float* out_nhwc) {
  if (cout == 64 && (cin == 32 || cin == 64) && f32r_fits(n, m, cin)) {
    // weights in registers, two persistent workgroups per CU
    constexpr int TRV = 2;
    const long long tiles = (long long)N * ((n + TRV - 1) / TRV) * ((m + 63) / 64);
    const long long cap = 2LL * 256;
    const unsigned blocks = (unsigned)(tiles < cap ? tiles : cap);
    if (cin == 64)
      OIC_LAUNCH(t, kclass, s, (k_conv_f32r<64, TRV, false>), dim3(blocks), dim3(256), 0, N, n, m, in_nhwc, wk,
                 bias, act, out_nhwc, nullptr);
    else
      OIC_LAUNCH(t, kclass, s, (k_conv_f32r<32, TRV, false>), dim3(blocks), dim3(256), 0, N, n, m, in_nhwc, wk,
                 bias, act, out_nhwc, nullptr);
    return;
  }
#define OIC_CONV_CASE(CI, CO)                                                                   \
  if (cin == CI && cout == CO) {                                                                \
    constexpr bool W8 = CI == 16 && CO == 16;  /* 8 waves, one row each */            \
    constexpr int TRV = W8 ? 8 : ((CI <= 16 && CO <= 32 && CO != CI) ? 8 : 4);                 \
    constexpr int WGM = W8 ? 2 : 1;                                                             \
    constexpr int CCH = CI <= 32 ? CI : 32;                                                     \
    const long long tiles = (long long)N * ((n + TRV - 1) / TRV) * ((m + 63) / 64);             \
    if constexpr (CCH == CI) {  /* persistent: as many workgroups as the CUs' LDS holds */      \
      constexpr int lds = 4 * ((TRV + 2) * 66 * (CI + 1) + 9 * CI * CO);                         \
      constexpr int per_cu = 160 * 1024 / lds < 4 / WGM ? 160 * 1024 / lds : 4 / WGM;            \
      constexpr long long cap = 256LL * (per_cu > 0 ? per_cu : 1);                               \
      const unsigned blocks = (unsigned)(tiles < cap ? tiles : cap);                            \
      OIC_LAUNCH(t, kclass, s, (k_conv_mfma_f32p<CI, CO, TRV, WGM>), dim3(blocks), dim3(256 * WGM), \
                 0, N, n, m, in_nhwc, wk, bias, act, out_nhwc);                                 \
    } else {                                                                                    \
      OIC_LAUNCH(t, kclass, s, (k_conv_mfma_f32<CI, CO, TRV, CCH>), dim3((unsigned)tiles), dim3(256), \
                 0, N, n, m, in_nhwc, wk, bias, act, out_nhwc);                                 \
    }                                                                                           \
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

bool conv_last_folds(int n, int m, int cin, int cout) {
  return cout == 64 && (cin == 32 || cin == 64) && f32r_fits(n, m, cin);
}

void launch_conv_mfma_last(hipStream_t s, Timer& t, int N, int n, int m, int cin, const float* in_nhwc,
                           const float* wk, const float* bias, int act, const float* w_last,
                           const float* bias_last, float* qbuf, FieldOut fo, const ObserveArgs* obs) {
  constexpr int TRV = 2;
  const long long tiles = (long long)N * ((n + TRV - 1) / TRV) * ((m + 63) / 64);
  const long long cap = 2LL * 256;
  const unsigned blocks = (unsigned)(tiles < cap ? tiles : cap);
  if (cin == 64)
    OIC_LAUNCH(t, KC_CONV_MID, s, (k_conv_f32r<64, TRV, true>), dim3(blocks), dim3(256), 0, N, n, m, in_nhwc, wk,
               bias, act, qbuf, w_last);
  else
    OIC_LAUNCH(t, KC_CONV_MID, s, (k_conv_f32r<32, TRV, true>), dim3(blocks), dim3(256), 0, N, n, m, in_nhwc, wk,
               bias, act, qbuf, w_last);
  const ObserveArgs oa = obs ? *obs : ObserveArgs{};
  OIC_GLAUNCH(t, KC_CONV_LAST, s, k_conv_last_sum, dim3((unsigned)(N * n), (unsigned)((m + 255) / 256)), dim3(256),
             0, N, n, m, qbuf, bias_last, fo, oa);
}

int rollout_fp32(hipStream_t s, Timer& t, const oic_config& c, const Fp32Net& net, float* act0,
                 float* act1, int batch, FieldRef X, FieldRef U, FieldOut out, const ObserveArgs* obs) {
  const int L = c.n_layers;
  float* act[2] = {act0, act1};
  int done = 0;
  int cur = 0;
  int k0 = 0;
  if (L > 1 && conv_first_supported(c.channels[1], c.l)) {
    // lift fused into the first layer
    launch_conv_first(s, t, batch, c.n, c.m, c.l, X, U, net.B, c.channels[1], net.W[0], net.bias[0],
                      c.activation, act[1], false, act[0], nullptr, obs);
    if (obs && obs->U_cur) done |= ROLL_U_ASSEMBLED;
    cur = 1;
    k0 = 1;
  } else {
    launch_lift(s, t, batch, c.n, c.m, c.l, X, U, net.B, act[0]);
  }
  for (int k = k0; k < L; ++k) {
    const int cin = c.channels[k], cout = c.channels[k + 1];
    const bool last = k == L - 1;
    const int cls = k == 0 ? KC_CONV_FIRST : (last ? KC_CONV_LAST : KC_CONV_MID);
    if (last && k > 0 && conv_last_supported(cin)) {
      launch_conv_last(s, t, batch, c.n, c.m, cin, act[cur], net.W[k], net.bias[k], out, false, obs);
      if (obs) done |= ROLL_X_OBSERVED;
      continue;
    }
    if (k == L - 2 && k > 0 && net.Wk[k] && conv_last_folds(c.n, c.m, cin, cout) && c.channels[L] == 1) {
      // the last hidden layer with the last layer folded into its epilogue
      launch_conv_mfma_last(s, t, batch, c.n, c.m, cin, act[cur], net.Wk[k], net.bias[k], c.activation,
                            net.W[L - 1], net.bias[L - 1], act[1 - cur], out, obs);
      if (obs) done |= ROLL_X_OBSERVED;
      break;
    }
    if (!last && net.Wk[k]) {
      launch_conv_mfma(s, t, cls, batch, c.n, c.m, cin, cout, act[cur], net.Wk[k], net.bias[k],
                       c.activation, act[1 - cur]);
      cur = 1 - cur;
      continue;
    }
    FieldOut fo = last ? out : FieldOut{nullptr, 0, 0};
    launch_conv(s, t, cls, batch, c.n, c.m, cin, cout, act[cur], net.W[k], net.bias[k], c.activation,
                last ? nullptr : act[1 - cur], fo);
    cur = 1 - cur;
  }
  return done;
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
