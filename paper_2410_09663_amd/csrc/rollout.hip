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

}  // namespace

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
  constexpr int CB = 16;
  const unsigned gy = (unsigned)((cout + CB - 1) / CB);
  OIC_LAUNCH(t, kclass, s, k_conv_direct<CB>, dim3(gx, gy), dim3(256), 0, N, n, m, cin, cout,
             in_nhwc, w_oihw, bias, act, out_nhwc, final_out);
}

}  // namespace oic
