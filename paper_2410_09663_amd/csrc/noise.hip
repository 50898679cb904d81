// Noise of the virtual system and the elementwise steps that consume it:
//  - Philox4x32-10 (Salmon et al., SC'11) standard normals for the seeded solve;
//  - the initial ensemble (Algorithm 1, line 4);
//  - the control part of the forecast, U_t = U_{t-1} + W_t (Eq. (4), Eq. (15b));
//  - the perturbed virtual observations Ybar^i = H Xbar^i + Vbar^i (Eq. (12)).
#include <algorithm>

#include "noise_value.h"
#include "oic_internal.h"

namespace oic {
namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kWeyl0 = 0x9E3779B9u;
constexpr uint32_t kWeyl1 = 0xBB67AE85u;

__device__ __forceinline__ void philox_rounds(uint32_t& x0, uint32_t& x1, uint32_t& x2,
                                              uint32_t& x3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kWeyl0;
      k1 += kWeyl1;
    }
    const uint32_t hi0 = __umulhi(kPhiloxM0, x0), lo0 = kPhiloxM0 * x0;
    const uint32_t hi1 = __umulhi(kPhiloxM1, x2), lo1 = kPhiloxM1 * x2;
    const uint32_t n0 = hi1 ^ x1 ^ k0;
    const uint32_t n2 = hi0 ^ x3 ^ k1;
    x0 = n0;
    x1 = lo1;
    x2 = n2;
    x3 = lo0;
  }
}

// Normal number e of noise kind `kind`: counter (e lo, e hi, kind, 0), key (seed lo, seed hi);
// two 53-bit uniforms, Box-Muller cosine branch in FP64, rounded to FP32.
__device__ __forceinline__ float philox_normal(uint64_t seed, uint32_t kind, uint64_t e) {
  uint32_t x0 = (uint32_t)e, x1 = (uint32_t)(e >> 32), x2 = kind, x3 = 0u;
  philox_rounds(x0, x1, x2, x3, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t a = ((((uint64_t)x1) << 32) | x0) >> 11;
  const uint64_t b = ((((uint64_t)x3) << 32) | x2) >> 11;
  const double u1 = ((double)a + 1.0) * 0x1.0p-53;
  const double u2 = (double)b * 0x1.0p-53;
  const double z = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
  return (float)z;
}

// The seed is read from device memory so that a captured solve can be replayed with a
// new seed without touching the graph.
__global__ void k_normals(float* __restrict__ out, size_t count, const uint64_t* __restrict__ seed_ptr,
                          uint32_t kind, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(out);
  OIC_GSH(seed_ptr);
  const uint64_t seed = *seed_ptr;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += stride)
    out[e] = philox_normal(seed, kind, e);
}

// Slice k of every member: X rows = X_k (no spread), U rows = U_prev + W_0^i.  Also
// clears the positive-definiteness flag of the solve.
__global__ void k_init_slice0(Dims d, float* __restrict__ traj, const float* __restrict__ X0,
                              const float* __restrict__ Uprev, NoiseRef w0, int* __restrict__ flag, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(traj);
  OIC_GSH(X0);
  OIC_GSH(Uprev);
  OIC_GSH(w0);
  OIC_GSH(flag);
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *flag = 0;
  const int NM = (int)d.NM();
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (col >= NM) return;
  const int i = col / d.m, x = col - i * d.m;
  float v;
  if (q < d.n) {
    v = X0[(size_t)q * d.m + x];
  } else {
    const int a = q - d.n;
    v = Uprev[(size_t)a * d.m + x] + noise_value(w0, a, i, x, d.m);
  }
  traj[(size_t)q * NM + col] = v;
}

// U rows of slice t: U_t^i = U_{t-1}^i (after the analysis at t-1) + W_t^i.
__global__ void k_assemble_u(Dims d, float* __restrict__ traj, int step, NoiseRef w, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(traj);
  OIC_GSH(w);
  const int NM = (int)d.NM();
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (col >= NM) return;
  const int i = col / d.m, x = col - i * d.m;
  const size_t rr = (size_t)d.rr();
  const float prev = traj[((size_t)(step - 1) * rr + d.n + a) * NM + col];
  traj[((size_t)step * rr + d.n + a) * NM + col] = prev + noise_value(w, a, i, x, d.m);
}

// Ybar^i_t = [X_t^i + V_X^i; U_t^i + V_U^i].
__global__ void k_observe(Dims d, const float* __restrict__ traj, int step, float* __restrict__ Y,
                          NoiseRef vx, NoiseRef vu, int row0, Grp grp) {
  OIC_GROUP_ENTER(grp);
  OIC_GSH(traj);
  OIC_GSH(Y);
  OIC_GSH(vx);
  OIC_GSH(vu);
  const int NM = (int)d.NM();
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = row0 + (int)blockIdx.y;
  if (col >= NM) return;
  const int i = col / d.m, x = col - i * d.m;
  const float s = traj[((size_t)step * d.rr() + q) * NM + col];
  const float v = q < d.n ? noise_value(vx, q, i, x, d.m) : noise_value(vu, q - d.n, i, x, d.m);
  Y[(size_t)q * NM + col] = s + v;
}

// Up to three device-to-device copies in one launch, skipped entirely when *guard is
// non-zero (guard may be NULL); with seed_dst set, thread 0 also stores the seed.
__global__ void k_copy_jobs(CopyJob j0, CopyJob j1, CopyJob j2, const int* __restrict__ guard,
                            uint64_t seed, uint64_t* __restrict__ seed_dst) {
  if (guard && *guard) return;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (seed_dst && t == 0) *seed_dst = seed;
  for (long long e = t; e < j0.count; e += stride) j0.dst[e] = j0.src[e];
  for (long long e = t; e < j1.count; e += stride) j1.dst[e] = j1.src[e];
  for (long long e = t; e < j2.count; e += stride) j2.dst[e] = j2.src[e];
}

// The constraint row of Ybar for every member and column (one thread per column).
__global__ void k_constraint_row(Dims d, const float* __restrict__ traj, int step, float* __restrict__ Y,
                                 const float* __restrict__ aX, const float* __restrict__ aU, float b,
                                 float alpha, float beta, float sqrt_rz, const float* __restrict__ Zvz) {
  const int NM = (int)d.NM();
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= NM) return;
  const float* slice = traj + (size_t)step * d.rr() * NM + col;
  float g = -b;
  for (int r = 0; r < d.n; ++r) g = fmaf(aX[r], slice[(size_t)r * NM], g);
  for (int a = 0; a < d.l; ++a) g = fmaf(aU[a], slice[(size_t)(d.n + a) * NM], g);
  // softplus without overflow: max(x, 0) + log1p(exp(-|x|))
  const float x = beta * g;
  const float sp = fmaxf(x, 0.f) + log1pf(expf(-fabsf(x)));
  Y[(size_t)(d.n + d.l) * NM + col] = sp / alpha + sqrt_rz * Zvz[col];
}

inline dim3 row_grid(long long NM, int rows) {
  return dim3((unsigned)((NM + 255) / 256), (unsigned)rows);
}

}  // namespace

void launch_normals(hipStream_t s, Timer& t, float* out, size_t count, const uint64_t* seed,
                    uint32_t kind) {
  if (!count) return;
  size_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  OIC_GLAUNCH(t, KC_NOISE, s, k_normals, dim3((unsigned)blocks), dim3(256), 0, out, count, seed, kind);
}

void launch_init_slice0(hipStream_t s, Timer& t, const Dims& d, float* traj, const float* X0,
                        const float* Uprev, NoiseRef w0, int* flag) {
  OIC_GLAUNCH(t, KC_INIT, s, k_init_slice0, row_grid(d.NM(), d.rr()), dim3(256), 0, d, traj, X0,
             Uprev, w0, flag);
}

void launch_assemble_u(hipStream_t s, Timer& t, const Dims& d, float* traj, int step, NoiseRef w) {
  OIC_GLAUNCH(t, KC_ASSEMBLE, s, k_assemble_u, row_grid(d.NM(), d.l), dim3(256), 0, d, traj, step, w);
}

void launch_observe(hipStream_t s, Timer& t, const Dims& d, const float* traj, int step, float* Y,
                    NoiseRef vx, NoiseRef vu, int row0, int row1) {
  if (row1 <= row0) return;
  OIC_GLAUNCH(t, KC_OBSERVE, s, k_observe, row_grid(d.NM(), row1 - row0), dim3(256), 0, d, traj, step, Y,
             vx, vu, row0);
}

void launch_copy_jobs(hipStream_t s, Timer& t, const CopyJob* jobs, int count, const int* guard, uint64_t seed,
                      uint64_t* seed_dst) {
  CopyJob j[3] = {};
  long long most = 1;
  for (int k = 0; k < count && k < 3; ++k) {
    j[k] = jobs[k];
    most = std::max(most, j[k].count);
  }
  const unsigned blocks = (unsigned)std::min<long long>((most + 255) / 256, 256);
  OIC_LAUNCH(t, KC_COPY, s, k_copy_jobs, dim3(blocks), dim3(256), 0, j[0], j[1], j[2], guard, seed, seed_dst);
}

void launch_constraint_row(hipStream_t s, Timer& t, const Dims& d, const float* traj, int step, float* Y,
                           const float* aX, const float* aU, float b, float alpha, float beta,
                           float sqrt_rz, const float* Zvz) {
  const long long NM = d.NM();
  OIC_LAUNCH(t, KC_OBSERVE, s, k_constraint_row, dim3((unsigned)((NM + 255) / 256)), dim3(256), 0, d, traj,
             step, Y, aX, aU, b, alpha, beta, sqrt_rz, Zvz);
}

}  // namespace oic
