// Internal declarations of liboic: the handle, the device buffer layout and the
// kernel launchers.  Not part of the ABI.
//
// Device layout of one solve (N members, horizon H, rows per slice rr = n + l):
//   traj  : (H+1) slices x rr rows x (N*m) columns, FP32, row-major.  Slice s,
//           row q, member i, column x sits at ((s*rr + q)*N + i)*m + x, i.e. the
//           members of one row lie side by side, [X^1 X^2 ... X^N], so that the
//           pooled sums of Eq. (13), sum_i A^i D^iT, are plain row-by-row dot
//           products over the N*m columns.  The dU rows of the augmented state
//           are not stored: no other row, gain or output depends on them.
//   Y     : p = n + l rows x (N*m) columns, the perturbed observations of Eq. (12).
//   act   : two NHWC activation buffers [N][n][m][C] for the rollout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <type_traits>
#include <vector>

#include "../../include/oic.h"

namespace oic {

// An FP8 rollout keeps each layer's largest |activation| as kAmaxSlots partial maxima
// (publishers spread their atomic maxima over the slots; readers take the maximum of all),
// so that a layer's hundreds of thousands of waves do not queue on one address.
constexpr int kAmaxSlots = 64;

enum KernelClass {
  KC_NOISE = 0,
  KC_INIT,
  KC_LIFT,
  KC_CONV_FIRST,
  KC_CONV_MID,
  KC_CONV_LAST,
  KC_ASSEMBLE,
  KC_OBSERVE,
  KC_MEANS,
  KC_STATS,
  KC_STATS_REDUCE,
  KC_CHOL,
  KC_GAIN,
  KC_UPDATE,
  KC_EXTRACT,
  KC_COPY,
  KC_COUNT
};

extern const char* const kKernelClassNames[KC_COUNT];

// Per-kernel-class timing with HIP events on the handle's stream.
struct Timer {
  bool enabled = false;
  std::vector<hipEvent_t> pool;
  std::vector<int> pending_class;  // class of each recorded pair, in order
  size_t cursor = 0;
  long long launches[KC_COUNT] = {};
  double total_ms[KC_COUNT] = {};
  void reset();
  // Records the start event of a launch of class c; returns the pair index or -1.
  int begin(int c, hipStream_t s);
  void end(int idx, hipStream_t s);
  // Call after the stream is synchronised: folds every pending pair into the totals.
  void harvest();
  void destroy();
};

// Noise source for one kind at one horizon step: standard normals Z laid out
// [member][row][col] (row stride m, member stride rows*m), and the row factor:
// either a diagonal scale (diag != null) or a dense lower-triangular L (rows x rows).
struct NoiseRef {
  const float* Z;
  const float* diag;
  const float* L;
  int rows;
};

struct Dims {
  int n, m, l, N, H;
  int nc = 0;  // barrier-observed constraint rows appended to Ybar (0 or 1)
  __host__ __device__ int rr() const { return n + l; }
  __host__ __device__ int p() const { return n + l + nc; }
  __host__ __device__ long long NM() const { return (long long)N * m; }
};

// ---- grouped launches ----
// A group is a set of handles of one configuration whose device buffers all sit at the
// same offsets inside equal slabs, slot g's slab `stride` bytes after slot 0's.  One
// launch then serves every slot: its grid is the plain grid repeated over blockIdx.z =
// slot, every buffer address a kernel receives is slot 0's and the kernel moves it by
// blockIdx.z * stride, and a slot whose entry in `active` is 0 leaves at once (the same
// captured launches serve any subset of the slots).  Each slot's workgroups do exactly
// what the plain launch does on that slot's buffers, so a slot's results do not depend
// on the other slots.  A plain launch has one z-slice, stride 0 and no mask.
struct Grp {
  unsigned long long stride;
  const int* active;
};
// The group the launches of the calling thread go to (one slot and no mask by default).
// Launchers of kernels with a grouped form repeat their grid over `slots` z-slices and
// pass `g`; any other launch made while slots > 1 is not made and sets `unsupported`.
struct LaunchGroup {
  unsigned slots = 1;
  Grp g{0, nullptr};
  bool unsupported = false;
};
LaunchGroup& launch_group();

template <typename T>
__device__ __forceinline__ T* gshift(T* p, unsigned long long off) {
  return p ? reinterpret_cast<T*>(reinterpret_cast<char*>(const_cast<typename std::remove_const<T>::type*>(p)) + off)
           : p;
}

// ---- kernel launchers (defined in the .hip files) ----
void launch_normals(hipStream_t s, Timer& t, float* out, size_t count, const uint64_t* seed,
                    uint32_t kind);

void launch_init_slice0(hipStream_t s, Timer& t, const Dims& d, float* traj, const float* X0,
                        const float* Uprev, NoiseRef w0, int* flag);
void launch_assemble_u(hipStream_t s, Timer& t, const Dims& d, float* traj, int step, NoiseRef w);
// observation rows row0 .. row1 - 1 of Ybar (X rows below n, U rows from n on)
void launch_observe(hipStream_t s, Timer& t, const Dims& d, const float* traj, int step, float* Y,
                    NoiseRef vx, NoiseRef vu, int row0, int row1);
// Row n + l of Ybar: the barrier observation z = ln(1 + exp(beta g)) / alpha + sqrt(rz) eps
// of the per-column constraint g = aX . X_t[:, c] + aU . U_t[:, c] - b of every member
// (slice `step` of the trajectory, before the observation noise); eps from Zvz (N x m).
void launch_constraint_row(hipStream_t s, Timer& t, const Dims& d, const float* traj, int step, float* Y,
                           const float* aX, const float* aU, float b, float alpha, float beta,
                           float sqrt_rz, const float* Zvz);

// Rollout.  Field element (i, y, x) of a strided source sits at base + i*si + y*sy + x.
// Side outputs of a solve's rollout (null pointers: none).  The last layer writes the X
// rows of Ybar next to the new states (Eq. (12)); with U_cur set, the first layer, which
// reads U_{t-1}, also writes the U rows of the new slice, U_t = U_{t-1} + W_t (Eq. (4)),
// and their rows of Ybar.  U_cur and Y are row-major with row stride NM, member i's
// columns at i*m ..
struct ObserveArgs {
  float* U_cur;
  float* Y;
  long long NM;
  NoiseRef w, vx, vu;
};
// One device-to-device copy of `count` floats (count 0: nothing).
struct CopyJob {
  const float* src;
  float* dst;
  long long count;
};
// Up to three copies in one kernel, all skipped when *guard != 0 (guard NULL: always
// done); with seed_dst set the seed is stored there too.
void launch_copy_jobs(hipStream_t s, Timer& t, const CopyJob* jobs, int count, const int* guard, uint64_t seed,
                      uint64_t* seed_dst);
struct FieldRef {
  const float* base;
  long long si, sy;
};
struct FieldOut {
  float* base;
  long long si, sy;
};
__device__ __forceinline__ NoiseRef gshift(NoiseRef r, unsigned long long off) {
  r.Z = gshift(r.Z, off);
  r.diag = gshift(r.diag, off);
  r.L = gshift(r.L, off);
  return r;
}
__device__ __forceinline__ ObserveArgs gshift(ObserveArgs o, unsigned long long off) {
  o.U_cur = gshift(o.U_cur, off);
  o.Y = gshift(o.Y, off);
  o.w = gshift(o.w, off);
  o.vx = gshift(o.vx, off);
  o.vu = gshift(o.vu, off);
  return o;
}
__device__ __forceinline__ FieldRef gshift(FieldRef f, unsigned long long off) {
  f.base = gshift(f.base, off);
  return f;
}
__device__ __forceinline__ FieldOut gshift(FieldOut f, unsigned long long off) {
  f.base = gshift(f.base, off);
  return f;
}

void launch_lift(hipStream_t s, Timer& t, int N, int n, int m, int l, FieldRef X, FieldRef U,
                 const float* B, float* out_nhwc);
void launch_conv(hipStream_t s, Timer& t, int kclass, int N, int n, int m, int cin, int cout,
                 const float* in_nhwc, const float* w_oihw, const float* bias, int act,
                 float* out_nhwc, FieldOut final_out);

// First layer with the lift fused (2 -> cout) and last layer (cin -> 1) on tiles.
bool conv_first_supported(int cout, int l);
bool conv_last_supported(int cin);
// bf16: activations are stored as BF16 (first layer output, last layer input).  lift:
// N n m floats that the 64-channel layer uses for its lift channel B U (not read after).
void launch_conv_first(hipStream_t s, Timer& t, int N, int n, int m, int l, FieldRef X, FieldRef U,
                       const float* B, int cout, const float* w, const float* bias, int act,
                       void* out_nhwc, bool bf16, float* lift, unsigned* amax = nullptr,
                       const ObserveArgs* obs = nullptr);
void launch_conv_last(hipStream_t s, Timer& t, int N, int n, int m, int cin, const void* in_nhwc,
                      const float* w, const float* bias, FieldOut fo, bool bf16,
                      const ObserveArgs* obs = nullptr);
// Hidden layers in BF16 on MFMA.  wt holds BF16 weights as [cout][tap*cin + c].
bool conv_mfma_bf16_supported(int cin, int cout);
void launch_conv_mfma_bf16(hipStream_t s, Timer& t, int kclass, int N, int n, int m, int cin, int cout,
                           const void* in_nhwc, const void* wt, const float* bias, int act,
                           void* out_nhwc);
// The last BF16 hidden layer (cin 32 or 64 -> 64) with the last layer (64 -> 1) folded into
// its epilogue: wl2 holds the last layer's weights as a BF16 pair [hi, lo][tap padded to 16]
// [c]; qbuf receives nine FP32 tap planes (9 N n m floats), then the tap sum writes fo and,
// with obs, the X rows of Ybar.
bool conv_last_folds_bf16(int cin, int cout);
void launch_conv_mfma_bf16_last(hipStream_t s, Timer& t, int N, int n, int m, int cin, const void* in_nhwc,
                                const void* wt, const float* bias, int act, const uint16_t* wl2,
                                const float* bias_last, float* qbuf, FieldOut fo, const ObserveArgs* obs);
// The last FP8 hidden layer (cin 32 or 64 -> 64) with the last layer folded, as above.
void launch_conv_mfma_fp8_last(hipStream_t s, Timer& t, int N, int n, int m, int cin, const void* in_nhwc,
                               const unsigned* amax_in, const uint8_t* wq, const float* ws, const float* bias,
                               int act, const uint16_t* wl2, const float* bias_last, float* qbuf, FieldOut fo,
                               const ObserveArgs* obs);
// FP8 hidden layer: BF16 NHWC in and out, input scale from *amax_in (largest |x| of the
// input layer), weights wq [cout][K padded to 128] e4m3 with per-channel scales ws;
// folds the largest |output| into *amax_out.
bool conv_mfma_fp8_supported(int cin, int cout);
void launch_conv_mfma_fp8(hipStream_t s, Timer& t, int kclass, int N, int n, int m, int cin, int cout,
                          const void* in_nhwc, const unsigned* amax_in, const uint8_t* wq, const float* ws,
                          const float* bias, int act, void* out_nhwc, unsigned* amax_out);
void launch_zero_u32(hipStream_t s, Timer& t, unsigned* p, int count);

// Hidden layers on MFMA (FP32).  wk holds the weights as [tap*cin + c][cout].
// Whether a handle with this configuration runs its batched rollouts in BF16, and the
// floats each of its two activation buffers holds.
bool bf16_rollout_possible(const oic_config& c);
size_t activation_floats(const oic_config& c);
// Device bytes a handle created with c holds (the serving admission footprint).
size_t handle_bytes(const oic_config& c);
// Device bytes of one slot of a group created with c (the stride of its grouped launches).
size_t group_slab_bytes(const oic_config& c);
bool conv_mfma_supported(int cin, int cout);
void launch_conv_mfma(hipStream_t s, Timer& t, int kclass, int N, int n, int m, int cin, int cout,
                      const float* in_nhwc, const float* wk, const float* bias, int act,
                      float* out_nhwc);

// The FP32 rollout of Eq. (1) through the layer kernels above: the lift fused into the
// first layer where that kernel exists (else a separate lift), MFMA hidden layers where
// Wk (weights as [tap*cin + c][cout]) is given (else the direct kernel on W in
// [cout][cin][3][3] order), the tiled last layer where it exists.  act0/act1 hold
// batch*n*m*max(hidden widths, 2) floats each.  With `obs`, the first and last layers
// also write the side outputs it names; returns ROLL_X_OBSERVED | ROLL_U_ASSEMBLED for
// what was written.
enum { ROLL_X_OBSERVED = 1, ROLL_U_ASSEMBLED = 2 };
struct Fp32Net {
  const float* B;
  const float* W[OIC_MAX_LAYERS];
  const float* Wk[OIC_MAX_LAYERS];
  const float* bias[OIC_MAX_LAYERS];
};
int rollout_fp32(hipStream_t s, Timer& t, const oic_config& c, const Fp32Net& net, float* act0,
                 float* act1, int batch, FieldRef X, FieldRef U, FieldOut out,
                 const ObserveArgs* obs = nullptr);

// Statistics and update.
void launch_means(hipStream_t s, Timer& t, const float* A, int rows, int N, int m, float* mean);
void launch_means_f64(hipStream_t s, Timer& t, const float* A, int rows, int N, int m, double* mean);
// S[a][b] (FP64, (Ma+ny) x p): sum over columns of left row a times the FP64-centred Ybar
// row b; left rows are the first Ma trajectory rows followed by the first ny rows of Ybar.
// f32: the products on the FP32 matrix cores (right operand rounded to FP32 after
// centring, FP32 sums over at most 256 columns, FP64 beyond), for the mixed-precision modes.
// Yc: Ybar already centred (FP32, p x N*m, from launch_center) for the FP32-matrix-core
// products, or null to centre inside the product kernel.  b3 (with f32 and Yc): the FP32
// products as three BF16 matrix-core products of split operands (about 2^-16 relative
// per product), for the BF16 and FP8 modes.
void launch_stats(hipStream_t s, Timer& t, const Dims& d, const float* traj, int Ma, int ny,
                  const float* Y, const double* muY, double* part, size_t part_cap, double* S, bool f32 = false,
                  const float* Yc = nullptr, bool b3 = false);
// Rc[b][c] = R[b][c] - mu[b][c mod m] (FP64 subtraction, FP32 result) for rows x NM floats
// (rows * NM divisible by 4).
void launch_center(hipStream_t s, Timer& t, const float* R, int rows, int NM, int m, const double* mu,
                   float* Rc);
// The same sums against an arbitrary right operand, times scale: S[a][b] = scale *
// sum_c L[a][c] (R[b][c] - muR[b][c mod m]) for the nr rows of R (row length N*m), S
// with leading dimension nr.  part_cap must hold at least (Ma + ny) * nr doubles.
void launch_cross(hipStream_t s, Timer& t, const Dims& d, const float* traj, int Ma, int ny,
                  const float* Y, const float* R, int nr, const double* muR, double* part, size_t part_cap,
                  double* S, double scale, bool f32 = false, const float* Rc = nullptr, bool b3 = false);
// FP64 Cholesky factor of the p x p Syy; flag is set to 1 when a pivot is not positive
// and finite.  p <= 90 (one workgroup, LDS): Sinv = (Sigma^Y)^{-1}, Syy untouched.
// p > 90 (blocked, chip-wide): Syy is overwritten by L in its lower triangle and
// Lwork receives the inverses of its 64 x 64 diagonal blocks; Sinv is not written.
// Lwork holds 2 p (p+1) doubles.
void launch_chol(hipStream_t s, Timer& t, int p, double* Syy, double* Lwork, double* Sinv, int* flag);
// true when Sigma^Y (p x p) is factored by the blocked multi-launch path rather than in one workgroup
bool chol_blocked(int p);
// K = Sxy (Sigma^Y)^{-1} (Ma x p, FP64 arithmetic, FP32 result), from Sinv for p <= 90
// and from L (lower triangle of the factored Syy) and its diagonal-block inverses
// (Lwork) otherwise; skipped when flag is set.
void launch_gain(hipStream_t s, Timer& t, int p, int Ma, const double* Sxy, const double* Sinv,
                 const double* L, const double* Linv, float* K, const int* flag);
// Analysis of the first Ma trajectory rows (in place).
// b3: the products as three BF16 matrix-core products of split operands (BF16 / FP8 modes);
// scratch (scratch_bytes, free during the call) then receives the split gain, or the update
// splits the gain rows itself where scratch is null or too small.
void launch_update(hipStream_t s, Timer& t, const Dims& d, float* traj, int Ma, const float* K,
                   const float* Y, const float* xref_t, bool b3 = false, void* scratch = nullptr,
                   size_t scratch_bytes = 0);
void launch_extract(hipStream_t s, Timer& t, const Dims& d, const float* mu_traj, float* Uout,
                    float* Xout, float* Uprev);

}  // namespace oic

// Launch `kernel` on `stream`, bracketed by timing events of class `cls` when enabled.
// A kernel without a grouped form is not launched inside a group (see LaunchGroup).
#define OIC_LAUNCH(timer, cls, stream, kernel, grid, block, shmem, ...)          \
  do {                                                                         \
    if (::oic::launch_group().slots > 1) {                                     \
      ::oic::launch_group().unsupported = true;                                \
      break;                                                                   \
    }                                                                          \
    int oic_ti_ = (timer).begin((cls), (stream));                              \
    hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);       \
    (timer).end(oic_ti_, (stream));                                            \
  } while (0)

// Launch a kernel that has a grouped form (its last parameter is a Grp, its body starts
// with OIC_GROUP_ENTER): the grid is repeated over the calling thread's group slots.
#define OIC_GLAUNCH(timer, cls, stream, kernel, grid, block, shmem, ...)                 \
  do {                                                                                 \
    const ::oic::LaunchGroup& oic_lg_ = ::oic::launch_group();                         \
    dim3 oic_gr_ = (grid);                                                             \
    oic_gr_.z *= oic_lg_.slots;                                                        \
    int oic_ti_ = (timer).begin((cls), (stream));                                      \
    hipLaunchKernelGGL(kernel, oic_gr_, block, shmem, stream, __VA_ARGS__, oic_lg_.g); \
    (timer).end(oic_ti_, (stream));                                                    \
  } while (0)

// First statement of a kernel with a grouped form: leave if this slot is not active,
// else the byte offset of this slot's buffers is oic_goff_ (move each address with
// OIC_GSH).
#define OIC_GROUP_ENTER(grp)                                          \
  if ((grp).active && !(grp).active[blockIdx.z]) return;              \
  const unsigned long long oic_goff_ = (unsigned long long)blockIdx.z * (grp).stride
#define OIC_GSH(x) x = ::oic::gshift(x, oic_goff_)
