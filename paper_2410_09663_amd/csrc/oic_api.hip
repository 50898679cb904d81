// liboic: C ABI and host orchestration of one Kalman-MPC solve (Algorithm 1).
//
// Per solve, on one stream:
//   init slice k (line 4)                      k_init_slice0
//   for t = k+1..k+H (line 5):
//     forecast X rows through the CNN (15b)   k_lift, conv layers (last one writes slice t)
//     forecast U rows, U_t = U_{t-1} + W_t    k_assemble_u
//     perturbed observations (12)             k_observe
//     means of slices k..t and of Ybar (11)   k_means
//     pooled cross-covariances (13b,c)        k_stats (+ split-K reduction)
//     Cholesky + gain (14b)                   k_chol, k_gain_rows (FP64)
//     analysis of all slices k..t (14b)       k_update
//   smoothed means of every slice (line 13)    k_means, k_extract
// The stream is synchronised once at the end to check the positive-definiteness
// flag before any output is written.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "oic_internal.h"

// The buffer of the allocation-free rollout (oic_cnn_forward_noalloc): its intermediate
// activations and FP8 maxima.  Every GPU the library runs on holds one copy until the
// process ends.  In host code this name is a host-side stand-in, not a device address:
// host code uses the per-device address that hipGetSymbolAddress returns (scratch_on).
static __device__ __align__(256) unsigned char scratch[OIC_NOALLOC_SCRATCH_BYTES];

namespace oic {

const char* const kKernelClassNames[KC_COUNT] = {
    "noise", "init", "lift", "conv_first", "conv_mid", "conv_last", "assemble", "observe",
    "means", "stats", "stats_reduce", "chol", "gain", "update", "extract", "copy"};

LaunchGroup& launch_group() {
  thread_local LaunchGroup g;
  return g;
}

void Timer::reset() {
  cursor = 0;
  pending_class.clear();
  for (int c = 0; c < KC_COUNT; ++c) {
    launches[c] = 0;
    total_ms[c] = 0.0;
  }
}

int Timer::begin(int c, hipStream_t s) {
  if (!enabled) return -1;
  if (2 * cursor + 2 > pool.size()) {
    for (int k = 0; k < 64; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      pool.push_back(e);
    }
  }
  const int idx = (int)cursor++;
  pending_class.push_back(c);
  hipEventRecord(pool[2 * idx], s);
  return idx;
}

void Timer::end(int idx, hipStream_t s) {
  if (idx < 0) return;
  hipEventRecord(pool[2 * idx + 1], s);
}

void Timer::harvest() {
  for (size_t k = 0; k < cursor; ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pool[2 * k], pool[2 * k + 1]) == hipSuccess) {
      total_ms[pending_class[k]] += ms;
      launches[pending_class[k]] += 1;
    }
  }
  cursor = 0;
  pending_class.clear();
}

void Timer::destroy() {
  for (auto e : pool) hipEventDestroy(e);
  pool.clear();
}

}  // namespace oic

using namespace oic;

struct oic_ctx {
  oic_config cfg{};
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  Timer timer;

  // surrogate
  bool weights_set = false;
  float* dB = nullptr;
  float* dW[OIC_MAX_LAYERS] = {};
  float* dWk[OIC_MAX_LAYERS] = {};     // [tap*cin + c][cout] FP32 copies for the MFMA layers
  uint16_t* dWb[OIC_MAX_LAYERS] = {};  // [cout][tap*cin + c] BF16 copies for the BF16 rollout
  uint16_t* dWl2 = nullptr;            // last layer as a BF16 pair [hi, lo][16 taps][c] (folded BF16 rollout)
  uint8_t* dWq[OIC_MAX_LAYERS] = {};   // [cout][tap*cin + c, zero-padded to 128] e4m3 for FP8
  float* dWs[OIC_MAX_LAYERS] = {};     // per-output-channel scales of dWq
  unsigned* amax = nullptr;            // per-layer activation maxima of an FP8 rollout
  float* dBias[OIC_MAX_LAYERS] = {};
  int cmax = 2;

  // solve buffers (capacity max_N, max_H)
  float* traj = nullptr;
  float* Y = nullptr;
  float* act[2] = {nullptr, nullptr};
  size_t act_floats = 0;  // capacity of each activation buffer in floats
  float* mu_traj = nullptr;
  double* muY = nullptr;  // FP64 means of Ybar
  double* S = nullptr;     // Sigma^{XY} (Ma x p)
  double* Syy = nullptr;   // Sigma^Y (p x p)
  double* Sinv = nullptr;  // (Sigma^Y)^{-1}
  hipStream_t side = nullptr;            // the gain solve overlaps Sigma^{XY} on this stream
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  double* part = nullptr;   // split-K partial sums of the statistics
  size_t part_cap = 0;      // its size in doubles
  double* Lwork = nullptr;
  float* K = nullptr;
  int* flag = nullptr;
  float* Z[5] = {};  // 0 init (N,l,m); 1 W (H,N,l,m); 2 V_X (H,N,n,m); 3 V_U (H,N,l,m); 4 eps (H,N,m)
  // barrier-observed constraint (one extra row of Ybar), off unless set
  bool con_on = false;
  float* con_a = nullptr;  // [aX (n)][aU (l)]
  float con_b = 0.f, con_alpha = 1.f, con_beta = 1.f, con_rz = 1.f;
  float* Uprev = nullptr;
  float* Uprev_new = nullptr;
  float* fac = nullptr;  // [Q factor (l*l)][R factor (n*n)]
  bool q_diag = true, r_diag = true;
  std::vector<float> q_cached, r_cached;  // inputs the factors were computed from
  float* io = nullptr;                    // staging for host-memory inputs and outputs
  size_t io_floats = 0;
  float* out_stage = nullptr;             // solve outputs before the success check
  uint64_t* dseed = nullptr;              // device copy of the solve's seed
  uint64_t* hseed = nullptr;              // pinned host staging for it

  // optional covariance outputs (Eqs. (14c), (15d)-(15f)): per horizon step the pooled
  // covariance of all stored trajectory rows before and after the analysis
  bool want_cov = false;
  double* cov_prior = nullptr;
  double* cov_post = nullptr;
  size_t cov_cap = 0;       // doubles in each of cov_prior / cov_post
  double* mu64 = nullptr;   // FP64 means of the trajectory rows
  size_t mu64_cap = 0;

  // device address of the library-wide allocation-free scratch buffer on this handle's
  // device (oic_cnn_forward_noalloc), or null if it could not be obtained
  unsigned char* scratch = nullptr;

  // A slot of a group (oic_group_create): every device buffer, the weights included, is
  // carved from `slab` (slab_cap bytes) in a fixed order, so that it sits at the same
  // offset as in the group's other slots.  The group owns the memory and the handle.
  char* slab = nullptr;
  size_t slab_cap = 0, slab_used = 0;

  // replay of the per-solve kernel sequence
  bool use_graph = true;
  hipGraphExec_t gexec = nullptr;
  int gN = 0, gH = 0;
  bool gSeeded = false;
};

// Handles of one configuration whose buffers lie in equal slabs of one allocation, so
// that one launch per kernel serves any subset of them (see Grp).
struct oic_group {
  oic_config cfg{};
  int slots = 0;
  size_t slab = 0;         // bytes per slot (the stride of the grouped launches)
  char* region = nullptr;  // slots x slab bytes
  std::vector<oic_ctx*> h;
  int* dactive = nullptr;  // device: 1 for the slots of the batch being solved
  int* hactive = nullptr;  // pinned staging of dactive
  int* hflags = nullptr;   // pinned: each slot's positive-definiteness flag after a batch
  hipGraphExec_t gexec = nullptr;  // the captured grouped solve and its key
  int gN = 0, gH = 0;
  bool gSeeded = false, gQd = true, gRd = true;
  std::string err;
};

namespace {

// Held while a solve is captured into a graph and while any handle creates or frees
// device resources (memory, streams, events, graphs): a resource call from another
// thread in the middle of a capture can invalidate that capture.
std::mutex& resource_mutex() {
  static std::mutex m;
  return m;
}

#define HIP_TRY(expr)                                                        \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess) {                                                  \
      h->err = std::string(#expr) + ": " + hipGetErrorString(e_);            \
      return OIC_EDEVICE;                                                    \
    }                                                                        \
  } while (0)

int fail(oic_ctx* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

// Forget the captured solve: the graph holds kernel arguments (buffer addresses, the
// layout of the Q and R factors) that a change of weights or factors makes stale.  The
// caller holds resource_mutex().
void drop_graph(oic_ctx* h) {
  if (h->gexec) {
    hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
}

// Device address of `scratch` on `device` (the current device), looked up once per device;
// null if the lookup failed.  The caller holds resource_mutex().
unsigned char* scratch_on(int device) {
  static std::vector<unsigned char*> addr;
  static std::vector<char> looked_up;
  if (device < 0) return nullptr;
  if ((size_t)device >= addr.size()) {
    addr.resize(device + 1, nullptr);
    looked_up.resize(device + 1, 0);
  }
  if (!looked_up[device]) {
    looked_up[device] = 1;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess)
      addr[device] = static_cast<unsigned char*>(p);
    else
      (void)hipGetLastError();  // the failure is reported by the entry point that needs it
  }
  return addr[device];
}

bool finite_all(const float* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

size_t noise_floats(const oic_config& c, int kind) {
  const size_t N = c.max_N, H = c.max_H, m = c.m;
  switch (kind) {
    case 0: return N * c.l * m;
    case 1: return H * N * c.l * m;
    case 2: return H * N * c.n * m;
    case 4: return H * N * m;
    default: return H * N * c.l * m;
  }
}

// Lower Cholesky factor in FP64 on the host; returns false if not SPD.
bool host_cholesky(const float* A, int k, std::vector<double>& L) {
  L.assign((size_t)k * k, 0.0);
  for (int j = 0; j < k; ++j) {
    double s = A[(size_t)j * k + j];
    for (int c = 0; c < j; ++c) s -= L[(size_t)j * k + c] * L[(size_t)j * k + c];
    if (!(s > 0.0) || !std::isfinite(s)) return false;
    const double d = sqrt(s);
    L[(size_t)j * k + j] = d;
    for (int i = j + 1; i < k; ++i) {
      double v = A[(size_t)i * k + j];
      for (int c = 0; c < j; ++c) v -= L[(size_t)i * k + c] * L[(size_t)j * k + c];
      L[(size_t)i * k + j] = v / d;
    }
  }
  return true;
}

bool is_symmetric(const float* A, int k) {
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < i; ++j)
      if (A[(size_t)i * k + j] != A[(size_t)j * k + i]) return false;
  return true;
}

bool is_diagonal(const float* A, int k) {
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j)
      if (i != j && A[(size_t)i * k + j] != 0.f) return false;
  return true;
}

// Factor Q and R (host), upload the FP32 factors (or diagonal scales) when they changed.
int prepare_factors(oic_ctx* h, const float* Q, const float* R) {
  const int l = h->cfg.l, n = h->cfg.n;
  if (!Q || !R) return fail(h, OIC_EINVAL, "Q and R must be non-NULL host pointers");
  if (!finite_all(Q, (size_t)l * l) || !finite_all(R, (size_t)n * n))
    return fail(h, OIC_EINVAL, "Q or R has a non-finite entry");
  const bool same = h->q_cached.size() == (size_t)l * l && h->r_cached.size() == (size_t)n * n &&
                    memcmp(h->q_cached.data(), Q, sizeof(float) * l * l) == 0 &&
                    memcmp(h->r_cached.data(), R, sizeof(float) * n * n) == 0;
  if (same) return OIC_OK;
  if (!is_symmetric(Q, l) || !is_symmetric(R, n))
    return fail(h, OIC_EINVAL, "Q and R must be symmetric");
  std::vector<double> Lq, Lr;
  if (!host_cholesky(Q, l, Lq)) return fail(h, OIC_EINVAL, "Q is not positive definite");
  if (!host_cholesky(R, n, Lr)) return fail(h, OIC_EINVAL, "R is not positive definite");
  std::vector<float> f((size_t)l * l + (size_t)n * n, 0.f);
  const bool qd = is_diagonal(Q, l), rd = is_diagonal(R, n);
  if (qd != h->q_diag || rd != h->r_diag) {
    // the captured noise kernels read the factors as diagonal scales or dense triangles
    std::lock_guard<std::mutex> guard(resource_mutex());
    drop_graph(h);
  }
  h->q_diag = qd;
  h->r_diag = rd;
  // Diagonal factors are stored as the first l (n) entries; dense ones row-major.
  if (h->q_diag)
    for (int a = 0; a < l; ++a) f[a] = (float)Lq[(size_t)a * l + a];
  else
    for (size_t e = 0; e < (size_t)l * l; ++e) f[e] = (float)Lq[e];
  float* fr = f.data() + (size_t)l * l;
  if (h->r_diag)
    for (int a = 0; a < n; ++a) fr[a] = (float)Lr[(size_t)a * n + a];
  else
    for (size_t e = 0; e < (size_t)n * n; ++e) fr[e] = (float)Lr[e];
  HIP_TRY(hipMemcpyAsync(h->fac, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->q_cached.assign(Q, Q + (size_t)l * l);
  h->r_cached.assign(R, R + (size_t)n * n);
  return OIC_OK;
}

// Noise source over the handle's factors, stored as diagonal scales (q_diag / r_diag)
// or dense triangles.
NoiseRef noise_ref(oic_ctx* h, const float* Z, bool is_q, bool q_diag, bool r_diag) {
  NoiseRef r;
  r.Z = Z;
  const int l = h->cfg.l;
  if (is_q) {
    r.rows = l;
    r.diag = q_diag ? h->fac : nullptr;
    r.L = q_diag ? nullptr : h->fac;
  } else {
    r.rows = h->cfg.n;
    const float* fr = h->fac + (size_t)l * l;
    r.diag = r_diag ? fr : nullptr;
    r.L = r_diag ? nullptr : fr;
  }
  return r;
}

template <typename T>
int dalloc(oic_ctx* h, T** p, size_t count) {
  if (count == 0) count = 1;
  if (h->slab) {
    const size_t bytes = (count * sizeof(T) + 255) / 256 * 256;
    if (h->slab_used + bytes > h->slab_cap) {
      *p = nullptr;
      h->err = "the group slot's buffers exceed its slab";
      return OIC_ENOMEM;
    }
    *p = reinterpret_cast<T*>(h->slab + h->slab_used);
    h->slab_used += bytes;
    return OIC_OK;
  }
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    h->err = std::string("hipMalloc of ") + std::to_string(count * sizeof(T)) + " bytes failed: " +
             hipGetErrorString(e);
    return OIC_ENOMEM;
  }
  return OIC_OK;
}

void free_all(oic_ctx* h) {
  auto f = [h](void* p) {
    if (p && !h->slab) hipFree(p);  // a group slot's buffers are the group's
  };
  f(h->dB);
  for (int k = 0; k < OIC_MAX_LAYERS; ++k) {
    f(h->dW[k]);
    f(h->dWk[k]);
    f(h->dWb[k]);
    f(h->dWq[k]);
    f(h->dWs[k]);
    f(h->dBias[k]);
  }
  f(h->amax);
  f(h->dWl2);
  f(h->traj);
  f(h->Y);
  f(h->act[0]);
  f(h->act[1]);
  f(h->mu_traj);
  f(h->muY);
  f(h->S);
  f(h->Syy);
  f(h->Sinv);
  if (h->ev_fork) hipEventDestroy(h->ev_fork);
  if (h->ev_join) hipEventDestroy(h->ev_join);
  if (h->side) hipStreamDestroy(h->side);
  f(h->part);
  f(h->Lwork);
  f(h->K);
  f(h->flag);
  for (int k = 0; k < 5; ++k) f(h->Z[k]);
  f(h->con_a);
  f(h->Uprev);
  f(h->Uprev_new);
  f(h->fac);
  f(h->io);
  f(h->out_stage);
  f(h->cov_prior);
  f(h->cov_post);
  f(h->mu64);
  f(h->dseed);
  if (h->hseed) hipHostFree(h->hseed);
  if (h->gexec) hipGraphExecDestroy(h->gexec);
  h->gexec = nullptr;
}

}  // namespace

namespace oic {

// Whether a handle's batched rollouts run with BF16 activations: BF16 or FP8 precision
// was requested and every layer has a kernel for it (first 2->C and last C->1 with
// BF16 storage; hidden C->C' in BF16, or in FP8 for the FP8 precision).
bool bf16_rollout_possible(const oic_config& c) {
  const int L = c.n_layers;
  if ((c.precision != OIC_PREC_BF16 && c.precision != OIC_PREC_FP8) || L < 2) return false;
  if (!conv_first_supported(c.channels[1], c.l) || !conv_last_supported(c.channels[L - 1])) return false;
  for (int k = 1; k < L - 1; ++k) {
    const int ci = c.channels[k], co = c.channels[k + 1];
    if (c.precision == OIC_PREC_FP8 ? !conv_mfma_fp8_supported(ci, co) : !conv_mfma_bf16_supported(ci, co))
      return false;
  }
  return true;
}

size_t activation_floats(const oic_config& c) {
  size_t cmax = 2;
  for (int k = 1; k < c.n_layers; ++k) cmax = std::max(cmax, (size_t)c.channels[k]);
  const size_t full = (size_t)c.max_N * c.n * c.m * cmax;
  if (!bf16_rollout_possible(c)) return full;
  // BF16 activations for batched rollouts; FP32 only for the one-field plant step
  return std::max((full + 1) / 2, (size_t)c.n * c.m * cmax);
}

// Device bytes oic_create allocates for c (plus the weights oic_set_weights adds),
// buffer by buffer as in oic_create.
size_t handle_bytes(const oic_config& c) {
  const size_t N = c.max_N, Hs = c.max_H + 1, n = c.n, m = c.m, l = c.l, rr = n + l, p = n + l + 1;
  const size_t NM = N * m, Ma = Hs * rr;
  size_t floats = Hs * rr * NM + p * NM + 2 * activation_floats(c) + Ma * m + Ma * p;
  for (int k = 0; k < 5; ++k) floats += noise_floats(c, k);
  floats += (n + l) + 2 * l * m + l * l + n * n;                                  // con_a, U_prev, factors
  floats += n * m + Hs * n * m + l * m + N * (n + l) * m + N * n * m + Hs * (l + n) * m;  // staging
  size_t doubles = p * m + (Ma + p) * p + std::max(32 * (Ma + p) * p, Ma * p) + 2 * p * (p + 1) + 2 * p * p;
  size_t weights = n * l * 4;
  for (int k = 0; k < c.n_layers; ++k)  // FP32, MFMA-layout FP32, BF16 and FP8 copies at most
    weights += (size_t)c.channels[k + 1] * c.channels[k] * 9 * 11 + (size_t)c.channels[k + 1] * 8;
  return 4 * floats + 8 * doubles + weights + 4096;
}

// Bytes of one group slot: handle_bytes with every buffer rounded up to 256 bytes,
// rounded up to 2 MiB.
size_t group_slab_bytes(const oic_config& c) {
  const size_t buffers = 32 + 8 * (size_t)OIC_MAX_LAYERS;
  const size_t b = handle_bytes(c) + 256 * buffers;
  return (b + (2u << 20) - 1) / (2u << 20) * (2u << 20);
}

}  // namespace oic

namespace {

enum RolloutMode { RM_FP32 = 0, RM_BF16 = 1, RM_FP8 = 2 };

// The handle's batched rollout mode once its weights are set.
RolloutMode rollout_mode(oic_ctx* h) {
  const oic_config& c = h->cfg;
  if (!h->weights_set || !bf16_rollout_possible(c)) return RM_FP32;
  return c.precision == OIC_PREC_FP8 ? RM_FP8 : RM_BF16;
}

// Runs the CNN of Eq. (1) on `batch` fields given as strided sources, writing the
// single output channel to `out`, in the given mode (the plant step always uses FP32).
// With `obs`, the first and last layers also write the side outputs it names where they
// run as the tiled kernels; returns ROLL_X_OBSERVED | ROLL_U_ASSEMBLED for what was written.
// The activations go to act0/act1 (each act_cap floats) and the FP8 maxima to amax (the
// handle's buffers unless given), with launches timed on tm (the handle's timer unless given).
int rollout(oic_ctx* h, int batch, FieldRef X, FieldRef U, FieldOut out, RolloutMode mode,
            const ObserveArgs* obs = nullptr, float* act0 = nullptr, float* act1 = nullptr,
            unsigned* amax = nullptr, Timer* tm = nullptr, size_t act_cap = 0) {
  const oic_config& c = h->cfg;
  const int L = c.n_layers;
  float* act[2] = {act0 ? act0 : h->act[0], act1 ? act1 : h->act[1]};
  const size_t cap = act0 ? act_cap : h->act_floats;
  if (!amax) amax = h->amax;
  Timer& timer = tm ? *tm : h->timer;
  if (mode != RM_FP32) {
    const bool f8 = mode == RM_FP8;
    // per-layer activation maxima: slot k holds the largest |x| written by layer k
    if (f8) launch_zero_u32(h->stream, timer, amax, L * kAmaxSlots);
    launch_conv_first(h->stream, timer, batch, c.n, c.m, c.l, X, U, h->dB, c.channels[1], h->dW[0],
                      h->dBias[0], c.activation, act[1], true, act[0], f8 ? amax : nullptr, obs);
    int cur = 1;
    for (int k = 1; k < L - 1; ++k) {
      if (k == L - 2 && h->dWl2 && conv_last_folds_bf16(c.channels[k], c.channels[k + 1]) &&
          (size_t)9 * batch * c.n * c.m <= cap) {
        // the last hidden layer with the last layer folded into its epilogue
        if (f8)
          launch_conv_mfma_fp8_last(h->stream, timer, batch, c.n, c.m, c.channels[k], act[cur],
                                    amax + (size_t)(k - 1) * kAmaxSlots,
                                    h->dWq[k], h->dWs[k], h->dBias[k], c.activation, h->dWl2, h->dBias[L - 1],
                                    act[1 - cur], out, obs);
        else
          launch_conv_mfma_bf16_last(h->stream, timer, batch, c.n, c.m, c.channels[k], act[cur], h->dWb[k],
                                     h->dBias[k], c.activation, h->dWl2, h->dBias[L - 1], act[1 - cur], out, obs);
        return obs ? ROLL_X_OBSERVED | (obs->U_cur ? ROLL_U_ASSEMBLED : 0) : 0;
      }
      if (f8)
        launch_conv_mfma_fp8(h->stream, timer, KC_CONV_MID, batch, c.n, c.m, c.channels[k],
                             c.channels[k + 1], act[cur], amax + (size_t)(k - 1) * kAmaxSlots, h->dWq[k],
                             h->dWs[k], h->dBias[k], c.activation, act[1 - cur], amax + (size_t)k * kAmaxSlots);
      else
        launch_conv_mfma_bf16(h->stream, timer, KC_CONV_MID, batch, c.n, c.m, c.channels[k],
                              c.channels[k + 1], act[cur], h->dWb[k], h->dBias[k], c.activation,
                              act[1 - cur]);
      cur = 1 - cur;
    }
    launch_conv_last(h->stream, timer, batch, c.n, c.m, c.channels[L - 1], act[cur],
                     h->dW[L - 1], h->dBias[L - 1], out, true, obs);
    return obs ? ROLL_X_OBSERVED | (obs->U_cur ? ROLL_U_ASSEMBLED : 0) : 0;
  }
  Fp32Net net{};
  net.B = h->dB;
  for (int k = 0; k < L; ++k) {
    net.W[k] = h->dW[k];
    net.Wk[k] = h->dWk[k];
    net.bias[k] = h->dBias[k];
  }
  return rollout_fp32(h->stream, timer, c, net, act[0], act[1], batch, X, U, out, obs);
}

// OCP FP8 e4m3: bias 7, no infinities, largest finite 448.  The finite non-negative
// codes 0x00..0x7E are increasing in value.
const std::vector<float>& e4m3_table() {
  static const std::vector<float> table = [] {
    std::vector<float> t(127);
    for (int c = 0; c < 127; ++c) {
      const int e = c >> 3, mant = c & 7;
      t[c] = e == 0 ? std::ldexp((float)mant / 8.0f, -6) : std::ldexp(1.0f + (float)mant / 8.0f, e - 7);
    }
    return t;
  }();
  return table;
}

float e4m3_value(uint8_t c) {
  const float v = e4m3_table()[c & 0x7F];
  return (c & 0x80) ? -v : v;
}

// The e4m3 code nearest to f, ties to the even code, saturating beyond 448 (found by
// bisection over the increasing codes).
uint8_t host_e4m3(float f) {
  const std::vector<float>& table = e4m3_table();
  const uint8_t sign = std::signbit(f) ? 0x80 : 0x00;
  const float a = std::fabs(f);
  if (!(a < table[126])) return sign | 0x7E;  // saturate (NaN does not occur: finite weights)
  int lo = 0, hi = 126;                       // table[lo] <= a < table[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (table[mid] <= a) lo = mid; else hi = mid;
  }
  const float dl = a - table[lo], dh = table[hi] - a;
  const int c = dl < dh ? lo : (dh < dl ? hi : ((lo & 1) ? hi : lo));
  return sign | (uint8_t)c;
}

uint16_t host_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, sizeof(u));
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Copies in the handle's memory mode on stream s (the handle's stream if null).
int copy_in(oic_ctx* h, float* dst, const float* src, size_t count, hipStream_t s = nullptr) {
  if (!s) s = h->stream;
  if (h->cfg.mem_mode == OIC_MEM_HOST)
    HIP_TRY(hipMemcpyAsync(dst, src, count * sizeof(float), hipMemcpyHostToDevice, s));
  else
    HIP_TRY(hipMemcpyAsync(dst, src, count * sizeof(float), hipMemcpyDeviceToDevice, s));
  return OIC_OK;
}

int copy_out(oic_ctx* h, float* dst, const float* src, size_t count, hipStream_t s = nullptr) {
  if (!s) s = h->stream;
  if (h->cfg.mem_mode == OIC_MEM_HOST)
    HIP_TRY(hipMemcpyAsync(dst, src, count * sizeof(float), hipMemcpyDeviceToHost, s));
  else
    HIP_TRY(hipMemcpyAsync(dst, src, count * sizeof(float), hipMemcpyDeviceToDevice, s));
  return OIC_OK;
}

// Offset (in doubles) of horizon step t's block in the covariance outputs: the blocks
// of steps 1..t-1, each ((s+1) rr)^2.
size_t cov_offset(int rr, int t) {
  size_t off = 0;
  for (int s = 1; s < t; ++s) off += (size_t)((s + 1) * rr) * ((s + 1) * rr);
  return off;
}

// out (Ma x Ma) = (lambda / N) sum_i A^i A^iT over the first Ma trajectory rows, with
// lambda = 1 / tr(Psi) = 1 / m, anomalies taken about the FP64 ensemble means.
void enqueue_cov(oic_ctx* h, const Dims& d, int Ma, double* out) {
  launch_means_f64(h->stream, h->timer, h->traj, Ma, d.N, d.m, h->mu64);
  launch_cross(h->stream, h->timer, d, h->traj, Ma, 0, h->Y, h->traj, Ma, h->mu64, h->part, h->part_cap, out,
               1.0 / ((double)d.m * d.N));
}

// Every kernel of one solve, in order, on the handle's stream.  Reads only handle-owned
// buffers (inputs and noise are copied in beforehand; the seed is in device memory),
// so the same sequence can be captured once and replayed.  `mode` is the rollout's
// arithmetic and q_diag / r_diag the layout of the noise factors; inside a group
// (launch_group) the launches serve every active slot.
void enqueue_solve(oic_ctx* h, const Dims& d, bool seeded, RolloutMode mode, bool q_diag, bool r_diag) {
  const oic_config& c = h->cfg;
  const int N = d.N, H = d.H, n = c.n, m = c.m, l = c.l, rr = d.rr(), p = d.p();
  const long long NM = d.NM();
  hipStream_t s = h->stream;
  float* dX0 = h->io;
  float* dRef = dX0 + (size_t)n * m;
  float* dUp = dRef + (size_t)(c.max_H + 1) * n * m;
  const size_t cnt[5] = {(size_t)N * l * m, (size_t)H * N * l * m, (size_t)H * N * n * m,
                         (size_t)H * N * l * m, (size_t)H * N * m};
  if (seeded)
    for (int k = 0; k < 4 + d.nc; ++k) launch_normals(s, h->timer, h->Z[k], cnt[k], h->dseed, (uint32_t)k);
  const float* const* Zd = h->Z;
  // Line 4: initial ensemble (also clears the failure flag).
  launch_init_slice0(s, h->timer, d, h->traj, dX0, dUp, noise_ref(h, Zd[0], true, q_diag, r_diag), h->flag);
  for (int t = 1; t <= H; ++t) {
    const size_t slice = (size_t)rr * NM;
    float* prev = h->traj + (size_t)(t - 1) * slice;
    float* cur = h->traj + (size_t)t * slice;
    // Line 6 / Eq. (15b): X rows of slice t through the CNN, from the analysed slice t-1.
    // Line 9 / Eq. (12) for the X rows rides along with the rollout's last layer; Eq. (4)
    // for the U rows of slice t (and their rows of Ybar) with its first layer while the
    // slice is small: for l*N*m above 2^17 the extra noise loads and stores in every
    // first-layer workgroup cost more than the separate launch saves.
    const bool small = (long long)l * NM <= (1LL << 17);
    const ObserveArgs oa{small ? cur + (size_t)n * NM : nullptr, h->Y, NM,
                         noise_ref(h, Zd[1] + (size_t)(t - 1) * N * l * m, true, q_diag, r_diag),
                         noise_ref(h, Zd[2] + (size_t)(t - 1) * N * n * m, false, q_diag, r_diag),
                         noise_ref(h, Zd[3] + (size_t)(t - 1) * N * l * m, true, q_diag, r_diag)};
    const int done = rollout(h, N, FieldRef{prev, m, NM}, FieldRef{prev + (size_t)n * NM, m, NM},
                             FieldOut{cur, m, NM}, mode, &oa);
    if (!(done & ROLL_U_ASSEMBLED)) launch_assemble_u(s, h->timer, d, h->traj, t, oa.w);
    launch_observe(s, h->timer, d, h->traj, t, h->Y, oa.vx, oa.vu, (done & ROLL_X_OBSERVED) ? n : 0,
                   (done & ROLL_U_ASSEMBLED) ? n : n + l);
    // Line 8 / Eqs. (15d)-(15f): covariance of the forecast trajectory (optional)
    if (h->want_cov) enqueue_cov(h, d, (t + 1) * rr, h->cov_prior + cov_offset(rr, t));
    // the barrier observation of the constraint, if one is set (actual value 0)
    if (d.nc)
      launch_constraint_row(s, h->timer, d, h->traj, t, h->Y, h->con_a, h->con_a + n, h->con_b, h->con_alpha,
                            h->con_beta, std::sqrt(h->con_rz), Zd[4] + (size_t)(t - 1) * N * m);
    // Eq. (13a): mean of Ybar in FP64.  The trajectory rows need no mean here: the
    // FP64-centred Ybar anomalies sum to zero, so sum_i X^i D^iT = sum_i A^i D^iT.
    const int Ma = (t + 1) * rr;
    launch_means_f64(s, h->timer, h->Y, p, N, m, h->muY);
    // Eq. (13b): Sigma^Y first; its Cholesky factor and inverse run on the side stream
    // while Eq. (13c), Sigma^{XY}, runs here.  Sigma^Y, which is factored, takes FP64
    // products in the FP32 mode; Sigma^{XY}, which enters the gain linearly, takes FP32
    // products folded into FP64 every 256 columns in every mode (twice the FP64 MFMA rate).
    const bool f32_stats = mode != RM_FP32;  // FP32 statistics in the BF16 / FP8 modes
    // the FP32 products take Ybar centred once per step (FP64 subtraction, FP32 result) in
    // the first activation buffer, which the rollout is done with until the next step
    const float* Yc = nullptr;
    if (NM % 4 == 0 && (size_t)p * NM <= h->act_floats) {
      launch_center(s, h->timer, h->Y, p, (int)NM, m, h->muY, h->act[0]);
      Yc = h->act[0];
    }
    // the BF16 / FP8 modes take the FP32 products as three BF16 products of split operands
    const bool b3 = f32_stats;
    launch_stats(s, h->timer, d, h->traj, 0, p, h->Y, h->muY, h->part, h->part_cap, h->Syy, f32_stats, Yc, b3);
    hipEventRecord(h->ev_fork, s);
    hipStreamWaitEvent(h->side, h->ev_fork, 0);
    launch_chol(h->side, h->timer, p, h->Syy, h->Lwork, h->Sinv, h->flag);
    hipEventRecord(h->ev_join, h->side);
    launch_stats(s, h->timer, d, h->traj, Ma, 0, h->Y, h->muY, h->part, h->part_cap, h->S, true, Yc, b3);
    hipStreamWaitEvent(s, h->ev_join, 0);
    // Eq. (14b): gain, then line 10: analysis of every stored slice.
    launch_gain(s, h->timer, p, Ma, h->S, h->Sinv, h->Syy, h->Lwork, h->K, h->flag);
    // (the split-K partials of the statistics are consumed by now: their buffer takes the
    // split gain of the BF16 / FP8 update)
    launch_update(s, h->timer, d, h->traj, Ma, h->K, h->Y, dRef + (size_t)t * n * m, b3, h->part,
                  h->part_cap * sizeof(double));
    // Line 11 / Eq. (14c): covariance after the analysis (optional)
    if (h->want_cov) enqueue_cov(h, d, Ma, h->cov_post + cov_offset(rr, t));
  }
  // Line 13: smoothed means of every slice.
  launch_means(s, h->timer, h->traj, (H + 1) * rr, N, m, h->mu_traj);
  float* sU = h->out_stage;
  float* sX = sU + (size_t)(c.max_H + 1) * l * m;
  launch_extract(s, h->timer, d, h->mu_traj, sU, sX, h->Uprev_new);
}

// First stage of a solve: checks the arguments, factors Q and R, and queues the copies
// of the inputs (and of explicit noise, or the seed) into the handle's buffers on stream
// s.  Sets d and whether the solve draws its own noise.
int solve_begin(oic_ctx* h, const oic_solve_args* a, hipStream_t s, Dims& d, bool& seeded) {
  if (!h) return OIC_EINVAL;
  h->err.clear();
  if (!a) return fail(h, OIC_EINVAL, "NULL argument block");
  const oic_config& c = h->cfg;
  if (!h->weights_set) return fail(h, OIC_EINVAL, "weights not set (call oic_set_weights first)");
  const int N = a->N, H = a->horizon;
  if (N < 2) return fail(h, OIC_EINVAL, "N must be at least 2");
  if (H < 1) return fail(h, OIC_EINVAL, "horizon must be at least 1");
  if (N > c.max_N || H > c.max_H)
    return fail(h, OIC_ENOMEM, "N or horizon exceeds the capacity the handle was created with");
  if ((long long)(N - 1) * c.m < c.n + c.l + (h->con_on ? 1 : 0))
    return fail(h, OIC_EINVAL, "(N-1)*m is below the observation rows: Sigma^Ybar cannot be positive definite");
  if (!a->X0 || !a->reference || !a->U_out) return fail(h, OIC_EINVAL, "NULL X0, reference or U_out");
  const bool explicit_noise = a->Z_init || a->Z_W || a->Z_VX || a->Z_VU;
  if (explicit_noise && !(a->Z_init && a->Z_W && a->Z_VX && a->Z_VU))
    return fail(h, OIC_EINVAL, "noise arrays must be all NULL or all non-NULL");
  if (explicit_noise && h->con_on && !a->Z_VZ)
    return fail(h, OIC_EINVAL, "a constraint is set: explicit noise needs Z_VZ too");
  if (c.mem_mode == OIC_MEM_HOST) {
    if (!finite_all(a->X0, (size_t)c.n * c.m) ||
        !finite_all(a->reference, (size_t)(H + 1) * c.n * c.m))
      return fail(h, OIC_EINVAL, "X0 or reference has a non-finite entry");
  }
  int rc = prepare_factors(h, a->Q, a->R);
  if (rc) return rc;

  d = Dims{c.n, c.m, c.l, N, H};
  d.nc = h->con_on ? 1 : 0;
  const int n = c.n, m = c.m, l = c.l;

  // Inputs into device memory.
  float* dX0 = h->io;
  float* dRef = dX0 + (size_t)n * m;
  float* dUp = dRef + (size_t)(c.max_H + 1) * n * m;
  const bool dev = c.mem_mode == OIC_MEM_DEVICE;
  if (dev) {
    // device pointers: X0, the reference window, U_prev and the seed in one launch
    const CopyJob in[3] = {{a->X0, dX0, (long long)n * m},
                           {a->reference, dRef, (long long)(H + 1) * n * m},
                           {a->U_prev ? a->U_prev : h->Uprev, dUp, (long long)l * m}};
    launch_copy_jobs(s, h->timer, in, 3, nullptr, a->seed, explicit_noise ? nullptr : h->dseed);
  } else {
    if ((rc = copy_in(h, dX0, a->X0, (size_t)n * m, s))) return rc;
    if ((rc = copy_in(h, dRef, a->reference, (size_t)(H + 1) * n * m, s))) return rc;
    if (a->U_prev) {
      if ((rc = copy_in(h, dUp, a->U_prev, (size_t)l * m, s))) return rc;
    } else {
      HIP_TRY(hipMemcpyAsync(dUp, h->Uprev, (size_t)l * m * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
  }
  const size_t cnt[5] = {(size_t)N * l * m, (size_t)H * N * l * m, (size_t)H * N * n * m,
                         (size_t)H * N * l * m, (size_t)H * N * m};
  const float* zsrc[5] = {a->Z_init, a->Z_W, a->Z_VX, a->Z_VU, a->Z_VZ};
  if (explicit_noise) {
    for (int k = 0; k < 4 + d.nc; ++k)
      if ((rc = copy_in(h, h->Z[k], zsrc[k], cnt[k], s))) return rc;
  } else if (!dev) {
    // (the pinned staging word is read by the copy engine later: one solve at a time
    // per handle)
    *h->hseed = a->seed;
    HIP_TRY(hipMemcpyAsync(h->dseed, h->hseed, sizeof(uint64_t), hipMemcpyHostToDevice, s));
  }
  seeded = !explicit_noise;
  return OIC_OK;
}

// Queues the outputs of a device-memory solve (and the carried U_prev) on stream s,
// skipped on the device when the positive-definiteness flag is set, then the flag into
// *flag_host (pinned or pageable host memory, read after s is synchronised).
int solve_end(oic_ctx* h, const oic_solve_args* a, hipStream_t s, int* flag_host) {
  const oic_config& c = h->cfg;
  const int H = a->horizon, n = c.n, m = c.m, l = c.l;
  float* sU = h->out_stage;
  float* sX = sU + (size_t)(c.max_H + 1) * l * m;
  if (c.mem_mode == OIC_MEM_DEVICE) {
    // outputs and the carried U_prev in one launch, which does nothing if the solve failed
    const CopyJob out[3] = {{sU, a->U_out, (long long)(H + 1) * l * m},
                            {sX, a->X_out, a->X_out ? (long long)(H + 1) * n * m : 0},
                            {h->Uprev_new, h->Uprev, (long long)l * m}};
    launch_copy_jobs(s, h->timer, out, 3, h->flag, 0, nullptr);
  }
  HIP_TRY(hipMemcpyAsync(flag_host, h->flag, sizeof(int), hipMemcpyDeviceToHost, s));
  return OIC_OK;
}

// Last stage, after stream s is synchronised: the flag's outcome, and the outputs of a
// host-memory solve.
int solve_finish(oic_ctx* h, const oic_solve_args* a, hipStream_t s, int flag) {
  const oic_config& c = h->cfg;
  const int H = a->horizon, n = c.n, m = c.m, l = c.l;
  if (flag) return fail(h, OIC_ENOTSPD, "Sigma^Ybar is not positive definite at some horizon step");
  if (c.mem_mode == OIC_MEM_HOST) {
    float* sU = h->out_stage;
    float* sX = sU + (size_t)(c.max_H + 1) * l * m;
    int rc;
    if ((rc = copy_out(h, a->U_out, sU, (size_t)(H + 1) * l * m, s))) return rc;
    if (a->X_out && (rc = copy_out(h, a->X_out, sX, (size_t)(H + 1) * n * m, s))) return rc;
    HIP_TRY(hipMemcpyAsync(h->Uprev, h->Uprev_new, (size_t)l * m * sizeof(float),
                           hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return OIC_OK;
}

// Captures enqueue_solve on stream s into *exec (replacing what it held).  The caller
// holds resource_mutex().
int capture_solve(oic_ctx* h, hipStream_t s, hipGraphExec_t* exec, const Dims& d, bool seeded, RolloutMode mode,
                  bool q_diag, bool r_diag) {
  if (*exec) {
    hipGraphExecDestroy(*exec);
    *exec = nullptr;
  }
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
  enqueue_solve(h, d, seeded, mode, q_diag, r_diag);
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamEndCapture(s, &g));
  hipError_t e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) {
    *exec = nullptr;
    return fail(h, OIC_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  return OIC_OK;
}

int solve_impl(oic_ctx* h, const oic_solve_args* a) {
  Dims d{};
  bool seeded = false;
  int rc = solve_begin(h, a, h ? h->stream : nullptr, d, seeded);
  if (rc) return rc;
  hipStream_t s = h->stream;
  const RolloutMode mode = rollout_mode(h);
  if (h->use_graph && !h->timer.enabled && !h->want_cov) {
    if (!h->gexec || h->gN != d.N || h->gH != d.H || h->gSeeded != seeded) {
      std::lock_guard<std::mutex> guard(resource_mutex());
      if ((rc = capture_solve(h, s, &h->gexec, d, seeded, mode, h->q_diag, h->r_diag))) return rc;
      h->gN = d.N;
      h->gH = d.H;
      h->gSeeded = seeded;
    }
    HIP_TRY(hipGraphLaunch(h->gexec, s));
  } else {
    enqueue_solve(h, d, seeded, mode, h->q_diag, h->r_diag);
  }
  int flag = 0;
  if ((rc = solve_end(h, a, s, &flag))) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  h->timer.harvest();
  return solve_finish(h, a, s, flag);
}

// Weight buffers of every layer that oic_set_weights fills for this configuration, in a
// fixed order (a group slot holds them from the start: a slot never allocates later, and
// its buffers keep the same offsets as the other slots').
int reserve_weights(oic_ctx* h) {
  const oic_config& c = h->cfg;
  int rc = dalloc(h, &h->dB, (size_t)c.n * c.l);
  for (int k = 0; k < c.n_layers && !rc; ++k) {
    const int cin = c.channels[k], cout = c.channels[k + 1];
    const size_t cnt = (size_t)cout * cin * 9;
    rc = dalloc(h, &h->dW[k], cnt);
    if (!rc && k < c.n_layers - 1 && conv_mfma_supported(cin, cout)) rc = dalloc(h, &h->dWk[k], cnt);
    if (!rc && c.precision == OIC_PREC_FP8 && k > 0 && k < c.n_layers - 1 && conv_mfma_fp8_supported(cin, cout)) {
      const size_t kd128 = ((size_t)9 * cin + 127) / 128 * 128;
      rc = dalloc(h, &h->dWq[k], (size_t)cout * kd128);
      if (!rc) rc = dalloc(h, &h->dWs[k], (size_t)cout);
    }
    if (!rc && c.precision == OIC_PREC_BF16 && k > 0 && k < c.n_layers - 1 && conv_mfma_bf16_supported(cin, cout))
      rc = dalloc(h, &h->dWb[k], cnt);
    if (!rc && (c.precision == OIC_PREC_BF16 || c.precision == OIC_PREC_FP8) && k == c.n_layers - 1 && k >= 2 &&
        cout == 1 && conv_last_folds_bf16(c.channels[k - 1], cin))
      rc = dalloc(h, &h->dWl2, (size_t)2 * 16 * cin);
    if (!rc) rc = dalloc(h, &h->dBias[k], (size_t)cout);
  }
  return rc;
}

// A new handle for c (the caller holds resource_mutex()).  With a slab, every device
// buffer comes from it (a group slot) and the weight buffers are reserved at once.
int create_handle(const oic_config& c, char* slab, size_t slab_cap, oic_ctx** out) {
  *out = nullptr;
  if (c.n < 4 || c.m < 4 || c.l < 1 || c.l > c.n || c.n_layers < 1 || c.n_layers > OIC_MAX_LAYERS ||
      c.max_N < 2 || c.max_H < 1 || (c.activation != OIC_ACT_TANH && c.activation != OIC_ACT_GELU) ||
      (c.precision != OIC_PREC_FP32 && c.precision != OIC_PREC_BF16 && c.precision != OIC_PREC_FP8) ||
      (c.mem_mode != OIC_MEM_HOST && c.mem_mode != OIC_MEM_DEVICE))
    return OIC_EINVAL;
  if (c.channels[0] != 2 || c.channels[c.n_layers] != 1) return OIC_EINVAL;
  // column indices of one trajectory row (N*m) are 32-bit in the kernels
  if ((long long)c.max_N * c.m >= (1LL << 31) || c.n + c.l > 512) return OIC_EINVAL;
  for (int k = 1; k < c.n_layers; ++k)
    if (c.channels[k] < 1 || c.channels[k] > 128) return OIC_EINVAL;
  oic_ctx* h = new (std::nothrow) oic_ctx();
  if (!h) return OIC_ENOMEM;
  h->cfg = c;
  h->slab = slab;
  h->slab_cap = slab_cap;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return OIC_EDEVICE;
  }
  if (c.stream) {
    h->stream = (hipStream_t)c.stream;
  } else {
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
      delete h;
      return OIC_EDEVICE;
    }
    h->own_stream = true;
  }
  for (int k = 1; k < c.n_layers; ++k) h->cmax = std::max(h->cmax, c.channels[k]);
  h->scratch = scratch_on(h->device);
  // observation rows: n + l, plus one if a constraint is set later
  const size_t N = c.max_N, Hs = c.max_H + 1, n = c.n, m = c.m, l = c.l, rr = n + l, p = n + l + 1;
  const size_t NM = N * m;
  const size_t Ma_max = Hs * rr;
  int rc = OIC_OK;
  rc = rc ? rc : dalloc(h, &h->traj, Hs * rr * NM);
  rc = rc ? rc : dalloc(h, &h->Y, p * NM);
  h->act_floats = activation_floats(c);
  rc = rc ? rc : dalloc(h, &h->act[0], h->act_floats);
  rc = rc ? rc : dalloc(h, &h->act[1], h->act_floats);
  rc = rc ? rc : dalloc(h, &h->mu_traj, Ma_max * m);
  rc = rc ? rc : dalloc(h, &h->muY, p * m);  // doubles
  rc = rc ? rc : dalloc(h, &h->S, (Ma_max + p) * p);
  h->part_cap = std::max((size_t)32 * (Ma_max + p) * p, Ma_max * p);
  rc = rc ? rc : dalloc(h, &h->part, h->part_cap);
  rc = rc ? rc : dalloc(h, &h->Lwork, 2 * p * (p + 1));
  rc = rc ? rc : dalloc(h, &h->Syy, p * p);
  rc = rc ? rc : dalloc(h, &h->Sinv, p * p);
  if (!rc && hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess) rc = OIC_EDEVICE;
  if (!rc && (hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess ||
              hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess))
    rc = OIC_EDEVICE;
  rc = rc ? rc : dalloc(h, &h->K, Ma_max * p);
  rc = rc ? rc : dalloc(h, &h->flag, 1);
  rc = rc ? rc : dalloc(h, &h->amax, (size_t)OIC_MAX_LAYERS * kAmaxSlots);
  for (int k = 0; k < 5 && !rc; ++k) rc = dalloc(h, &h->Z[k], noise_floats(c, k));
  rc = rc ? rc : dalloc(h, &h->con_a, n + l);
  rc = rc ? rc : dalloc(h, &h->Uprev, l * m);
  rc = rc ? rc : dalloc(h, &h->Uprev_new, l * m);
  rc = rc ? rc : dalloc(h, &h->fac, l * l + n * n);
  // staging: X0, reference window, U_prev, and batched CNN inputs/outputs
  h->io_floats = n * m + Hs * n * m + l * m + N * (n + l) * m + N * n * m;
  rc = rc ? rc : dalloc(h, &h->io, h->io_floats);
  rc = rc ? rc : dalloc(h, &h->out_stage, Hs * (l + n) * m);
  rc = rc ? rc : dalloc(h, &h->dseed, 1);
  if (!rc && hipHostMalloc((void**)&h->hseed, sizeof(uint64_t), hipHostMallocDefault) != hipSuccess) {
    h->hseed = nullptr;
    rc = OIC_ENOMEM;
  }
  if (!rc && hipMemsetAsync(h->Uprev, 0, l * m * sizeof(float), h->stream) != hipSuccess)
    rc = OIC_EDEVICE;
  if (!rc && hipStreamSynchronize(h->stream) != hipSuccess) rc = OIC_EDEVICE;
  if (!rc && slab) rc = reserve_weights(h);
  if (rc) {
    free_all(h);
    if (h->own_stream) hipStreamDestroy(h->stream);
    delete h;
    return rc;
  }
  *out = h;
  return OIC_OK;
}

void destroy_handle(oic_ctx* h) {
  hipStreamSynchronize(h->stream);
  free_all(h);
  h->timer.destroy();
  if (h->own_stream) hipStreamDestroy(h->stream);
  delete h;
}

}  // namespace

extern "C" {

int oic_create(const oic_config* cfg, oic_handle* out) {
  if (!cfg || !out) return OIC_EINVAL;
  std::lock_guard<std::mutex> guard(resource_mutex());
  return create_handle(*cfg, nullptr, 0, out);
}

void oic_destroy(oic_handle h) {
  if (!h || h->slab) return;  // a group slot goes with its group
  std::lock_guard<std::mutex> guard(resource_mutex());
  destroy_handle(h);
}

const char* oic_last_error(oic_handle h) { return h ? h->err.c_str() : "NULL handle"; }

int oic_set_weights(oic_handle h, const float* B, const float* const* W, const float* const* bias) {
  if (!h) return OIC_EINVAL;
  std::lock_guard<std::mutex> guard(resource_mutex());
  h->err.clear();
  const oic_config& c = h->cfg;
  if (!B || !W) return fail(h, OIC_EINVAL, "NULL B or W");
  if (!finite_all(B, (size_t)c.n * c.l)) return fail(h, OIC_EINVAL, "B has a non-finite entry");
  for (int k = 0; k < c.n_layers; ++k) {
    const size_t cnt = (size_t)c.channels[k + 1] * c.channels[k] * 9;
    if (!W[k] || !finite_all(W[k], cnt)) return fail(h, OIC_EINVAL, "NULL or non-finite layer weights");
    if (bias && bias[k] && !finite_all(bias[k], c.channels[k + 1]))
      return fail(h, OIC_EINVAL, "non-finite bias");
  }
  // A captured solve holds the weight buffers' addresses, not their contents: it stays valid
  // when new values are copied into the same buffers and is dropped only if a buffer is
  // allocated or freed here (first call, or a bias switched on or off).
  const auto addresses = [h]() {
    std::vector<const void*> a{h->dB, h->dWl2};
    for (int k = 0; k < OIC_MAX_LAYERS; ++k) {
      a.push_back(h->dW[k]);
      a.push_back(h->dWk[k]);
      a.push_back(h->dWb[k]);
      a.push_back(h->dWq[k]);
      a.push_back(h->dWs[k]);
      a.push_back(h->dBias[k]);
    }
    return a;
  };
  const std::vector<const void*> before = addresses();
  struct DropIfMoved {
    oic_ctx* h;
    const std::vector<const void*>& before;
    decltype(addresses)& now;
    ~DropIfMoved() {
      if (now() != before) drop_graph(h);
    }
  } drop_if_moved{h, before, addresses};
  h->weights_set = false;  // until every copy below has succeeded
  int rc;
  if (!h->dB && (rc = dalloc(h, &h->dB, (size_t)c.n * c.l))) return rc;
  HIP_TRY(hipMemcpyAsync(h->dB, B, (size_t)c.n * c.l * sizeof(float), hipMemcpyHostToDevice, h->stream));
  for (int k = 0; k < c.n_layers; ++k) {
    const size_t cnt = (size_t)c.channels[k + 1] * c.channels[k] * 9;
    if (!h->dW[k] && (rc = dalloc(h, &h->dW[k], cnt))) return rc;
    HIP_TRY(hipMemcpyAsync(h->dW[k], W[k], cnt * sizeof(float), hipMemcpyHostToDevice, h->stream));
    const int cin = c.channels[k], cout = c.channels[k + 1];
    if (k < c.n_layers - 1 && conv_mfma_supported(cin, cout)) {
      // re-lay out [o][c][dy][dx] -> [(dy*3+dx)*cin + c][o]
      std::vector<float> wk(cnt);
      for (int o = 0; o < cout; ++o)
        for (int ci = 0; ci < cin; ++ci)
          for (int tap = 0; tap < 9; ++tap)
            wk[((size_t)tap * cin + ci) * cout + o] = W[k][((size_t)o * cin + ci) * 9 + tap];
      if (!h->dWk[k] && (rc = dalloc(h, &h->dWk[k], cnt))) return rc;
      HIP_TRY(hipMemcpy(h->dWk[k], wk.data(), cnt * sizeof(float), hipMemcpyHostToDevice));
    }
    if (c.precision == OIC_PREC_FP8 && k > 0 && k < c.n_layers - 1 && conv_mfma_fp8_supported(cin, cout)) {
      // e4m3 copy scaled per output channel, [o][c][dy][dx] -> [o][(dy*3+dx)*cin + c],
      // each row zero-padded to a multiple of 128
      const size_t kd = (size_t)9 * cin, kd128 = (kd + 127) / 128 * 128;
      std::vector<uint8_t> wq((size_t)cout * kd128, 0);
      std::vector<float> ws(cout);
      for (int o = 0; o < cout; ++o) {
        float mx = 0.f;
        for (size_t e = 0; e < kd; ++e) mx = std::max(mx, std::fabs(W[k][(size_t)o * kd + e]));
        ws[o] = mx > 0.f ? mx / 448.0f : 1.0f;
        // The rounding error of each tap is carried into the next tap of the same
        // (o, c) kernel, so the 9 rounded taps keep the exact sum up to the last
        // rounding: on locally smooth inputs (the fields here) the layer output then sees
        // much less of the weight rounding (measured at 256x256: smoothed-control error
        // 0.17 instead of 0.21, closed-loop cost 1.5% instead of 2.9% off FP32).
        for (int ci = 0; ci < cin; ++ci) {
          float carry = 0.f;
          for (int tap = 0; tap < 9; ++tap) {
            const float target = W[k][((size_t)o * cin + ci) * 9 + tap] / ws[o] + carry;
            const uint8_t q = host_e4m3(target);
            carry = target - e4m3_value(q);
            wq[(size_t)o * kd128 + (size_t)tap * cin + ci] = q;
          }
        }
      }
      if (!h->dWq[k] && (rc = dalloc(h, &h->dWq[k], wq.size()))) return rc;
      if (!h->dWs[k] && (rc = dalloc(h, &h->dWs[k], (size_t)cout))) return rc;
      HIP_TRY(hipMemcpy(h->dWq[k], wq.data(), wq.size(), hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(h->dWs[k], ws.data(), cout * sizeof(float), hipMemcpyHostToDevice));
    }
    if (c.precision == OIC_PREC_BF16 && k > 0 && k < c.n_layers - 1 && conv_mfma_bf16_supported(cin, cout)) {
      // BF16 copy, [o][c][dy][dx] -> [o][(dy*3+dx)*cin + c]
      std::vector<uint16_t> wb(cnt);
      for (int o = 0; o < cout; ++o)
        for (int ci = 0; ci < cin; ++ci)
          for (int tap = 0; tap < 9; ++tap)
            wb[(size_t)o * 9 * cin + (size_t)tap * cin + ci] =
                host_bf16(W[k][((size_t)o * cin + ci) * 9 + tap]);
      if (!h->dWb[k] && (rc = dalloc(h, &h->dWb[k], cnt))) return rc;
      HIP_TRY(hipMemcpy(h->dWb[k], wb.data(), cnt * sizeof(uint16_t), hipMemcpyHostToDevice));
    }
    if ((c.precision == OIC_PREC_BF16 || c.precision == OIC_PREC_FP8) && k == c.n_layers - 1 && k >= 2 && cout == 1 &&
        conv_last_folds_bf16(c.channels[k - 1], cin)) {
      // the last layer as a BF16 pair for the folded epilogue: [hi, lo][tap (16, zero past 9)][c]
      std::vector<uint16_t> w2((size_t)2 * 16 * cin, 0);
      for (int ci = 0; ci < cin; ++ci)
        for (int tap = 0; tap < 9; ++tap) {
          const float v = W[k][(size_t)ci * 9 + tap];
          const uint16_t hi = host_bf16(v);
          uint32_t hb = (uint32_t)hi << 16;
          float hf;
          memcpy(&hf, &hb, sizeof(hf));
          w2[(size_t)tap * cin + ci] = hi;
          w2[(size_t)(16 + tap) * cin + ci] = host_bf16(v - hf);
        }
      if (!h->dWl2 && (rc = dalloc(h, &h->dWl2, w2.size()))) return rc;
      HIP_TRY(hipMemcpy(h->dWl2, w2.data(), w2.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
    }
    if (bias && bias[k]) {
      if (!h->dBias[k] && (rc = dalloc(h, &h->dBias[k], (size_t)c.channels[k + 1]))) return rc;
      HIP_TRY(hipMemcpyAsync(h->dBias[k], bias[k], c.channels[k + 1] * sizeof(float),
                             hipMemcpyHostToDevice, h->stream));
    } else if (h->dBias[k] && h->slab) {
      // a group slot keeps its buffer (the slots share one set of launches): no bias is
      // a zero bias, which every kernel adds as exactly what it uses without one
      HIP_TRY(hipMemsetAsync(h->dBias[k], 0, c.channels[k + 1] * sizeof(float), h->stream));
    } else if (h->dBias[k]) {
      hipFree(h->dBias[k]);
      h->dBias[k] = nullptr;
    }
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->weights_set = true;
  return OIC_OK;
}

int oic_set_u_prev(oic_handle h, const float* U_prev) {
  if (!h) return OIC_EINVAL;
  h->err.clear();
  if (!U_prev) return fail(h, OIC_EINVAL, "NULL U_prev");
  int rc = copy_in(h, h->Uprev, U_prev, (size_t)h->cfg.l * h->cfg.m);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(h->stream));
  return OIC_OK;
}

int oic_get_u_prev(oic_handle h, float* U_prev) {
  if (!h) return OIC_EINVAL;
  h->err.clear();
  if (!U_prev) return fail(h, OIC_EINVAL, "NULL U_prev");
  int rc = copy_out(h, U_prev, h->Uprev, (size_t)h->cfg.l * h->cfg.m);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(h->stream));
  return OIC_OK;
}

int oic_solve(oic_handle h, const float* X0, const float* reference, const float* Q, const float* R,
              int N, int horizon, uint64_t seed, float* U_out, float* X_out) {
  oic_solve_args a{};
  a.X0 = X0;
  a.reference = reference;
  a.Q = Q;
  a.R = R;
  a.N = N;
  a.horizon = horizon;
  a.seed = seed;
  a.U_out = U_out;
  a.X_out = X_out;
  return solve_impl(h, &a);
}

int oic_solve_ex(oic_handle h, const oic_solve_args* a) { return solve_impl(h, a); }

int oic_solve_cov(oic_handle h, const oic_solve_args* a, double* prior_cov, double* post_cov) {
  if (!h) return OIC_EINVAL;
  h->err.clear();
  if (!a) return fail(h, OIC_EINVAL, "NULL argument block");
  if (!prior_cov || !post_cov) return fail(h, OIC_EINVAL, "NULL covariance output");
  const oic_config& c = h->cfg;
  const int H = a->horizon;
  if (H < 1 || H > c.max_H) return solve_impl(h, a);  // reports the error
  const size_t rr = (size_t)c.n + c.l;
  const size_t need = cov_offset((int)rr, H + 1);
  const size_t ma = (size_t)(H + 1) * rr;
  int rc;
  // buffers on first use (this entry point allocates; the solve itself does not)
  std::unique_lock<std::mutex> guard(resource_mutex());
  if (h->cov_cap < need) {
    if (h->cov_prior) hipFree(h->cov_prior);
    if (h->cov_post) hipFree(h->cov_post);
    h->cov_prior = h->cov_post = nullptr;
    h->cov_cap = 0;
    if ((rc = dalloc(h, &h->cov_prior, need)) || (rc = dalloc(h, &h->cov_post, need))) return rc;
    h->cov_cap = need;
  }
  if (h->mu64_cap < ma * c.m) {
    if (h->mu64) hipFree(h->mu64);
    h->mu64 = nullptr;
    h->mu64_cap = 0;
    if ((rc = dalloc(h, &h->mu64, ma * c.m))) return rc;
    h->mu64_cap = ma * c.m;
  }
  if (h->part_cap < ma * ma) {  // one split of the largest covariance must fit
    double* bigger = nullptr;     // the old buffer stays in place if this fails
    if ((rc = dalloc(h, &bigger, ma * ma))) return rc;
    HIP_TRY(hipStreamSynchronize(h->stream));
    hipFree(h->part);
    h->part = bigger;
    h->part_cap = ma * ma;
    drop_graph(h);  // a captured solve refers to the old buffer
  }
  guard.unlock();
  h->want_cov = true;
  rc = solve_impl(h, a);
  h->want_cov = false;
  if (rc) return rc;
  const hipMemcpyKind kind = c.mem_mode == OIC_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  HIP_TRY(hipMemcpyAsync(prior_cov, h->cov_prior, need * sizeof(double), kind, h->stream));
  HIP_TRY(hipMemcpyAsync(post_cov, h->cov_post, need * sizeof(double), kind, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return OIC_OK;
}

namespace {
int cnn_forward_impl(oic_handle h, int batch, const float* X, const float* U, float* X_next,
                     bool fp32_only) {
  if (!h) return OIC_EINVAL;
  h->err.clear();
  const oic_config& c = h->cfg;
  if (!h->weights_set) return fail(h, OIC_EINVAL, "weights not set");
  if (batch < 1 || batch > c.max_N) return fail(h, OIC_EINVAL, "batch must be in 1..max_N");
  if (!X || !U || !X_next) return fail(h, OIC_EINVAL, "NULL pointer");
  const size_t n = c.n, m = c.m, l = c.l;
  if (c.mem_mode == OIC_MEM_DEVICE) {
    // device pointers go straight to the kernels (X_next may alias X: the first layer has
    // read all of X before the last layer writes)
    rollout(h, batch, FieldRef{X, (long long)(n * m), (long long)m}, FieldRef{U, (long long)(l * m), (long long)m},
            FieldOut{X_next, (long long)(n * m), (long long)m}, fp32_only ? RM_FP32 : rollout_mode(h));
    // on a private stream the caller cannot order against the work: finish it here
    if (h->own_stream || h->timer.enabled) {
      HIP_TRY(hipStreamSynchronize(h->stream));
      h->timer.harvest();
    }
    return OIC_OK;
  }
  float* dX = h->io + n * m + (size_t)(c.max_H + 1) * n * m + l * m;
  float* dU = dX + (size_t)c.max_N * n * m;
  float* dO = dU + (size_t)c.max_N * l * m;
  int rc;
  if ((rc = copy_in(h, dX, X, batch * n * m))) return rc;
  if ((rc = copy_in(h, dU, U, batch * l * m))) return rc;
  rollout(h, batch, FieldRef{dX, (long long)(n * m), (long long)m},
          FieldRef{dU, (long long)(l * m), (long long)m}, FieldOut{dO, (long long)(n * m), (long long)m},
          fp32_only ? RM_FP32 : rollout_mode(h));
  if ((rc = copy_out(h, X_next, dO, batch * n * m))) return rc;
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->timer.harvest();
  return OIC_OK;
}

}  // namespace

int oic_cnn_forward(oic_handle h, int batch, const float* X, const float* U, float* X_next) {
  return cnn_forward_impl(h, batch, X, U, X_next, false);
}

int oic_cnn_forward_noalloc(oic_handle h, int batch, const float* X, const float* U, float* X_next) {
  if (!h) return OIC_EINVAL;
  h->err.clear();
  const oic_config& c = h->cfg;
  if (c.mem_mode != OIC_MEM_DEVICE)
    return fail(h, OIC_EINVAL, "oic_cnn_forward_noalloc needs a handle created with OIC_MEM_DEVICE");
  if (!h->weights_set) return fail(h, OIC_EINVAL, "weights not set");
  if (batch < 1 || batch > c.max_N) return fail(h, OIC_EINVAL, "batch must be in 1..max_N");
  if (!X || !U || !X_next) return fail(h, OIC_EINVAL, "NULL pointer");
  if (!h->scratch)
    return fail(h, OIC_EDEVICE, "the device address of the allocation-free buffer could not be obtained");
  const RolloutMode mode = rollout_mode(h);
  const size_t n = c.n, m = c.m, l = c.l;
  // layout: [per-layer FP8 maxima][activations A][activations B], 256-byte aligned
  constexpr size_t head = ((size_t)OIC_MAX_LAYERS * kAmaxSlots * sizeof(unsigned) + 255) / 256 * 256;
  const size_t act_bytes = ((size_t)batch * n * m * h->cmax * (mode == RM_FP32 ? 4 : 2) + 255) / 256 * 256;
  const size_t need = head + 2 * act_bytes;
  if (need > OIC_NOALLOC_SCRATCH_BYTES)
    return fail(h, OIC_ENOMEM, "batch needs " + std::to_string(need) + " bytes of scratch; the fixed buffer holds " +
                                   std::to_string((size_t)OIC_NOALLOC_SCRATCH_BYTES));
  unsigned char* base = h->scratch;
  Timer untimed;  // a timed launch would create events on first use
  rollout(h, batch, FieldRef{X, (long long)(n * m), (long long)m}, FieldRef{U, (long long)(l * m), (long long)m},
          FieldOut{X_next, (long long)(n * m), (long long)m}, mode, nullptr,
          reinterpret_cast<float*>(base + head), reinterpret_cast<float*>(base + head + act_bytes),
          reinterpret_cast<unsigned*>(base), &untimed, act_bytes / sizeof(float));
  HIP_TRY(hipGetLastError());
  // on a private stream the caller cannot order against the work: finish it here
  if (h->own_stream) HIP_TRY(hipStreamSynchronize(h->stream));
  return OIC_OK;
}

int oic_plant_step(oic_handle h, const float* X, const float* U, float* X_next) {
  // the plant stands for the real system: always the FP32 surrogate
  return cnn_forward_impl(h, 1, X, U, X_next, true);
}

int oic_normals(oic_handle h, uint64_t seed, int kind, size_t count, float* out) {
  if (!h) return OIC_EINVAL;
  h->err.clear();
  if (kind < 0 || kind > 4 || !out) return fail(h, OIC_EINVAL, "bad kind or NULL output");
  if (count > noise_floats(h->cfg, kind)) return fail(h, OIC_ENOMEM, "count exceeds the noise capacity");
  *h->hseed = seed;
  HIP_TRY(hipMemcpyAsync(h->dseed, h->hseed, sizeof(uint64_t), hipMemcpyHostToDevice, h->stream));
  launch_normals(h->stream, h->timer, h->Z[kind], count, h->dseed, (uint32_t)kind);
  int rc = copy_out(h, out, h->Z[kind], count);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->timer.harvest();
  return OIC_OK;
}

int oic_timing(oic_handle h, int enable) {
  if (!h) return OIC_EINVAL;
  hipStreamSynchronize(h->stream);
  h->timer.harvest();
  h->timer.reset();
  h->timer.enabled = enable != 0;
  return OIC_OK;
}

int oic_kernel_class_count(void) { return KC_COUNT; }

int oic_kernel_stats(oic_handle h, int id, const char** name, long long* launches, double* total_ms) {
  if (!h || id < 0 || id >= KC_COUNT) return OIC_EINVAL;
  if (name) *name = kKernelClassNames[id];
  if (launches) *launches = h->timer.launches[id];
  if (total_ms) *total_ms = h->timer.total_ms[id];
  return OIC_OK;
}

void* oic_stream(oic_handle h) { return h ? (void*)h->stream : nullptr; }

namespace {
// sum over columns of e^T M^{-1} e with e = E - E0 (E0 may be NULL) and M = L L^T
// (host FP64): solve L z = e, add |z|^2.
double quad_form_inv(const std::vector<double>& L, int k, const float* E, const float* E0, int m) {
  double total = 0.0;
  std::vector<double> z(k);
  for (int x = 0; x < m; ++x) {
    for (int i = 0; i < k; ++i) {
      double v = (double)E[(size_t)i * m + x] - (E0 ? (double)E0[(size_t)i * m + x] : 0.0);
      for (int c = 0; c < i; ++c) v -= L[(size_t)i * k + c] * z[c];
      z[i] = v / L[(size_t)i * k + i];
      total += z[i] * z[i];
    }
  }
  return total;
}
}  // namespace

int oic_stage_cost(int n, int m, int l, const float* X, const float* Xref, const float* U,
                   const float* dU, const float* Q, const float* R, double* cost) {
  if (n < 1 || m < 1 || l < 1 || !X || !Xref || !U || !dU || !Q || !R || !cost) return OIC_EINVAL;
  std::vector<double> Lq, Lr;
  if (!host_cholesky(Q, l, Lq) || !host_cholesky(R, n, Lr)) return OIC_EINVAL;
  *cost = quad_form_inv(Lr, n, X, Xref, m) + quad_form_inv(Lq, l, U, nullptr, m) +
          quad_form_inv(Lq, l, dU, nullptr, m);
  return OIC_OK;
}

int oic_set_constraint(oic_handle h, const float* aX, const float* aU, float b, float alpha, float beta,
                       float rz) {
  if (!h) return OIC_EINVAL;
  h->err.clear();
  const oic_config& c = h->cfg;
  bool on = aX || aU;
  if (on) {
    if (!aX || !aU) return fail(h, OIC_EINVAL, "aX and aU must both be given (or both NULL)");
    if (!(alpha > 0.f) || !(beta > 0.f) || !(rz > 0.f) || !std::isfinite(b) || !std::isfinite(alpha) ||
        !std::isfinite(beta) || !std::isfinite(rz))
      return fail(h, OIC_EINVAL, "alpha, beta and rz must be positive and finite, b finite");
    if (!finite_all(aX, c.n) || !finite_all(aU, c.l)) return fail(h, OIC_EINVAL, "non-finite aX or aU");
    if (c.n + c.l + 1 > 512) return fail(h, OIC_EINVAL, "n + l + 1 observation rows exceed 512");
  }
  std::lock_guard<std::mutex> guard(resource_mutex());
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (on) {
    HIP_TRY(hipMemcpy(h->con_a, aX, c.n * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(h->con_a + c.n, aU, c.l * sizeof(float), hipMemcpyHostToDevice));
    h->con_b = b;
    h->con_alpha = alpha;
    h->con_beta = beta;
    h->con_rz = rz;
  }
  h->con_on = on;
  drop_graph(h);  // the captured solve has the old observation rows and parameters
  return OIC_OK;
}

int oic_columns_expand(int l, int q, int m, const float* u, const float* T, float* U) {
  if (l < 1 || q < 1 || m < 1 || !u || !T || !U) return OIC_EINVAL;
  for (int a = 0; a < l; ++a)
    for (int c = 0; c < m; ++c) {
      double s = 0.0;
      for (int j = 0; j < q; ++j) s += (double)u[(size_t)a * q + j] * T[(size_t)j * m + c];
      U[(size_t)a * m + c] = (float)s;
    }
  return OIC_OK;
}

int oic_columns_project(int l, int m, int q, const float* U, const float* T, float* u) {
  if (l < 1 || q < 1 || m < 1 || q > m || !U || !T || !u) return OIC_EINVAL;
  // G = T T^T (q x q, SPD when T has full row rank), then u^T = G^{-1} T U^T column by
  // column with the Cholesky factor of G, all in FP64
  std::vector<double> L((size_t)q * q, 0.0);  // Cholesky factor of G, built row by row
  for (int i = 0; i < q; ++i)
    for (int j = 0; j <= i; ++j) {
      double g = 0.0;
      for (int c = 0; c < m; ++c) g += (double)T[(size_t)i * m + c] * T[(size_t)j * m + c];
      for (int k = 0; k < j; ++k) g -= L[(size_t)i * q + k] * L[(size_t)j * q + k];
      if (i == j) {
        if (!(g > 0.0) || !std::isfinite(g)) return OIC_ENOTSPD;
        L[(size_t)i * q + i] = std::sqrt(g);
      } else {
        L[(size_t)i * q + j] = g / L[(size_t)j * q + j];
      }
    }
  std::vector<double> y(q);
  for (int a = 0; a < l; ++a) {
    for (int i = 0; i < q; ++i) {  // rhs_i = (U T^T)[a][i]
      double s = 0.0;
      for (int c = 0; c < m; ++c) s += (double)U[(size_t)a * m + c] * T[(size_t)i * m + c];
      y[i] = s;
    }
    for (int i = 0; i < q; ++i) {  // L z = rhs
      double v = y[i];
      for (int j = 0; j < i; ++j) v -= L[(size_t)i * q + j] * y[j];
      y[i] = v / L[(size_t)i * q + i];
    }
    for (int i = q - 1; i >= 0; --i) {  // L^T x = z
      double v = y[i];
      for (int j = i + 1; j < q; ++j) v -= L[(size_t)j * q + i] * y[j];
      y[i] = v / L[(size_t)i * q + i];
    }
    for (int i = 0; i < q; ++i) u[(size_t)a * q + i] = (float)y[i];
  }
  return OIC_OK;
}

size_t oic_group_footprint_bytes(const oic_config* cfg, int slots) {
  if (!cfg || slots < 1) return 0;
  return (size_t)slots * group_slab_bytes(*cfg) + 4096;
}

int oic_group_create(const oic_config* cfg, int slots, oic_group_handle* out) {
  if (!cfg || !out || slots < 1 || slots > OIC_MAX_GROUP_SLOTS) return OIC_EINVAL;
  *out = nullptr;
  const oic_config& c = *cfg;
  // several slots per launch: the BF16 rollout and the statistics and update of its mode
  if (slots > 1 && (c.precision != OIC_PREC_BF16 || !bf16_rollout_possible(c))) return OIC_EINVAL;
  std::lock_guard<std::mutex> guard(resource_mutex());
  oic_group* g = new (std::nothrow) oic_group();
  if (!g) return OIC_ENOMEM;
  g->cfg = c;
  g->slots = slots;
  g->slab = group_slab_bytes(c);
  int rc = OIC_OK;
  if (hipMalloc((void**)&g->region, g->slab * slots) != hipSuccess) {
    g->region = nullptr;
    rc = OIC_ENOMEM;
  }
  for (int i = 0; i < slots && !rc; ++i) {
    oic_ctx* h = nullptr;
    rc = create_handle(c, g->region + (size_t)i * g->slab, g->slab, &h);
    if (!rc) g->h.push_back(h);
  }
  if (!rc && hipMalloc((void**)&g->dactive, slots * sizeof(int)) != hipSuccess) {
    g->dactive = nullptr;
    rc = OIC_ENOMEM;
  }
  if (!rc && (hipHostMalloc((void**)&g->hactive, slots * sizeof(int), hipHostMallocDefault) != hipSuccess ||
              hipHostMalloc((void**)&g->hflags, slots * sizeof(int), hipHostMallocDefault) != hipSuccess))
    rc = OIC_ENOMEM;
  if (rc) {
    for (oic_ctx* h : g->h) destroy_handle(h);
    if (g->region) hipFree(g->region);
    if (g->dactive) hipFree(g->dactive);
    if (g->hactive) hipHostFree(g->hactive);
    if (g->hflags) hipHostFree(g->hflags);
    delete g;
    return rc;
  }
  *out = g;
  return OIC_OK;
}

void oic_group_destroy(oic_group_handle g) {
  if (!g) return;
  std::lock_guard<std::mutex> guard(resource_mutex());
  for (oic_ctx* h : g->h) hipStreamSynchronize(h->stream);
  if (g->gexec) hipGraphExecDestroy(g->gexec);
  for (oic_ctx* h : g->h) destroy_handle(h);
  hipFree(g->region);
  hipFree(g->dactive);
  hipHostFree(g->hactive);
  hipHostFree(g->hflags);
  delete g;
}

oic_handle oic_group_slot(oic_group_handle g, int slot) {
  return g && slot >= 0 && slot < g->slots ? g->h[slot] : nullptr;
}

const char* oic_group_last_error(oic_group_handle g) { return g ? g->err.c_str() : "NULL group"; }

int oic_group_solve(oic_group_handle g, int count, const int* slots, const oic_solve_args* args, int* rc_out) {
  if (!g) return OIC_EINVAL;
  g->err.clear();
  if (count < 1 || count > g->slots || !slots || !args) {
    g->err = "count must be 1 .. slots, with slots and args given";
    return OIC_EINVAL;
  }
  std::vector<char> on(g->slots, 0);
  for (int i = 0; i < count; ++i) {
    if (slots[i] < 0 || slots[i] >= g->slots || on[slots[i]]) {
      g->err = "slot indices must be distinct and below the group's slot count";
      return OIC_EINVAL;
    }
    on[slots[i]] = 1;
  }
  std::vector<int> rcs(count, OIC_OK);
  auto report = [&]() {
    int first = OIC_OK;
    for (int i = 0; i < count; ++i) {
      if (rc_out) rc_out[i] = rcs[i];
      if (rcs[i] && !first) {
        first = rcs[i];
        g->err = "slot " + std::to_string(slots[i]) + ": " + g->h[slots[i]]->err;
      }
    }
    return first;
  };
  if (count == 1) {  // one request: the slot's own solve
    rcs[0] = solve_impl(g->h[slots[0]], &args[0]);
    return report();
  }
  oic_ctx* h0 = g->h[0];
  hipStream_t s = h0->stream;
  // inputs of every request into its slot, on slot 0's stream; the batch's N, horizon,
  // noise source and factor layout come from its first request that passes the checks
  Dims d{};
  bool seeded = false, qd = true, rd = true, have = false;
  for (int i = 0; i < count; ++i) {
    oic_ctx* h = g->h[slots[i]];
    on[slots[i]] = 0;
    if (h->con_on || h->want_cov || h->timer.enabled) {
      rcs[i] = fail(h, OIC_EINVAL, "grouped solves take no constraint, covariance outputs or timing");
      continue;
    }
    Dims di{};
    bool si = false;
    rcs[i] = solve_begin(h, &args[i], s, di, si);
    if (rcs[i]) continue;
    if (!have) {
      d = di;
      seeded = si;
      qd = h->q_diag;
      rd = h->r_diag;
      have = true;
    } else if (di.N != d.N || di.H != d.H || si != seeded || h->q_diag != qd || h->r_diag != rd) {
      rcs[i] = fail(h, OIC_EINVAL, "N, horizon, noise source or Q/R structure differs from the batch's");
      continue;
    }
    on[slots[i]] = 1;
  }
  if (!have) return report();
  for (int k = 0; k < g->slots; ++k) g->hactive[k] = on[k];
  int rc = OIC_OK;
  hipError_t e = hipMemcpyAsync(g->dactive, g->hactive, g->slots * sizeof(int), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    g->err = std::string("hipMemcpyAsync: ") + hipGetErrorString(e);
    return OIC_EDEVICE;
  }
  {
    // the kernels of the solve, once for all slots
    LaunchGroup& lg = launch_group();
    lg = LaunchGroup{(unsigned)g->slots, Grp{g->slab, g->dactive}, false};
    struct Reset {
      ~Reset() { launch_group() = LaunchGroup{}; }
    } reset;
    if (h0->use_graph) {
      if (!g->gexec || g->gN != d.N || g->gH != d.H || g->gSeeded != seeded || g->gQd != qd || g->gRd != rd) {
        std::lock_guard<std::mutex> guard(resource_mutex());
        rc = capture_solve(h0, s, &g->gexec, d, seeded, RM_BF16, qd, rd);
        if (!rc && lg.unsupported) {
          hipGraphExecDestroy(g->gexec);
          g->gexec = nullptr;
        }
        g->gN = d.N;
        g->gH = d.H;
        g->gSeeded = seeded;
        g->gQd = qd;
        g->gRd = rd;
      }
      if (!rc && g->gexec && hipGraphLaunch(g->gexec, s) != hipSuccess) rc = OIC_EDEVICE;
    } else {
      enqueue_solve(h0, d, seeded, RM_BF16, qd, rd);
    }
    if (rc) {
      g->err = "capture of the grouped solve failed: " + h0->err;
      hipStreamSynchronize(s);
      return rc;
    }
    if (lg.unsupported) {
      g->err = "this configuration's solve uses a kernel without a grouped form";
      hipStreamSynchronize(s);
      return OIC_EINVAL;
    }
  }
  for (int i = 0; i < count; ++i)
    if (!rcs[i]) rcs[i] = solve_end(g->h[slots[i]], &args[i], s, &g->hflags[slots[i]]);
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    g->err = std::string("hipStreamSynchronize: ") + hipGetErrorString(e);
    return OIC_EDEVICE;
  }
  for (int i = 0; i < count; ++i)
    if (!rcs[i]) rcs[i] = solve_finish(g->h[slots[i]], &args[i], s, g->hflags[slots[i]]);
  return report();
}

int oic_set_graph(oic_handle h, int enable) {
  if (!h) return OIC_EINVAL;
  std::lock_guard<std::mutex> guard(resource_mutex());
  h->use_graph = enable != 0;
  if (!h->use_graph && h->gexec) {
    hipStreamSynchronize(h->stream);
    hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  return OIC_OK;
}

}  // extern "C"
