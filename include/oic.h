/*
 * oic.h - C ABI of liboic, the MI355X (gfx950) Kalman-MPC library.
 *
 * Kalman-MPC ("Optimal Inferential Control of Convolutional Neural Networks",
 * Vaziri & Fang, Algorithm 1) controls a CNN surrogate X_{k+1} = CNN(X_k, U_k)
 * (Eq. (1)) by recasting the reference-tracking MPC problem (Eq. (3)) as state
 * smoothing of a virtual system (Eqs. (4)-(5)) and solving that with a
 * single-pass ensemble Kalman smoother over matrix-valued members
 * (Eqs. (11)-(15)).  One call of oic_solve is one MPC solve at one time k.
 *
 * Conventions shared by every entry point:
 *  - Matrices are row-major FP32.  The state X is n x m, the control U is l x m.
 *  - The CNN takes two input channels, X and B U (B is n x l), applies
 *    zero-padded 3x3 cross-correlations with the chosen activation between
 *    layers (none after the last) and returns one channel, the next state.
 *  - R (n x n) is the row covariance of the state observation noise V_X; Q
 *    (l x l) is the row covariance of both the control-increment noise W and
 *    the control observation noise V_U (the paper's Q_dU and Q_U taken equal);
 *    the column covariance is the identity.  The control reference U^ref is 0.
 *    R and Q are always HOST pointers; they are factorised on the host in FP64.
 *  - Weights and B are always HOST pointers; the library copies them.
 *  - Every other array argument is a host pointer when the handle was created
 *    with OIC_MEM_HOST and a device pointer (on the handle's device) with
 *    OIC_MEM_DEVICE; device-pointer work is ordered on the handle's stream.
 *  - The caller owns every buffer it passes; the library keeps no pointer to
 *    caller memory after a call returns.
 *  - Return values: OIC_OK (0) or a negative error code.  On error no output
 *    buffer is written and oic_last_error(h) describes the reason.  No C++
 *    exception crosses the ABI.
 *  - A handle is not thread-safe: one handle per controller per thread.  The
 *    same inputs, seed and precision give bitwise-identical outputs.
 */
#ifndef OIC_H
#define OIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OIC_OK 0
#define OIC_EINVAL (-1)   /* bad dimension, pointer, non-finite input, or weights not set */
#define OIC_ENOMEM (-2)   /* device allocation failed or the request exceeds the handle's capacity */
#define OIC_EDEVICE (-3)  /* a HIP runtime call failed */
#define OIC_ENOTSPD (-4)  /* Sigma^Ybar was not positive definite at some horizon step */

#define OIC_ACT_TANH 0
#define OIC_ACT_GELU 1    /* exact form 0.5 x (1 + erf(x / sqrt 2)) */

#define OIC_PREC_FP32 0   /* rollout in FP32 */
#define OIC_PREC_BF16 1   /* rollout in BF16 x BF16 products with FP32 accumulation */
#define OIC_PREC_FP8 2    /* hidden layers in OCP FP8 e4m3 x e4m3 products with FP32 accumulation:
                             weights scaled per output channel, activations per layer by their
                             largest magnitude over the ensemble; BF16 storage between layers;
                             hidden widths 32 or 64 in, 16, 32 or 64 out */

#define OIC_MEM_HOST 0
#define OIC_MEM_DEVICE 1

#define OIC_MAX_LAYERS 8

typedef struct oic_ctx* oic_handle;

/* Static description of one controller.  channels[0] must be 2 and
 * channels[n_layers] must be 1; hidden widths are at most 128. */
typedef struct {
  int n, m, l;                            /* state n x m, control l x m; n, m >= 4; 1 <= l <= n */
  int n_layers;                           /* 1..OIC_MAX_LAYERS */
  int channels[OIC_MAX_LAYERS + 1];
  int activation;                         /* OIC_ACT_* */
  int precision;                          /* OIC_PREC_*; statistics stay FP32/FP64, the gain solve FP64 */
  int max_N;                              /* largest ensemble size a solve may use (>= 2) */
  int max_H;                              /* largest horizon a solve may use (>= 1) */
  int mem_mode;                           /* OIC_MEM_HOST or OIC_MEM_DEVICE */
  void* stream;                           /* hipStream_t to order work on, or NULL for a private stream */
} oic_config;

/* Create a handle and allocate all device memory a solve of up to max_N
 * members and max_H steps needs.  *out receives the handle.  Errors:
 * OIC_EINVAL for a bad config, OIC_ENOMEM, OIC_EDEVICE. */
int oic_create(const oic_config* cfg, oic_handle* out);

/* Release the handle and its device memory.  NULL-safe. */
void oic_destroy(oic_handle h);

/* Human-readable reason for the last error on this handle ("" if none).
 * The string stays valid until the next call on the handle. */
const char* oic_last_error(oic_handle h);

/* Set the surrogate of Eq. (1).  B: n x l.  W[k]: layer k weights in
 * [C_out][C_in][3][3] order.  bias: NULL, or bias[k] NULL or C_out floats.
 * Host pointers, copied (and re-laid out or converted for the chosen
 * precision) before return.  Errors: OIC_EINVAL for NULL or non-finite values. */
int oic_set_weights(oic_handle h, const float* B, const float* const* W, const float* const* bias);

/* The control applied before time k, U_{k-1} (l x m), which seeds the initial
 * ensemble U_k^i = U_prev + W_0^i, dU_k^i = W_0^i (Algorithm 1, line 4).  It
 * starts at zero and every successful solve sets it to the applied control
 * U_hat_k (line 14).  Memory per mem_mode. */
int oic_set_u_prev(oic_handle h, const float* U_prev);
int oic_get_u_prev(oic_handle h, float* U_prev);

/* One MPC solve at time k (Algorithm 1, lines 4-13).
 *   X0:        n x m, the measured state X_k.
 *   reference: (horizon+1) x n x m, X^ref_t for t = k..k+horizon.
 *   Q, R:      l x l and n x n SPD (host).
 *   N:         ensemble size, 2..max_N, with (N-1) m >= n + l.
 *   horizon:   H, 1..max_H.
 *   seed:      key of the Philox4x32-10 stream the noise is drawn from: the
 *              normal with C-order index e in the (H, N, rows, m) array of noise
 *              kind c (0: initial control spread, shape (N, l, m); 1: W_t; 2: V_X,t;
 *              3: V_U,t; 4: the constraint row's eps_t, shape (H, N, 1, m), drawn only
 *              when a constraint is set) uses counter (e mod 2^32, e div 2^32, c, 0) and key
 *              (seed mod 2^32, seed div 2^32); two 53-bit uniforms feed the
 *              Box-Muller cosine branch in FP64, rounded to FP32.
 *   U_out:     (horizon+1) x l x m, the smoothed control means U_hat_{k..k+H}.
 *   X_out:     (horizon+1) x n x m smoothed state means, or NULL.
 * Errors: OIC_EINVAL, OIC_ENOMEM (N or H beyond capacity), OIC_ENOTSPD, OIC_EDEVICE. */
int oic_solve(oic_handle h, const float* X0, const float* reference, const float* Q,
              const float* R, int N, int horizon, uint64_t seed, float* U_out, float* X_out);

/* oic_solve with explicit noise.  When Z_init, Z_W, Z_VX and Z_VU are all
 * non-NULL they are used instead of the seeded stream (standard normals,
 * member-major: Z_init N x l x m; Z_W and Z_VU H x N x l x m; Z_VX H x N x n x m;
 * index t-1 of the leading axis belongs to horizon step t).  They must be all
 * NULL or all non-NULL.  U_prev, when non-NULL, replaces the handle's stored
 * value for this solve (and is then overwritten by U_hat_k as usual). */
typedef struct {
  const float* X0;
  const float* reference;
  const float* Q;
  const float* R;
  int N;
  int horizon;
  uint64_t seed;
  const float* U_prev;
  const float* Z_init;
  const float* Z_W;
  const float* Z_VX;
  const float* Z_VU;
  float* U_out;
  float* X_out;
  const float* Z_VZ;  /* H x N x m: noise of the constraint row (only with oic_set_constraint) */
} oic_solve_args;

int oic_solve_ex(oic_handle h, const oic_solve_args* a);

/* oic_solve_ex plus the optional covariance outputs of Algorithm 1 (lines 8 and 11):
 * for every horizon step t = 1..horizon, the pooled covariance of all stored
 * trajectory rows, Sigma = (lambda / N) sum_i A^i A^iT with lambda = 1/tr(Psi) = 1/m
 * and A^i the member's anomaly, before the analysis of step t (Eqs. (15d)-(15f)) in
 * prior_cov and after it (Eq. (14c)) in post_cov.  Step t's block is Ma_t x Ma_t
 * row-major FP64 with Ma_t = (t+1)(n+l): slices k..k+t, each its n X rows then its l
 * U rows (the Delta U rows are not carried).  The blocks follow one another for
 * t = 1..horizon, sum_t Ma_t^2 doubles in each output, in host or device memory per
 * mem_mode.  The first call allocates the covariance buffers; the solve runs kernel by
 * kernel (not from a captured graph).  Results otherwise identical to oic_solve_ex. */
int oic_solve_cov(oic_handle h, const oic_solve_args* a, double* prior_cov, double* post_cov);

/* The surrogate alone, Eq. (1), on `batch` independent fields:
 * X: batch x n x m, U: batch x l x m, X_next: batch x n x m (memory per
 * mem_mode).  batch <= max_N.  Runs the same rollout kernels a solve runs. */
int oic_cnn_forward(oic_handle h, int batch, const float* X, const float* U, float* X_next);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving or control loops, harnesses that forbid hipMalloc): oic_cnn_forward
 * with its intermediate activations (and the FP8 rollout's per-layer maxima) in one
 * fixed library-wide device buffer of OIC_NOALLOC_SCRATCH_BYTES per GPU instead of the
 * handle's buffers.  The call allocates nothing, launches the same kernels and returns
 * the same values bitwise as oic_cnn_forward on the same handle.
 *   h:  a handle created with OIC_MEM_DEVICE (X, U and X_next are device pointers,
 *       the work is ordered on the handle's stream; with a private stream the call
 *       waits for it, as oic_cnn_forward does).
 *   batch, X, U, X_next: as for oic_cnn_forward (X_next may alias X).
 * The buffer must hold two activation arrays of batch x n x m x C elements, C the
 * widest hidden layer, 4 bytes each in the FP32 mode and 2 in the BF16 and FP8 modes,
 * plus 2 KiB; a larger request returns OIC_ENOMEM with the size in
 * oic_last_error, before any work is queued.  OIC_EINVAL for a host-memory handle,
 * unset weights, a batch outside 1..max_N or a NULL pointer; OIC_EDEVICE if the buffer's
 * device address could not be obtained when the handle was created.
 * Every handle on one GPU shares the buffer and a call leaves its contents behind:
 * calls that overlap on one GPU (different streams or threads) race and must be
 * ordered by the caller. */
#define OIC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int oic_cnn_forward_noalloc(oic_handle h, int batch, const float* X, const float* U, float* X_next);

/* The nominal plant of the closed loop (Algorithm 1, line 14): the applied
 * control drives the surrogate itself, X_{k+1} = CNN(X_k, U_k).  Same as
 * oic_cnn_forward with batch 1. */
int oic_plant_step(oic_handle h, const float* X, const float* U, float* X_next);

/* The normals of one noise kind of the seeded stream (see oic_solve), count
 * values in C order from element index 0, written to `out` (memory per
 * mem_mode).  count <= the handle's noise capacity. */
int oic_normals(oic_handle h, uint64_t seed, int kind, size_t count, float* out);

/* Per-kernel timing.  When enabled, every launch of the library's kernels is
 * bracketed by HIP events on the handle's stream and its duration is added to
 * its kernel class.  oic_kernel_stats reports, for class `id`
 * (0 <= id < oic_kernel_class_count()), the class name, number of launches
 * and total milliseconds since the last reset (oic_timing(h, 1) resets). */
int oic_timing(oic_handle h, int enable);
int oic_kernel_class_count(void);
int oic_kernel_stats(oic_handle h, int id, const char** name, long long* launches, double* total_ms);

/* Stream the handle orders its work on (a hipStream_t). */
void* oic_stream(oic_handle h);

/* Stage cost of the tracking objective (problem setup), in FP64 on the host:
 *   tr[(X - Xref)^T R^{-1} (X - Xref)] + tr[U^T Q^{-1} U] + tr[dU^T Q^{-1} dU],
 * with U^ref = 0 and Q_U = Q_dU = Q.  X, Xref: n x m; U, dU: l x m; Q: l x l; R: n x n
 * (host pointers).  Summed over the realised steps of a closed loop this is the
 * closed-loop tracking cost.  Errors: OIC_EINVAL (NULL, bad size, Q or R not SPD). */
int oic_stage_cost(int n, int m, int l, const float* X, const float* Xref, const float* U,
                   const float* dU, const float* Q, const float* R, double* cost);

/* Replay the kernel sequence of a solve from a HIP graph, captured on the first
 * solve of each (N, horizon, seeded or explicit noise) and reused while those stay
 * the same.  On by default.  While per-kernel timing is enabled the sequence is
 * launched kernel by kernel instead.  Results are identical either way. */
int oic_set_graph(oic_handle h, int enable);

/* A constraint observed through a barrier (the extension after Table 1 of the
 * paper): z_t = phi(g) + eps_t, phi(x) = ln(1 + exp(beta x)) / alpha, eps_t ~ N(0, rz),
 * is appended to Ybar_t as one more row whose actual value is 0, so that the
 * smoother steers away from g > 0.  The constraint is applied column by column as
 * the linear form g_c = aX . X_t[:, c] + aU . U_t[:, c] - b on each member's forecast
 * state and control (aX: n values, aU: l values, host pointers, copied).  Passing
 * aX = aU = NULL removes it.  alpha, beta, rz > 0.  With a constraint set, explicit-
 * noise solves also take Z_VZ (standard normals, H x N x m, index t-1 for step t);
 * seeded solves draw them as kind 4 of the stream (see oic_normals).  Needs
 * (N-1) m >= n + l + 1 and n + l + 1 <= 512. */
int oic_set_constraint(oic_handle h, const float* aX, const float* aU, float b, float alpha, float beta,
                       float rz);

/* Right transformation of the control (the extension after Table 1 of the paper):
 * when the system's actual input u_t has q < m columns, the method runs on
 * U_t = u_t T with a q x m matrix T of full row rank, and the smoothed control is
 * mapped back by least squares, u_hat = U_hat T^T (T T^T)^{-1}.  Host pointers,
 * row-major FP32, FP64 arithmetic inside; no GPU work.
 * oic_columns_expand:  U (l x m) = u (l x q) T (q x m).
 * oic_columns_project: u (l x q) = U (l x m) T^T (T T^T)^{-1}; OIC_ENOTSPD when T T^T is
 * not positive definite (T lacks full row rank), OIC_EINVAL for bad sizes (q > m). */
int oic_columns_expand(int l, int q, int m, const float* u, const float* T, float* U);
int oic_columns_project(int l, int m, int q, const float* U, const float* T, float* u);

/* ---- Groups: same-shape solves of several controllers in shared launches ----
 *
 * Serving many controllers (the closed loop of Algorithm 1 run for each of them) repeats
 * the same kernels with the same shapes.  A group holds `slots` handles of one
 * configuration whose device buffers lie in equal slabs of one allocation; one launch of
 * each kernel of a solve then serves any subset of the slots (the kernels' grids are
 * repeated over the slots), and that sequence is captured once into a HIP graph and
 * replayed for every batch.  Each slot computes exactly what its own solve computes, so
 * a slot's results are bitwise the same alone and in any batch.
 *
 * Every slot is an ordinary handle (oic_group_slot) for oic_set_weights, oic_set_u_prev,
 * oic_get_u_prev and solves of its own; it belongs to the group (oic_destroy ignores it)
 * and a slot without bias for a layer holds a zero bias (identical results).  A group
 * solve and calls on its slots must not overlap.  Several slots per group need
 * precision OIC_PREC_BF16 with a BF16 kernel for every layer (OIC_EINVAL otherwise);
 * one slot takes any configuration.  A batch whose solve would need a kernel without a
 * grouped form (N*m not a multiple of 4, n + l above 448) fails with OIC_EINVAL and
 * writes no output; its slots can still solve one at a time. */
#define OIC_MAX_GROUP_SLOTS 64
typedef struct oic_group* oic_group_handle;

/* Device bytes of a group of `slots` slots created with cfg. */
size_t oic_group_footprint_bytes(const oic_config* cfg, int slots);

/* A group of 1..OIC_MAX_GROUP_SLOTS slots, each as oic_create(cfg) would make it.
 * OIC_EINVAL (bad configuration or slot count), OIC_ENOMEM, OIC_EDEVICE. */
int oic_group_create(const oic_config* cfg, int slots, oic_group_handle* out);

/* Frees the group and its slots.  NULL-safe. */
void oic_group_destroy(oic_group_handle g);

/* The handle of slot `slot` (0 <= slot < slots), or NULL. */
oic_handle oic_group_slot(oic_group_handle g, int slot);

/* One solve (as oic_solve_ex, Algorithm 1 lines 4-13) for each of `count` distinct
 * slots: request i runs on slot slots[i] with args[i] (array memory per the group's
 * mem_mode), in one launch per kernel for all of them on slot 0's stream.  The
 * requests share N, horizon, the noise source (seeded or explicit) and whether Q and R
 * are diagonal; a request that differs, or whose slot has a constraint, covariance
 * outputs or timing set, fails alone.  rc_out (NULL or count ints) receives each
 * request's status; the return value is the first failure's (OIC_OK if none), and
 * oic_group_last_error names its slot and reason.  A request that fails writes no
 * output.  count 1 is the slot's own solve. */
int oic_group_solve(oic_group_handle g, int count, const int* slots, const oic_solve_args* args, int* rc_out);

/* Reason for the last failed oic_group_solve. */
const char* oic_group_last_error(oic_group_handle g);

/* ---- Serving: one request loop for many independent controllers ----
 *
 * A server owns a set of controllers.  Controllers of one shape (grid, control rows,
 * layer widths, activation, precision, N, horizon) are resident in the slots of packs,
 * each pack a group (see above) with its device-resident ensemble buffers, captured
 * grouped solve and every slot's applied-control state U_prev, carried from solve to
 * solve.  Requests (one MPC solve each) are admitted and batched continuously: a pool
 * of max_inflight worker threads takes the oldest request whose controller can run
 * (resident in a pack that is not solving, or placeable in a free slot, in the slot of
 * an idle controller of its shape, or in a new pack whose footprint fits the HBM
 * budget after evicting least-recently-used idle packs; U_prev of a controller that
 * leaves its slot is kept on the host), then adds the oldest queued requests of other
 * controllers that the pack can take, up to its slot count, and runs them as one
 * grouped solve.  Otherwise the request waits.  Packs solve concurrently; solves of one
 * controller run in submission order.  A pack has several slots where one solve of its
 * shape leaves the GPU idle (BF16 rollout, fewer than about 2^22 pixels x members),
 * no more than the controllers of the shape and the budget allow.  Each result is the
 * same as the controller's solve alone.  All array arguments are HOST pointers,
 * copied before the call returns. */
typedef struct oic_server* oic_server_handle;

/* Device bytes the server holds for a controller of cfg alone in its pack (the smallest
 * admission footprint; a pack of k slots holds oic_group_footprint_bytes(cfg, k)). */
size_t oic_footprint_bytes(const oic_config* cfg);

/* hbm_budget_bytes: device bytes the server may hold for controller buffers.
 * max_inflight: worker threads = solves on the device at once (1..64). */
int oic_server_create(size_t hbm_budget_bytes, int max_inflight, oic_server_handle* out);

/* Stops the workers (after their current solves) and frees every controller. NULL-safe. */
void oic_server_destroy(oic_server_handle s);

/* Largest slot count of a pack (1..OIC_MAX_GROUP_SLOTS, default 8; 1: every controller
 * solves on its own, concurrently with the others).  Only before the first request:
 * OIC_EINVAL afterwards. */
int oic_server_set_group_slots(oic_server_handle s, int max_slots);

/* Register a controller: cfg as for oic_create (mem_mode must be OIC_MEM_HOST;
 * max_N, max_H and stream are ignored), surrogate as for oic_set_weights, and the
 * fixed ensemble size N, horizon, Q and R of its solves.  Nothing is allocated on
 * the device until its first request.  OIC_ENOMEM if its footprint exceeds the budget. */
int oic_server_add(oic_server_handle s, const oic_config* cfg, const float* B, const float* const* W,
                   const float* const* bias, int N, int horizon, const float* Q, const float* R,
                   int* controller_id);

/* Queue one solve for a controller: X0 (n x m) and reference ((horizon+1) x n x m)
 * as for oic_solve, with the seeded noise stream.  *ticket identifies the result. */
int oic_server_submit(oic_server_handle s, int controller_id, const float* X0, const float* reference,
                      uint64_t seed, long long* ticket);

/* Block until the ticket's solve has finished and copy its outputs: U_out
 * ((horizon+1) x l x m), X_out ((horizon+1) x n x m) or NULL.  latency_ms (submit to
 * completion) and queue_ms (submit to start) may be NULL.  Returns the solve's
 * status; each ticket can be waited for once. */
int oic_server_wait(oic_server_handle s, long long ticket, float* U_out, float* X_out,
                    double* latency_ms, double* queue_ms);

/* Counters: completed solves, controller admissions into a slot and evictions from one,
 * admissions that took over the slot of an idle controller of the same shape (weights
 * and U_prev swapped in place, no device allocation), device bytes held now and at
 * peak. Any pointer may be NULL. */
int oic_server_stats(oic_server_handle s, long long* completed, long long* admissions,
                     long long* evictions, long long* recycled, size_t* bytes_in_use, size_t* peak_bytes);

/* Batching counters: batches run (grouped solves, one or more requests each), requests
 * solved in batches of two or more, and packs created.  Any pointer may be NULL. */
int oic_server_batch_stats(oic_server_handle s, long long* batches, long long* grouped_solves,
                           long long* packs_created);

/* Reason for the last failed oic_server_wait. */
const char* oic_server_last_error(oic_server_handle s);

#ifdef __cplusplus
}
#endif

#endif /* OIC_H */
