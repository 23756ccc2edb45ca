/*
 * pi2rh.h -- C ABI of the MI355X (gfx950) PI^2-RH rollout library.
 *
 * Receding-horizon path-integral control with a learned LWPR dynamics model,
 * after Williams, Rombokas and Daniel, "GPU based Path Integral Control with
 * Learned Dynamics" (arXiv:1503.00330).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers marked "dev" are device (HBM) pointers; "host" pointers are read
 *    only during the call.  Every buffer is owned by the caller.  No entry
 *    point allocates device or pinned memory; scratch space is the caller's
 *    workspace `ws` of at least pi_workspace_bytes(...) bytes (except for
 *    pi_rollout_cost_noalloc, whose scratch is a static device array).
 *  - All device work is enqueued on `stream` (a hipStream_t; NULL = the null
 *    stream) and is asynchronous; results are valid once the stream has been
 *    synchronised.  Because nothing is allocated and nothing is copied from
 *    host memory, every call may be captured into a HIP graph.
 *  - Validation runs before any device work.  On failure a call returns a
 *    non-zero pi_status, enqueues nothing, writes nothing and records a
 *    message for pi_last_error().  A failed kernel launch maps to
 *    PI_ERR_DEVICE.  No C++ exception crosses this interface.
 *  - `dtype` of a problem and of its model must agree.  PI_F32 computes in
 *    single precision (the update's normalisation and weighted sums are
 *    always double; the pieces variants, PI_VARIANT_MFMA_BF16X3 and
 *    PI_VARIANT_MFMA_F16X2, form the mixture contraction's float32 products
 *    from 16-bit pieces on the matrix cores, to float32 accuracy); PI_F64
 *    runs the same method entirely in double.
 *  - Non-finite inputs propagate (NaN/Inf in x0, u_nom or a model parameter
 *    reach the affected costs and updates as they would in exact IEEE
 *    arithmetic).  The one clamp: the spread term sum_j w_j (y_j - mean)^2 of
 *    the mixture variance (Eq. 1), non-negative by definition, is held at
 *    >= 0 where float32 rounding of its running form would make it negative.
 */
#ifndef PI2RH_H_
#define PI2RH_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PI_OK = 0,
  PI_ERR_NULL = 1,        /* a required pointer is NULL                       */
  PI_ERR_SHAPE = 2,       /* a size is out of range or inconsistent           */
  PI_ERR_VALUE = 3,       /* a scalar is out of its domain (dt <= 0, ...)     */
  PI_ERR_DTYPE = 4,       /* unknown dtype or problem/model dtype mismatch    */
  PI_ERR_WORKSPACE = 5,   /* workspace NULL or smaller than required          */
  PI_ERR_DEVICE = 6,      /* no usable gfx950 device or a launch failed       */
  PI_ERR_UNSUPPORTED = 7  /* valid request the library does not implement     */
} pi_status;

typedef enum { PI_F32 = 0, PI_F64 = 1 } pi_dtype;

/* Dynamics families; every step is explicit Euler with the LWPR outputs as
 * accelerations.
 *   POINTMASS2D: state [px,py,vx,vy], control 2, z = [state ; control] (d = 6),
 *                outputs [ax,ay]
 *   QUAD12:      state [p(3), v(3), euler(3), rates(3)], control 4,
 *                z = [state ; control] (d = 16),
 *                outputs [linear acc(3), angular acc(3)]
 *   QUAD_HYBRID: the paper's quadrotor model (Sec. 4.1): state [p(3), v(3),
 *                euler(3)], control [commanded euler rates(3), thrust F];
 *                the angles follow d(euler)/dt = 25 (commanded - euler), and
 *                three LWPR models of z = [euler(3), F] (d = 4) give the
 *                linear accelerations (outputs 3)                            */
enum { PI_DYN_POINTMASS2D = 0, PI_DYN_QUAD12 = 1, PI_DYN_QUAD_HYBRID = 2 };
/* Obstacle term of the state cost q(x) (Sec. 5): an indicator with a fixed
 * penalty for being strictly inside any disc/vertical cylinder, or the smooth
 * form penalty * sum_i exp(-decay * (dx_i^2 + dy_i^2)).                     */
enum { PI_OBS_INDICATOR = 0, PI_OBS_SMOOTH = 1 };
/* Weighting of the update: Eq. (2) with the cost-to-go S(tau_i) of every
 * time step (default), or the whole-trajectory cost S(tau_0) for all steps. */
enum { PI_W_COST_TO_GO = 0, PI_W_TRAJECTORY = 1 };
/* Kernel variants.  The matrix-core form (PI_VARIANT_MFMA) needs float32,
 * d in {4, 6, 16} and folded tiles under 2 GiB (about 3 M local models at
 * d = 16); PI_VARIANT_AUTO picks it whenever those hold, and requesting it
 * otherwise returns PI_ERR_UNSUPPORTED.  PI_VARIANT_DIRECT is the per-sample
 * form (any d, float32 or float64).  PI_VARIANT_MFMA_BF16X3 (rollouts of the
 * float32 12-state quadrotor, d = 16; 8 waves need tiles of <= 16) runs the same
 * contraction on the bf16 matrix instructions: every float32 operand is the
 * exact sum of three bf16 pieces and the six piece products of weight at
 * least 2^-24 are summed in float32, which reproduces the float32 products
 * to within float32 rounding.  With it, tiles of 33..128 samples select the
 * shared-tile launch: 128 rows, 16 per wave on 8 waves or 32 on 4, and the
 * workgroup stages every model tile once in LDS (for problems with many
 * rollouts).  PI_VARIANT_MFMA_F16X2 (the same rollouts and launch shapes)
 * runs it on the fp16 matrix instructions: each model's coefficients and
 * each sample row's features are scaled by powers of two that keep them
 * below 2^14, every scaled value is the sum of two fp16 pieces (hi, lo; lo
 * may be subnormal) and the three piece products hi hi, hi lo, lo hi are
 * summed in float32, half the products of the bf16 form, to about 2^-22
 * relative per product; the scales are undone exactly in float32.  For
 * both, tile_samples 0 means the shared tile (128 samples, 8 waves) when
 * K max(M,1) >= 32768, else the 16-sample tiles.  Neither form has a
 * prediction entry point (lwpr_predict: PI_ERR_UNSUPPORTED).                */
enum { PI_VARIANT_AUTO = 0, PI_VARIANT_DIRECT = 1, PI_VARIANT_MFMA = 2, PI_VARIANT_MFMA_BF16X3 = 3,
       PI_VARIANT_MFMA_F16X2 = 4 };
/* Operations for pi_workspace_bytes. */
enum { PI_OP_PREDICT = 0, PI_OP_ROLLOUT = 1, PI_OP_UPDATE = 2, PI_OP_ADJOINT = 3,
       PI_OP_RH_SHIFT = 4 };

enum { PI_MAX_OUT = 8, PI_MAX_U = 4, PI_MAX_D = 16, PI_MAX_R = 16, PI_MAX_OBS = 64 };

/* n_out independent LWPR mixtures over one input z in R^d (Sec. 2, Eq. 1).
 * Local model j has centre c_j, distance metric D_j, PLS projection
 * directions u_{j,r}, deflation loadings p_{j,r}, regression coefficients
 * beta_{j,0..R} and a local noise variance sigma_j^2.  The models of output o
 * are rows L_off[o] .. L_off[o+1]-1 of every array; Ltot = L_off[n_out].
 * Arrays are dense row-major in the model's dtype.                           */
typedef struct {
  int32_t dtype;                   /* pi_dtype                               */
  int32_t d, n_out, R;             /* 1<=d<=16, 1<=n_out<=8, 0<=R<=16        */
  int32_t L_off[PI_MAX_OUT + 1];   /* host; L_off[0]=0, nondecreasing, each output >= 1 model */
  const void *centre;              /* dev [Ltot][d]                          */
  const void *metric;              /* dev [Ltot][d][d]  (only the symmetric part matters) */
  const void *proj_u;              /* dev [Ltot][R][d]                       */
  const void *proj_p;              /* dev [Ltot][R][d], or NULL for p = u    */
  const void *beta;                /* dev [Ltot][R+1]                        */
  const void *sigma2;              /* dev [Ltot], >= 0                       */
  const void *folded;              /* dev, optional: this model's folded forms as
                                    * written by pi_model_fold.  When non-NULL,
                                    * prediction, rollouts and the RH shift read
                                    * them instead of folding the model into their
                                    * workspace on every call; the caller re-folds
                                    * after changing any model array.           */
  size_t folded_bytes;             /* size of `folded` (>= pi_model_fold_bytes) */
} pi_lwpr;

/* One PI^2-RH instance (Sec. 3.1, 3.2, 5). */
typedef struct {
  int32_t dtype;                   /* pi_dtype                               */
  int32_t dyn;                     /* PI_DYN_*                               */
  int32_t K, T;                    /* rollouts (>=1) and horizon (>=1)       */
  int32_t M;                       /* 0: mean-only rollouts; >=1: M sampled sub-rollouts per rollout (Sec. 3.2) */
  double dt, lambda;               /* step (>0) and temperature (>0)         */
  double noise_std[PI_MAX_U];      /* control noise std per control (>=0)    */
  double goal[3], w_pos[3];        /* goal and per-axis position weights     */
  double w_ang, w_vel;             /* weights of |euler|^2 and |v|^2         */
  int32_t obs_kind, n_obs;         /* PI_OBS_*, 0 <= n_obs <= 64             */
  const void *obs;                 /* dev [n_obs][3] = (cx, cy, r), problem dtype; may be NULL if n_obs = 0 */
  double obs_penalty, obs_decay;   /* indicator penalty / smooth amplitude, smooth decay */
  int32_t weighting;               /* PI_W_*                                 */
  uint32_t problem_id;             /* counter word of the random stream      */
  uint64_t seed;                   /* Philox key                             */
  int32_t variant;                 /* PI_VARIANT_* (0 = library's choice)    */
  int32_t tile_samples;            /* samples per workgroup, <= 32, or <= 128 with
                                    * PI_VARIANT_MFMA_BF16X3 or _F16X2 (0 =
                                    * library's choice) */
  int32_t tile_waves;              /* waves per workgroup, 4 or 8 (8: 12-state
                                    * quadrotor only); 0 = library's choice:
                                    * 8 for the quadrotor when the launch has
                                    * at most one workgroup per compute unit,
                                    * else 4                                  */
  int32_t tile_split;              /* workgroups per tile of 16 samples: 1 (one
                                    * workgroup runs every local model) or 2 (a
                                    * pair of workgroups, on two compute units,
                                    * each runs half and they exchange partial
                                    * sums every step); 0 = library's choice:
                                    * 2 when the problem has fewer tiles than
                                    * the device has compute units and the
                                    * pairs fit on the device at once.  Float32
                                    * matrix-core rollouts with tile_samples
                                    * <= 16 (4 waves, or 8 for the quadrotor)
                                    * only; otherwise 1.                       */
  int32_t ctrl_cost;               /* 1: add the control terms of the
                                    * cost-to-go S-tilde (Sec. 3.1, below
                                    * Eq. 2), which the experiments drop
                                    * (Sec. 5), to every step's cost:
                                    * u^T G_c^T H^-1 G_c u dt + u^T G_c^T H^-1 B dw
                                    * with u the nominal control.  Hybrid model
                                    * only (PI_ERR_UNSUPPORTED otherwise): its
                                    * commanded rates are the control-affine
                                    * channel, G_c = 25 I, the noise enters
                                    * through it (B dw = G_c eps dt) and
                                    * B B^T = lambda G_c R^-1 G_c^T fixes
                                    * R = lambda diag(1/sigma^2)/dt, so the terms
                                    * are sum_a lambda/sigma_a^2 u_a (u_a + eps_a)
                                    * over the three rates; noise_std[0..2]
                                    * must be > 0 (PI_ERR_VALUE).  0: off.     */
} pi_problem;

/* Bytes of workspace `op` needs for this problem/model (0 is a valid answer;
 * a NULL ws is accepted then).  Returns (size_t)-1 and sets pi_last_error()
 * if the arguments are invalid.  For PI_OP_PREDICT, `p` may be NULL and the
 * query count is taken as p ? p->K : 0 (prediction needs no per-query space). */
size_t pi_workspace_bytes(int32_t op, const pi_problem *p, const pi_lwpr *m);

/* Model folding (Sec. 2 local models, Eq. 1): the PLS chain of every local
 * model reduces to an affine map y = beta0 + b.(z - c); the kernels read the
 * model in folded forms -- per-model records (c, D + D^T packed, b, beta0,
 * sigma^2) and, for float32 with d in {6, 16}, the matrix-core tiles.
 * pi_model_fold_bytes gives the size of both (or (size_t)-1 on an invalid
 * model); pi_model_fold writes them to `folded` (dev, caller-owned, at least
 * that many bytes), stream-ordered.  Pass the buffer in pi_lwpr.folded to skip
 * the per-call fold.                                                          */
size_t pi_model_fold_bytes(const pi_lwpr *m);
pi_status pi_model_fold(const pi_lwpr *m, void *folded, size_t folded_bytes, void *stream);

/* The launch pi_rollout_cost would make for this problem and model on the
 * current device (no work is done): out[0] = PI_VARIANT_DIRECT or
 * PI_VARIANT_MFMA, out[1] = samples per tile, out[2] = waves per workgroup,
 * out[3] = workgroups per tile (1 or 2, see tile_split).  out is a host array
 * of 4.  Returns PI_ERR_* for invalid arguments as pi_rollout_cost would.   */
pi_status pi_rollout_describe(const pi_problem *p, const pi_lwpr *m, int32_t *out);

/* Eq. (1): for N inputs Z (dev [N][d]) writes the mixture mean and variance
 * of every output: mean, var dev [N][n_out] in the model's dtype.
 * `variant` selects the kernel (PI_VARIANT_*).                               */
pi_status lwpr_predict(const pi_lwpr *m, const void *Z, int64_t N, void *mean, void *var,
                       int32_t variant, void *ws, size_t ws_bytes, void *stream);

/* Sampled rollouts (Sec. 3.1 cost-to-go, Sec. 3.2 sub-rollouts): for every
 * rollout k and sub-rollout m, from x0 (dev [n_x]) under the controls
 * u_nom[t] + eps_{k,t} (u_nom dev [T][n_u]; eps = noise_std * N(0,I) from the
 * random stream, shared by the sub-rollouts of k), the next state is drawn
 * from the LWPR prediction N(mean, var) (mean only when M = 0) and advanced by
 * explicit Euler; the step cost is dt * q(x_{t+1}).  Writes
 *   cost dev [K][T]: cbar_{k,t} = mean over sub-rollouts of the step cost,
 * so S_k = sum_t cost[k][t].  `iter` (dev, one uint32) is the iteration
 * counter of the random stream.  With paired workgroups (tile_split) every
 * wait of a workgroup on its partner is bounded; should one run out (the
 * pair was not resident at once), that pair abandons its tile: its costs are
 * written as NaN from that step on (never finite values from a half whose
 * state went stale) and the abandonment is counted (pi_pair_give_ups).
 * The library pairs only grids that fit the device's compute units at once;
 * the 8-wave paired grid of the library's choice can fill them exactly (one
 * workgroup per unit), so a caller that runs other kernels concurrently on
 * the same device passes tile_waves 4 (or tile_split 1).                   */
pi_status pi_rollout_cost(const pi_problem *p, const pi_lwpr *m, const void *x0,
                          const void *u_nom, const uint32_t *iter, void *cost, void *ws,
                          size_t ws_bytes, void *stream);

/* Workgroups of paired rollout launches (pi_rollout_cost with tile_split)
 * that abandoned their tile because a bounded wait on their partner ran out,
 * counted on the current device since the library was loaded: writes one
 * uint64 to *count (dev), stream-ordered after the launches before it.  Read
 * it before and after a launch: an increase means some of that launch's costs
 * are NaN.  (The environment variable PI2RH_PAIR_SPIN_LIMIT, read at each
 * launch, sets the polls of one wait -- for tests that force a give-up.)     */
pi_status pi_pair_give_ups(uint64_t *count, void *stream);

/* Allocation-free sampled rollouts, for callers that cannot allocate device
 * memory or size a workspace (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): pi_rollout_cost with the same
 * arguments, results and launches, minus the workspace.  Its scratch (the
 * folded model unless pi_lwpr.folded is given, the sub-rollout costs when
 * M > 1 and the pair-exchange slots) lives in a static device array of
 * PI_NOALLOC_SCRATCH_BYTES per device, held from the first call on a device
 * until the process ends; a rollout whose pi_workspace_bytes(PI_OP_ROLLOUT)
 * exceeds it returns PI_ERR_WORKSPACE and enqueues nothing.  Calls allocate
 * nothing; the first call on a device looks up the array's address (make it
 * outside stream capture).  Every call on a device shares that one array:
 * calls that overlap on the same device (concurrent streams or host threads)
 * race and give undefined costs; calls ordered on one stream are safe.      */
enum { PI_NOALLOC_SCRATCH_BYTES = 32 << 20 };
pi_status pi_rollout_cost_noalloc(const pi_problem *p, const pi_lwpr *m, const void *x0,
                                  const void *u_nom, const uint32_t *iter, void *cost,
                                  void *stream);

/* Path-integral update, Eq. (2): S_{k,i} = sum_{t>=i} cost[k][t] (or S_{k,0}
 * for PI_W_TRAJECTORY); P_{k,i} = softmax_k(-S_{k,i}/lambda);
 * u_nom[i] += sum_k P_{k,i} eps_{k,i}, with eps regenerated from the same
 * stream.  cost dev [K][T] (problem dtype), u_nom dev [T][n_u] in/out,
 * weights dev [T][K] double (nullable).  Normalisation and sums in double.
 * The iteration's draws are then consumed: *iter (dev) is incremented, so
 * the next rollout of the same control step draws fresh noise.               */
pi_status pi_update(const pi_problem *p, const void *cost, const uint32_t *iter, void *u_nom,
                    void *weights, void *ws, size_t ws_bytes, void *stream);

/* Receding-horizon advance (Sec. 3.1, last paragraph): executes u_nom[0] on
 * the plant -- a draw from the learned model under the PLANT stream at the
 * current *iter (dev, read only) -- writing the new state to x0 (dev [n_x],
 * in/out), and shifts u_nom left by one step (repeating the last control).  */
pi_status pi_rh_shift(const pi_problem *p, const pi_lwpr *m, void *x0, void *u_nom,
                      const uint32_t *iter, void *ws, size_t ws_bytes, void *stream);

/* Adjoint of the expected rollout cost with the noise held fixed
 * (reparameterised; not in the paper, which optimises by sampling alone):
 *   J = (1/(K max(M,1))) sum_{k,m,t} dt q(x_{k,m,t+1}),
 * the mean over sub-rollouts of the sampled cost S of Sec. 3.1/3.2 under the
 * LWPR dynamics of Eq. (1).  Writes J (dev, one double, unscaled) and the
 * gradients of gJ * J w.r.t. the nominal controls g_u_nom dev [T][n_u], the
 * centres g_centre dev [Ltot][d] and every entry of the metrics g_metric dev
 * [Ltot][d][d] (problem dtype; the metric gradient is symmetric).  gJ (dev,
 * one double) seeds the reverse pass; NULL means 1.  States are checkpointed
 * every `ckpt_every` steps (0: ceil(sqrt(T))) and each segment is recomputed
 * from its checkpoints before its reverse sweep, so the workspace holds the
 * checkpoints and one segment: pi_adjoint_workspace_bytes(p, m, ckpt_every)
 * (or pi_workspace_bytes(PI_OP_ADJOINT), for ckpt_every 0).  Float32
 * problems whose model has a matrix-core form (see PI_VARIANT_MFMA; variant
 * not PI_VARIANT_DIRECT) run the forward, the recompute and the reverse sweep
 * on the matrix cores and keep per-step records for one segment only; the
 * direct kernels (float64, PI_VARIANT_DIRECT) keep them for every step.
 * With PI_VARIANT_MFMA_BF16X3 or PI_VARIANT_MFMA_F16X2 (the float32 12-state
 * quadrotor with d = 16; PI_ERR_UNSUPPORTED otherwise) the forward and the
 * segment recomputes run that contraction, the reverse sweep and the
 * parameter pass the float32 one, with the forward's traced anchors and
 * normalisers.  The indicator obstacle term has zero derivative almost
 * everywhere.
 * (PI_DYN_POINTMASS2D and PI_DYN_QUAD12 without ctrl_cost;
 * PI_ERR_UNSUPPORTED otherwise.)                                             */
size_t pi_adjoint_workspace_bytes(const pi_problem *p, const pi_lwpr *m, int32_t ckpt_every);
pi_status pi_rollout_adjoint(const pi_problem *p, const pi_lwpr *m, const void *x0,
                             const void *u_nom, const uint32_t *iter, int32_t ckpt_every,
                             const void *gJ, void *J, void *g_u_nom, void *g_centre,
                             void *g_metric, void *ws, size_t ws_bytes, void *stream);

/* Batched controllers: B independent PI^2-RH problems (Sec. 3.1, 3.2 each;
 * batching is this library's, not the paper's) that may differ in K, T, M,
 * models, obstacles, goals and start states, with every problem's rollout
 * tiles in one persistent launch: a grid sized to the device pulls (problem,
 * tile) work items, ordered by decreasing work, from a queue.  Per-problem
 * arrays are host arrays of B device pointers: x0[b] [n_x], u_nom[b]
 * [T_b][n_u], iter[b] (one uint32), cost[b] [K_b][T_b].  All problems must be
 * PI_F32 and PI_DYN_QUAD12 with matrix-core models (PI_ERR_UNSUPPORTED
 * otherwise).  A problem's tile_samples (<= 32, or <= 128 when the batch
 * runs the bf16x3 or f16x2 form; 0 = 16, or 128 in the f16x2 form) sets
 * its tile; the variant and tile_waves of problem 0 apply to the batch (8
 * waves need every tile <= 16, or the largest above 32 in the pieces forms).
 * Models given pre-folded (pi_lwpr.folded) are read in place; the others are
 * folded into the workspace on every call.  The launch plan (descriptors and
 * work list) is written into the workspace by kernels on `stream`, so these
 * calls copy no host memory and may be captured into a HIP graph.
 *
 * pi_batched_workspace_bytes: the workspace of either call ((size_t)-1 and
 * pi_last_error() on invalid arguments).
 * pi_rollout_cost_batched: writes every cost[b] exactly as pi_rollout_cost
 * would with one 4-wave (or tile_waves) workgroup per tile (tile_split 1).
 * pi_control_step_batched: the same rollouts, then per problem, in problem
 * order, the update of pi_update (Eq. 2; *iter[b] advances) and the
 * receding-horizon advance of pi_rh_shift (Sec. 3.1, last paragraph):
 * x0[b], u_nom[b] and iter[b] end exactly as after one plain control step
 * (pi_rollout_cost, pi_update, pi_rh_shift) of each problem.                 */
size_t pi_batched_workspace_bytes(int32_t B, const pi_problem *p, const pi_lwpr *m);
pi_status pi_rollout_cost_batched(int32_t B, const pi_problem *p, const pi_lwpr *m,
                                  const void *const *x0, const void *const *u_nom,
                                  const uint32_t *const *iter, void *const *cost, void *ws,
                                  size_t ws_bytes, void *stream);
pi_status pi_control_step_batched(int32_t B, const pi_problem *p, const pi_lwpr *m,
                                  void *const *x0, void *const *u_nom, uint32_t *const *iter,
                                  void *const *cost, void *ws, size_t ws_bytes, void *stream);

/* Streams of the counter-based generator (see pi_noise). */
enum { PI_TAG_CTRL = 0, PI_TAG_DYN = 1, PI_TAG_PLANT = 2 };

/* Raw Philox4x32-10 blocks (Salmon et al., SC'11) as used by every kernel:
 * ctr dev [N][4] uint32 counters, key = (low word, high word) of `key`,
 * out dev [N][4] uint32.                                                     */
pi_status pi_philox4x32_10(const uint32_t *ctr, uint64_t key, uint32_t *out, int64_t N,
                           void *stream);

/* The random draws of the method exactly as the kernels form them, for
 * rollouts k0 .. k0+nk-1 and all T steps at iteration *iter:
 *   PI_TAG_CTRL : eps_{k,t} = noise_std * N(0, I)      out [nk][T][n_u]
 *   PI_TAG_DYN  : xi_{k,m,t} ~ N(0, I) of sub-rollout m out [nk][T][n_out]
 *   PI_TAG_PLANT: the plant draw of pi_rh_shift        out [n_out] (k0, nk, m ignored)
 * The counter of draw (tag, k, m, t) is (t, k, (m << 4) | block,
 * tag << 30 | (problem_id & 0x3FF) << 20 | (iter & 0xFFFFF)); uniforms are
 * ((r >> 9) + 0.5) 2^-23 and normals come from Box-Muller pairs.  `out` is in
 * the problem's dtype.                                                       */
pi_status pi_noise(const pi_problem *p, int32_t tag, const uint32_t *iter, int32_t k0, int32_t nk,
                   int32_t m, void *out, void *stream);

/* Thread-local message of the last non-OK status ("" if none). */
const char *pi_last_error(void);

/* Library version string and the device architecture it was built for. */
const char *pi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PI2RH_H_ */
