// C ABI of the PI^2-RH library: argument validation, workspace layout and
// kernel dispatch.  Every check runs before the first device call; no entry
// point allocates memory.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "internal.hpp"

using namespace pi2rh;

// Workspace of pi_rollout_cost_noalloc (folded model, sub-rollout costs,
// pair-exchange slots), used instead of a caller buffer.  Each device the
// library runs on holds its own copy until the process ends.  In host code
// `scratch` names a host-side stand-in, never the device memory: kernels
// receive the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[PI_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local char g_err[512] = "";

pi_status fail(pi_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

// The current message prefixed by "problem b: " (the message is copied first:
// formatting g_err into itself would overlap).
pi_status fail_problem(pi_status st, int b) {
  char msg[sizeof(g_err)];
  snprintf(msg, sizeof(msg), "%s", g_err);
  return fail(st, "problem %d: %s", b, msg);
}

pi_status ok() {
  g_err[0] = 0;
  return PI_OK;
}

#define PI_TRY(expr)                  \
  do {                                \
    pi_status _st = (expr);           \
    if (_st != PI_OK) return _st;     \
  } while (0)

int dyn_nx(int dyn) { return dyn == PI_DYN_POINTMASS2D ? 4 : dyn == PI_DYN_QUAD_HYBRID ? 9 : 12; }
int dyn_nu(int dyn) { return dyn == PI_DYN_POINTMASS2D ? 2 : 4; }
int dyn_no(int dyn) { return dyn == PI_DYN_POINTMASS2D ? 2 : dyn == PI_DYN_QUAD_HYBRID ? 3 : 6; }
// LWPR input size: [state ; control], or [euler angles ; thrust] for the hybrid model
int dyn_d(int dyn) { return dyn == PI_DYN_QUAD_HYBRID ? 4 : dyn_nx(dyn) + dyn_nu(dyn); }

pi_status check_model(const pi_lwpr *m) {
  if (!m) return fail(PI_ERR_NULL, "model is NULL");
  if (m->dtype != PI_F32 && m->dtype != PI_F64) return fail(PI_ERR_DTYPE, "unknown model dtype %d", m->dtype);
  if (m->d < 1 || m->d > PI_MAX_D) return fail(PI_ERR_SHAPE, "d=%d outside [1,%d]", m->d, PI_MAX_D);
  if (m->n_out < 1 || m->n_out > PI_MAX_OUT)
    return fail(PI_ERR_SHAPE, "n_out=%d outside [1,%d]", m->n_out, PI_MAX_OUT);
  if (m->R < 0 || m->R > PI_MAX_R) return fail(PI_ERR_SHAPE, "R=%d outside [0,%d]", m->R, PI_MAX_R);
  if (m->L_off[0] != 0) return fail(PI_ERR_SHAPE, "L_off[0]=%d must be 0", m->L_off[0]);
  for (int o = 0; o < m->n_out; ++o)
    if (m->L_off[o + 1] <= m->L_off[o])
      return fail(PI_ERR_SHAPE, "output %d has no local models (L_off not increasing)", o);
  if (m->L_off[m->n_out] > (1 << 26)) return fail(PI_ERR_SHAPE, "too many local models");
  if (!m->centre || !m->metric || !m->beta || !m->sigma2 || (m->R > 0 && !m->proj_u))
    return fail(PI_ERR_NULL, "a required model array is NULL");
  return PI_OK;
}

pi_status check_problem(const pi_problem *p) {
  if (!p) return fail(PI_ERR_NULL, "problem is NULL");
  if (p->dtype != PI_F32 && p->dtype != PI_F64) return fail(PI_ERR_DTYPE, "unknown problem dtype %d", p->dtype);
  if (p->dyn != PI_DYN_POINTMASS2D && p->dyn != PI_DYN_QUAD12 && p->dyn != PI_DYN_QUAD_HYBRID)
    return fail(PI_ERR_VALUE, "unknown dyn %d", p->dyn);
  if (p->K < 1) return fail(PI_ERR_SHAPE, "K=%d must be >= 1", p->K);
  if (p->T < 1) return fail(PI_ERR_SHAPE, "T=%d must be >= 1", p->T);
  if (p->M < 0 || p->M > (1 << 27)) return fail(PI_ERR_SHAPE, "M=%d outside [0, 2^27]", p->M);
  if ((int64_t)p->K * (p->M > 0 ? p->M : 1) > (int64_t)INT32_MAX)
    return fail(PI_ERR_SHAPE, "K*max(M,1) exceeds 2^31-1");
  if ((int64_t)p->K * p->T > (int64_t)1 << 40) return fail(PI_ERR_SHAPE, "K*T too large");
  if (!(p->dt > 0) || !isfinite(p->dt)) return fail(PI_ERR_VALUE, "dt must be finite and > 0");
  if (!(p->lambda > 0) || !isfinite(p->lambda)) return fail(PI_ERR_VALUE, "lambda must be finite and > 0");
  for (int a = 0; a < dyn_nu(p->dyn); ++a)
    if (!(p->noise_std[a] >= 0)) return fail(PI_ERR_VALUE, "noise_std[%d] must be >= 0", a);
  if (p->obs_kind != PI_OBS_INDICATOR && p->obs_kind != PI_OBS_SMOOTH)
    return fail(PI_ERR_VALUE, "unknown obs_kind %d", p->obs_kind);
  if (p->n_obs < 0 || p->n_obs > PI_MAX_OBS) return fail(PI_ERR_SHAPE, "n_obs=%d outside [0,%d]", p->n_obs, PI_MAX_OBS);
  if (p->n_obs > 0 && !p->obs) return fail(PI_ERR_NULL, "obs is NULL with n_obs > 0");
  if (p->weighting != PI_W_COST_TO_GO && p->weighting != PI_W_TRAJECTORY)
    return fail(PI_ERR_VALUE, "unknown weighting %d", p->weighting);
  if (p->variant < PI_VARIANT_AUTO || p->variant > PI_VARIANT_MFMA_F16X2)
    return fail(PI_ERR_VALUE, "unknown variant %d", p->variant);
  // 128 only for the pieces forms (their shared-tile launch)
  const int max_spw = p->variant == PI_VARIANT_MFMA_BF16X3 || p->variant == PI_VARIANT_MFMA_F16X2 ? 128 : 32;
  if (p->tile_samples < 0 || p->tile_samples > max_spw)
    return fail(PI_ERR_VALUE, "tile_samples=%d outside [0,%d]", p->tile_samples, max_spw);
  if (p->tile_waves != 0 && p->tile_waves != 4 && p->tile_waves != 8)
    return fail(PI_ERR_VALUE, "tile_waves=%d must be 0, 4 or 8", p->tile_waves);
  if (p->tile_split < 0 || p->tile_split > 2)
    return fail(PI_ERR_VALUE, "tile_split=%d must be 0, 1 or 2", p->tile_split);
  if (p->ctrl_cost != 0 && p->ctrl_cost != 1) return fail(PI_ERR_VALUE, "ctrl_cost=%d must be 0 or 1", p->ctrl_cost);
  if (p->ctrl_cost) {
    if (p->dyn != PI_DYN_QUAD_HYBRID)
      return fail(PI_ERR_UNSUPPORTED, "ctrl_cost needs the hybrid model's control-affine rate channel");
    for (int a = 0; a < 3; ++a)
      if (!(p->noise_std[a] > 0) || !isfinite(p->noise_std[a]))
        return fail(PI_ERR_VALUE, "ctrl_cost needs finite noise_std[%d] > 0 (R = lambda diag(1/sigma^2)/dt)", a);
  }
  return PI_OK;
}

pi_status check_pair(const pi_problem *p, const pi_lwpr *m) {
  PI_TRY(check_problem(p));
  PI_TRY(check_model(m));
  if (p->dtype != m->dtype) return fail(PI_ERR_DTYPE, "problem dtype %d != model dtype %d", p->dtype, m->dtype);
  if (m->d != dyn_d(p->dyn))
    return fail(PI_ERR_SHAPE, "model input d=%d != %d for this dynamics family", m->d, dyn_d(p->dyn));
  if (m->n_out != dyn_no(p->dyn))
    return fail(PI_ERR_SHAPE, "model n_out=%d != %d accelerations", m->n_out, dyn_no(p->dyn));
  return PI_OK;
}

// Device check: a gfx950 device must be current.  Cached per device id.
constexpr int kMaxDevices = 64;

pi_status check_device() {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1) {
    (void)hipGetLastError();
    return fail(PI_ERR_DEVICE, "no HIP device available");
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(PI_ERR_DEVICE, "hipGetDevice failed");
  static std::mutex mu;
  static int known[kMaxDevices] = {0};  // 0 unknown, 1 ok, 2 wrong arch
  if (dev < 0 || dev >= kMaxDevices) return fail(PI_ERR_DEVICE, "device id out of range");
  std::lock_guard<std::mutex> lk(mu);
  if (known[dev] == 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(PI_ERR_DEVICE, "hipGetDeviceProperties failed");
    known[dev] = strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
    if (known[dev] == 2) return fail(PI_ERR_DEVICE, "device arch %s is not gfx950", prop.gcnArchName);
  }
  if (known[dev] == 2) return fail(PI_ERR_DEVICE, "device is not gfx950");
  return PI_OK;
}

pi_status launched(hipError_t e, const char *what) {
  if (e != hipSuccess) return fail(PI_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
  return ok();
}

ModelArgs model_args(const pi_lwpr *m) {
  ModelArgs a;
  a.d = m->d;
  a.n_out = m->n_out;
  a.R = m->R;
  a.Ltot = m->L_off[m->n_out];
  for (int o = 0; o <= kMaxOut; ++o) a.L_off[o] = o <= m->n_out ? m->L_off[o] : m->L_off[m->n_out];
  a.centre = m->centre;
  a.metric = m->metric;
  a.proj_u = m->proj_u;
  a.proj_p = m->proj_p;
  a.beta = m->beta;
  a.sigma2 = m->sigma2;
  return a;
}

template <typename Real>
ProbDev<Real> prob_dev(const pi_problem *p) {
  ProbDev<Real> d;
  d.dyn = p->dyn;
  d.K = p->K;
  d.T = p->T;
  d.M = p->M;
  d.Ms = p->M > 0 ? p->M : 1;
  d.n_x = dyn_nx(p->dyn);
  d.n_u = dyn_nu(p->dyn);
  d.n_out = dyn_no(p->dyn);
  d.d = dyn_d(p->dyn);
  d.dt = (Real)p->dt;
  for (int a = 0; a < kMaxU; ++a) d.noise_std[a] = (Real)p->noise_std[a];
  for (int a = 0; a < 3; ++a) {
    d.goal[a] = (Real)p->goal[a];
    d.w_pos[a] = (Real)p->w_pos[a];
  }
  d.w_ang = (Real)p->w_ang;
  d.w_vel = (Real)p->w_vel;
  d.obs_kind = p->obs_kind;
  d.n_obs = p->n_obs;
  d.obs = (const Real *)p->obs;
  d.obs_penalty = (Real)p->obs_penalty;
  d.obs_decay = (Real)p->obs_decay;
  d.key0 = (uint32_t)p->seed;
  d.key1 = (uint32_t)(p->seed >> 32);
  d.problem_id = p->problem_id;
  d.ctrl_cost = p->ctrl_cost;
  for (int a = 0; a < 3; ++a)
    d.ctrl_w[a] = p->ctrl_cost ? (Real)(p->lambda / (p->noise_std[a] * p->noise_std[a])) : (Real)0;
  return d;
}

bool mfma_ok(int dtype, int d) { return dtype == PI_F32 && (d == 16 || d == 6 || d == 4); }

// The matrix-core kernels address a model's folded tiles with 32-bit byte
// offsets: a model whose tiles would reach 2 GiB keeps the direct form.
bool mfma_model_ok(const pi_lwpr *m) {
  return mfma_ok(m->dtype, m->d) && mfma_layout(m->d, m->n_out, m->L_off).w_floats * 4 < ((size_t)1 << 31);
}

// The three-piece bf16 and two-piece fp16 contractions: float32, d = 16,
// their pieces (18 and 12 KB per tile of 16 models) addressable with 32-bit
// offsets.
bool bf_model_ok(const pi_lwpr *m) {
  if (!mfma_model_ok(m) || m->d != kBfD) return false;
  return mfma_layout(m->d, m->n_out, m->L_off).wb_u32 * 4 < ((size_t)1 << 31);
}

// Piece format of a requested variant (0: float32 products).
int variant_pf(int variant) {
  return variant == PI_VARIANT_MFMA_BF16X3 ? kPfBf16x3 : variant == PI_VARIANT_MFMA_F16X2 ? kPfF16x2 : kPfF32;
}

// Rollout variant, samples per workgroup and whether tiles may be split over
// a pair of workgroups (pair_ok; the launch decides with the device's
// compute-unit count and residency).  The workspace never depends on the
// device: a pair-capable plan always reserves the exchange slots.
struct RolloutPlan {
  bool mfma, bf, pair_ok;   // bf: a pieces form (pf != 0)
  int pf, spw, waves;
  int64_t groups;
};

constexpr int64_t kMaxPairGroups = 2048;
constexpr int64_t kSharedTileMinSamples = 128 * 256;

RolloutPlan rollout_plan(const pi_problem *p, const pi_lwpr *m) {
  RolloutPlan r;
  r.pf = variant_pf(p->variant);
  r.mfma = p->variant == PI_VARIANT_MFMA || r.pf != kPfF32 || (p->variant == PI_VARIANT_AUTO && mfma_model_ok(m));
  r.bf = r.pf != kPfF32;
  const int64_t n = (int64_t)p->K * (p->M > 0 ? p->M : 1);
  // the pieces forms' default for problems that fill a 256-unit device with
  // 128-sample tiles: the shared-tile launch on 8 waves
  const bool shared = r.bf && p->tile_samples == 0 && n >= (int64_t)kSharedTileMinSamples;
  r.waves = p->tile_waves > 0 ? p->tile_waves : shared ? 8 : 4;
  const bool split_allowed = r.mfma && (r.waves == 4 || (r.waves == 8 && p->dyn == PI_DYN_QUAD12)) &&
                             p->tile_split != 1 && p->dtype == PI_F32;
  if (p->tile_samples > 0) {
    r.spw = p->tile_samples;
  } else if (shared) {
    r.spw = 128;
  } else if (split_allowed) {
    r.spw = 16;   // full 16-row tiles; small problems are spread by pairing
  } else {
    // enough workgroups to cover the 256 compute units, at most 32 rows each
    r.spw = n >= 256 * 16 ? 16 : 8;
  }
  r.groups = (n + r.spw - 1) / r.spw;
  r.pair_ok = split_allowed && r.spw <= 16 && r.groups <= kMaxPairGroups;
  return r;
}

// The pieces forms' requirements (rollouts): the float32 12-state quadrotor
// with d = 16 pieces under 2 GiB; on 8 waves, tiles of at most 16 or more
// than 32 samples.
pi_status check_pieces(const pi_problem *p, const pi_lwpr *m, const RolloutPlan &pl) {
  if (!pl.bf) return PI_OK;
  if (p->dyn != PI_DYN_QUAD12 || !bf_model_ok(m))
    return fail(PI_ERR_UNSUPPORTED, "the %s contraction needs the float32 12-state quadrotor (d = 16) and pieces "
                                    "under 2 GiB", pl.pf == kPfF16x2 ? "f16x2" : "bf16x3");
  if (pl.spw > 16 && pl.spw <= 32 && p->tile_waves == 8)
    return fail(PI_ERR_UNSUPPORTED, "the %s contraction on 8 waves takes tiles of at most 16 or more than 32 "
                                    "samples", pl.pf == kPfF16x2 ? "f16x2" : "bf16x3");
  return PI_OK;
}

// Compute units of the current device (0 if the query fails).
int device_cus(int *dev_out = nullptr) {
  int dev = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (dev_out) *dev_out = dev;
  return n_cu;
}

// Pairing at launch: requested (tile_split 2) or, by default, when the tiles
// leave compute units idle; in both cases only if the whole grid is resident.
bool use_pair(const pi_problem *p, const RolloutPlan &pl) {
  if (!pl.pair_ok) return false;
  int dev = 0;
  const int n_cu = device_cus(&dev);
  if (n_cu == 0) return false;
  static std::mutex mu;
  // resident pair workgroups per compute unit, +1 (0 = unknown), by kernel:
  // point mass 0, hybrid 3, quadrotor 1 + (8 waves) + 3 pf (1..2, 4..5, 7..8)
  static int per_cu[kMaxDevices][9];
  if (dev < 0 || dev >= kMaxDevices) return false;
  const int di = p->dyn == PI_DYN_QUAD12 ? (pl.waves == 8 ? 2 : 1) + 3 * pl.pf
                                         : (p->dyn == PI_DYN_QUAD_HYBRID ? 3 : 0);
  int cap;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (per_cu[dev][di] == 0) per_cu[dev][di] = pair_blocks_per_cu(p->dyn, pl.waves, pl.pf) + 1;
    cap = per_cu[dev][di] - 1;
  }
  const bool resident = (int64_t)pair_grid(pl.groups) <= (int64_t)cap * n_cu;
  if (!resident) return false;
  return p->tile_split == 2 || pl.groups < n_cu;
}

// The rollout launch on the current device: the plan, whether its tiles are
// paired, and the waves per workgroup when the caller leaves them to the
// library.  With at most one workgroup per compute unit, eight waves (two per
// SIMD) keep the matrix cores busier than four; once workgroups share a unit
// they already do, and four waves are faster (12-state quadrotor, 16-row
// tiles; the other families have 4-wave kernels only).
struct RolloutLaunch {
  RolloutPlan pl;
  bool pair;
};

RolloutLaunch rollout_launch(const pi_problem *p, const pi_lwpr *m) {
  RolloutLaunch r{rollout_plan(p, m), false};
  r.pair = use_pair(p, r.pl);
  if (p->tile_waves == 0 && r.pl.mfma && p->dyn == PI_DYN_QUAD12 && r.pl.spw <= 16) {
    const int n_cu = device_cus();
    const int64_t wgs = r.pair ? 2 * r.pl.groups : r.pl.groups;
    if (n_cu > 0 && wgs <= n_cu) {
      RolloutPlan p8 = r.pl;
      p8.waves = 8;
      // a pair keeps four waves if its 8-wave grid would not be resident
      if (!r.pair || use_pair(p, p8)) r.pl = p8;
    }
  }
  return r;
}

// Layout of a pi_model_fold buffer: direct records, then (float32, d in
// {6, 16}) the matrix-core tiles.
struct FoldedLayout {
  size_t direct_off, mfma_off, bytes;
  bool has_mfma;
};
FoldedLayout folded_layout(const pi_lwpr *m) {
  FoldedLayout f;
  f.direct_off = 0;
  f.has_mfma = mfma_model_ok(m);
  f.mfma_off = align_up(direct_bytes(m->dtype, m->d, m->L_off[m->n_out]), 256);
  f.bytes = f.mfma_off + (f.has_mfma ? align_up(mfma_layout(m->d, m->n_out, m->L_off).bytes, 256) : 0);
  return f;
}

// Where the kernels read the folded model from: the caller's pi_model_fold
// buffer, or the start of the workspace after folding into it on `s`.
hipError_t folded_base(const pi_lwpr *m, bool mfma, void *ws, hipStream_t s, const void **base) {
  if (m->folded) {
    const FoldedLayout f = folded_layout(m);
    *base = (const char *)m->folded + (mfma ? f.mfma_off : f.direct_off);
    return hipSuccess;
  }
  *base = ws;
  const ModelArgs a = model_args(m);
  if (mfma) return launch_fold_mfma(m->dtype, a, mfma_layout(m->d, m->n_out, m->L_off), ws, s);
  return launch_fold_direct(m->dtype, a, ws, s);
}

pi_status check_folded(const pi_lwpr *m, bool mfma) {
  if (!m->folded) return PI_OK;
  const FoldedLayout f = folded_layout(m);
  if (m->folded_bytes < f.bytes)
    return fail(PI_ERR_WORKSPACE, "folded model of %zu bytes needed, %zu given", f.bytes, m->folded_bytes);
  if (mfma && !f.has_mfma) return fail(PI_ERR_UNSUPPORTED, "folded model has no matrix-core form");
  return PI_OK;
}

// The float32 adjoint runs its forward, recompute and reverse sweep on the
// matrix cores when the model has a matrix-core form: bytes of that form
// (tiles and reverse-sweep parameters), or 0 for the direct kernels.
size_t adjoint_mfma_bytes(const pi_problem *p, const pi_lwpr *m) {
  if (p->dtype != PI_F32 || !mfma_model_ok(m) || p->dyn == PI_DYN_QUAD_HYBRID) return 0;
  if (p->variant == PI_VARIANT_DIRECT) return 0;
  const MfmaLayout l = mfma_layout(m->d, m->n_out, m->L_off);
  return align_up(l.bytes, 256) + adj_rfold_bytes(l);   // forward tiles + reverse-sweep parameters
}

pi_status check_adjoint(const pi_problem *p, const pi_lwpr *m, int32_t ckpt_every, int *ckpt) {
  PI_TRY(check_pair(p, m));
  if (p->dyn == PI_DYN_QUAD_HYBRID) return fail(PI_ERR_UNSUPPORTED, "the adjoint covers POINTMASS2D and QUAD12");
  if (p->ctrl_cost) return fail(PI_ERR_UNSUPPORTED, "the adjoint does not cover the control terms of S-tilde");
  if (ckpt_every < 0) return fail(PI_ERR_VALUE, "ckpt_every=%d must be >= 0", ckpt_every);
  if ((int64_t)p->K * (p->M > 0 ? p->M : 1) * p->T > ((int64_t)1 << 36))
    return fail(PI_ERR_SHAPE, "K*max(M,1)*T too large for the adjoint records");
  if (variant_pf(p->variant) != kPfF32 && (p->dtype != PI_F32 || p->dyn != PI_DYN_QUAD12 || !bf_model_ok(m)))
    return fail(PI_ERR_UNSUPPORTED, "the adjoint's %s forward needs the float32 12-state quadrotor (d = 16) and "
                                    "pieces under 2 GiB", p->variant == PI_VARIANT_MFMA_F16X2 ? "f16x2" : "bf16x3");
  *ckpt = ckpt_every == 0 ? adjoint_default_ckpt(p->T) : std::min<int>(ckpt_every, p->T);
  return PI_OK;
}

size_t adjoint_ws(const pi_problem *p, const pi_lwpr *m, int ckpt) {
  return adjoint_ws_bytes(p->dtype, p->dyn, p->K, p->M, p->T, m->L_off[m->n_out], m->d, ckpt,
                          adjoint_mfma_bytes(p, m));
}

size_t fold_bytes(const pi_lwpr *m, bool mfma) {
  if (mfma) return mfma_layout(m->d, m->n_out, m->L_off).bytes;
  return direct_bytes(m->dtype, m->d, m->L_off[m->n_out]);
}

size_t sub_bytes(const pi_problem *p) {
  const int Ms = p->M > 0 ? p->M : 1;
  return Ms > 1 ? align_up((size_t)p->K * Ms * p->T * (p->dtype == PI_F64 ? 8 : 4), 256) : 0;
}

// Workspace of a rollout: the folded model (none when the caller passes one in
// pi_lwpr.folded), then the sub-rollout costs (M > 1), then the exchange slots
// of a pair-capable plan.
size_t rollout_fold_region(const pi_lwpr *m, const RolloutPlan &pl) { return m->folded ? 0 : fold_bytes(m, pl.mfma); }

size_t rollout_ws(const pi_problem *p, const pi_lwpr *m) {
  const RolloutPlan pl = rollout_plan(p, m);
  size_t b = rollout_fold_region(m, pl) + sub_bytes(p);
  if (pl.pair_ok) b += pair_ws_bytes(pl.groups);
  return b;
}

pi_status check_ws(void *ws, size_t ws_bytes, size_t need) {
  if (need > 0 && (!ws || ws_bytes < need))
    return fail(PI_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given%s", need, ws_bytes,
                ws ? "" : " (NULL)");
  return PI_OK;
}

// ---- allocation-free rollouts ---------------------------------------------------
// The address of `scratch` on the current device (see its definition),
// looked up once per device and cached.
pi_status noalloc_scratch(void **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(PI_ERR_DEVICE, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return fail(PI_ERR_DEVICE, "device id out of range");
  static std::mutex mu;
  static void *addr[kMaxDevices] = {nullptr};
  std::lock_guard<std::mutex> lk(mu);
  if (addr[dev] == nullptr) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      return fail(PI_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    addr[dev] = ptr;
  }
  *out = addr[dev];
  return PI_OK;
}

// ---- batched problems ------------------------------------------------------------
// Workspace of a batched call (pi_rollout_cost_batched, pi_control_step_batched):
//   [problem descriptors B][work items][queue word]
//   [per problem: matrix-core fold (unless pre-folded), sub-rollout costs (M > 1)]
//   [update scratch, shared in stream order: the largest of the problems']
//   [RH-shift scratch, shared: the largest direct fold (unless pre-folded) + partials]
// The descriptors and items are written by kernels on the stream, so a call
// never copies host memory and may be captured into a HIP graph.
struct BatchLayout {
  int max_spw, waves, n_items, pf;
  bool bf;
  size_t probs_off, items_off, queue_off, upd_off, shift_off, bytes;
  std::vector<size_t> fold_off, sub_off;   // (size_t)-1: none
  std::vector<int> spw;
  std::vector<int64_t> n_tiles, item_off;
};

int batch_spw(const pi_problem &p) {
  return p.tile_samples > 0 ? p.tile_samples : p.variant == PI_VARIANT_MFMA_F16X2 ? 128 : 16;
}

pi_status batch_layout(int32_t B, const pi_problem *p, const pi_lwpr *m, BatchLayout *out) {
  if (B < 1 || B > (1 << 20)) return fail(PI_ERR_SHAPE, "B=%d outside [1, 2^20]", B);
  if (!p || !m) return fail(PI_ERR_NULL, "problem and model arrays must be non-NULL");
  for (int b = 0; b < B; ++b) {
    pi_status st = check_pair(&p[b], &m[b]);
    if (st != PI_OK) return fail_problem(st, b);
    if (p[b].dtype != PI_F32 || p[b].dyn != PI_DYN_QUAD12)
      return fail(PI_ERR_UNSUPPORTED, "problem %d: batched rollouts need float32 quadrotor problems", b);
    if (!mfma_model_ok(&m[b]))
      return fail(PI_ERR_UNSUPPORTED, "problem %d: the model's matrix-core tiles must stay under 2 GiB", b);
    st = check_folded(&m[b], true);
    if (st != PI_OK) return fail_problem(st, b);
  }
  BatchLayout L;
  L.waves = p[0].tile_waves > 0 ? p[0].tile_waves : 4;
  L.max_spw = 0;
  L.spw.resize(B);
  L.n_tiles.resize(B);
  for (int b = 0; b < B; ++b) {
    L.spw[b] = batch_spw(p[b]);
    L.max_spw = std::max(L.max_spw, L.spw[b]);
    L.n_tiles[b] = ((int64_t)p[b].K * (p[b].M > 0 ? p[b].M : 1) + L.spw[b] - 1) / L.spw[b];
  }
  L.pf = variant_pf(p[0].variant);
  L.bf = L.pf != kPfF32;
  // tiles of 33..128 samples: the pieces forms' shared-tile launch
  if (L.max_spw > (L.bf ? 128 : 32))
    return fail(PI_ERR_UNSUPPORTED, "batched launches take tile_samples <= 32 (<= 128 with the pieces forms)");
  if (L.waves == 8 && L.max_spw > 16 && L.max_spw <= 32)
    return fail(PI_ERR_UNSUPPORTED, "tile_waves 8 needs tile_samples <= 16 (or > 32 with the pieces forms)");
  if (L.bf) {
    for (int b = 0; b < B; ++b)
      if (!bf_model_ok(&m[b])) return fail(PI_ERR_UNSUPPORTED, "problem %d: no pieces form of its model", b);
  }
  // work list: problems by decreasing per-tile work (T * model tiles), each
  // problem's tiles in order
  std::vector<int> order(B);
  for (int b = 0; b < B; ++b) order[b] = b;
  auto work = [&](int b) {
    return (int64_t)p[b].T * mfma_layout(m[b].d, m[b].n_out, m[b].L_off).n_tiles * L.spw[b];
  };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
  L.item_off.resize(B);
  int64_t n = 0;
  for (int b : order) {
    L.item_off[b] = n;
    n += L.n_tiles[b];
  }
  if (n > INT32_MAX) return fail(PI_ERR_SHAPE, "too many work items");
  L.n_items = (int)n;
  size_t off = 0;
  L.probs_off = off;
  off += align_up((size_t)B * sizeof(BatchedProblem), 256);
  L.items_off = off;
  off += align_up((size_t)n * sizeof(BatchedItem), 256);
  L.queue_off = off;
  off += 256;
  L.fold_off.assign(B, (size_t)-1);
  L.sub_off.assign(B, (size_t)-1);
  size_t upd = 0, shift = 0;
  for (int b = 0; b < B; ++b) {
    if (!m[b].folded) {
      L.fold_off[b] = off;
      off += align_up(mfma_layout(m[b].d, m[b].n_out, m[b].L_off).bytes, 256);
    }
    const size_t sb = sub_bytes(&p[b]);
    if (sb) {
      L.sub_off[b] = off;
      off += sb;
    }
    upd = std::max(upd, update_ws_bytes(p[b].K, p[b].T));
    shift = std::max(shift, (m[b].folded ? 0 : align_up(fold_bytes(&m[b], false), 256)) +
                                shift_partial_bytes(model_args(&m[b]), PI_F32));
  }
  L.upd_off = off;
  off += align_up(upd, 256);
  L.shift_off = off;
  off += align_up(shift, 256);
  L.bytes = off;
  *out = std::move(L);
  return PI_OK;
}

// The device-side plan (descriptors and work items) and the persistent
// rollout launch of a validated batch, then each problem's sub-rollout means.
hipError_t run_batched_rollouts(int32_t B, const pi_problem *p, const pi_lwpr *m, const void *const *x0,
                                const void *const *u_nom, const uint32_t *const *iter, void *const *cost,
                                const BatchLayout &L, char *ws, hipStream_t s) {
  BatchedProblem *probs = (BatchedProblem *)(ws + L.probs_off);
  BatchedItem *items = (BatchedItem *)(ws + L.items_off);
  hipError_t e = hipSuccess;
  for (int b = 0; b < B && e == hipSuccess; ++b) {
    const MfmaLayout l = mfma_layout(m[b].d, m[b].n_out, m[b].L_off);
    const void *base;
    if (m[b].folded) {
      base = (const char *)m[b].folded + folded_layout(&m[b]).mfma_off;
    } else {
      base = ws + L.fold_off[b];
      e = launch_fold_mfma(PI_F32, model_args(&m[b]), l, ws + L.fold_off[b], s);
      if (e != hipSuccess) break;
    }
    BatchedProblem bp;
    bp.p = prob_dev<float>(&p[b]);
    bp.x0 = (const float *)x0[b];
    bp.u_nom = (const float *)u_nom[b];
    bp.iter = iter[b];
    bp.cost = L.sub_off[b] != (size_t)-1 ? (float *)(ws + L.sub_off[b]) : (float *)cost[b];
    bp.md = mfma_model_view(l, base);
    e = launch_batched_describe(bp, probs, items, b, L.item_off[b], L.n_tiles[b], L.spw[b], s);
  }
  int *queue = (int *)(ws + L.queue_off);
  if (e == hipSuccess) e = launch_zero_int(queue, s);
  if (e == hipSuccess) {
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const int per_cu = L.waves == 8 || L.max_spw > 32 ? 1 : 2;
    const int grid = std::max(1, std::min(L.n_items, ncu * per_cu));
    e = launch_rollout_batched(probs, items, L.n_items, L.max_spw, L.waves, L.pf, grid, queue, s);
  }
  for (int b = 0; b < B && e == hipSuccess; ++b)
    if (L.sub_off[b] != (size_t)-1)
      e = launch_subcost_reduce(PI_F32, ws + L.sub_off[b], cost[b], p[b].K, p[b].M, p[b].T, s);
  return e;
}

pi_status check_batched_args(int32_t B, const void *const *x0, const void *const *u_nom,
                             const uint32_t *const *iter, void *const *cost) {
  if (!x0 || !u_nom || !iter || !cost) return fail(PI_ERR_NULL, "x0, u_nom, iter and cost arrays must be non-NULL");
  for (int b = 0; b < B; ++b)
    if (!x0[b] || !u_nom[b] || !iter[b] || !cost[b]) return fail(PI_ERR_NULL, "problem %d: NULL pointer", b);
  return PI_OK;
}

// Validation of a rollout request (everything but the workspace).
pi_status check_rollout(const pi_problem *p, const pi_lwpr *m, const void *x0, const void *u_nom,
                        const uint32_t *iter, const void *cost) {
  PI_TRY(check_pair(p, m));
  if (!x0 || !u_nom || !iter || !cost) return fail(PI_ERR_NULL, "x0, u_nom, iter and cost must be non-NULL");
  const RolloutPlan pl = rollout_plan(p, m);
  if (pl.mfma && (p->dtype != PI_F32 || !mfma_model_ok(m)))
    return fail(PI_ERR_UNSUPPORTED, "MFMA rollout needs float32, d in {4,6,16} and folded tiles under 2 GiB");
  PI_TRY(check_pieces(p, m, pl));
  return check_folded(m, pl.mfma);
}

// The launches of a validated rollout, with its workspace at `ws` (laid out
// as rollout_ws describes).
hipError_t run_rollout(const pi_problem *p, const pi_lwpr *m, const void *x0, const void *u_nom,
                       const uint32_t *iter, void *cost, void *ws, hipStream_t s) {
  const RolloutPlan pl = rollout_plan(p, m);
  const ModelArgs a = model_args(m);
  const int Ms = p->M > 0 ? p->M : 1;
  const size_t fb = rollout_fold_region(m, pl);
  void *sub = Ms > 1 ? (void *)((char *)ws + fb) : cost;
  const void *base = nullptr;
  hipError_t e = folded_base(m, pl.mfma, ws, s, &base);
  if (e == hipSuccess) {
    if (p->dtype == PI_F64) {
      RolloutArgs<double> ra{prob_dev<double>(p), (const double *)x0, (const double *)u_nom, iter, (double *)sub};
      e = launch_rollout_direct(PI_F64, &ra, a, base, s);
    } else {
      RolloutArgs<float> ra{prob_dev<float>(p), (const float *)x0, (const float *)u_nom, iter, (float *)sub};
      if (pl.mfma) {
        const MfmaLayout l = mfma_layout(m->d, m->n_out, m->L_off);
        const RolloutLaunch rl = rollout_launch(p, m);
        if (rl.pair)
          e = launch_rollout_pair(ra, l, base, rl.pl.spw, rl.pl.waves, rl.pl.pf, (char *)ws + fb + sub_bytes(p), s);
        else
          e = launch_rollout_mfma(ra, a, l, base, rl.pl.spw, rl.pl.waves, rl.pl.pf, s);
      } else {
        e = launch_rollout_direct(PI_F32, &ra, a, base, s);
      }
    }
  }
  if (e == hipSuccess && Ms > 1) e = launch_subcost_reduce(p->dtype, sub, cost, p->K, Ms, p->T, s);
  return e;
}

}  // namespace

extern "C" {

const char *pi_last_error(void) { return g_err; }

const char *pi_version(void) { return "pi2rh 0.1 (gfx950)"; }

size_t pi_model_fold_bytes(const pi_lwpr *m) {
  if (check_model(m) != PI_OK) return (size_t)-1;
  return folded_layout(m).bytes;
}

pi_status pi_model_fold(const pi_lwpr *m, void *folded, size_t folded_bytes, void *stream) {
  PI_TRY(check_model(m));
  const FoldedLayout f = folded_layout(m);
  if (!folded) return fail(PI_ERR_NULL, "folded must be non-NULL");
  if (folded_bytes < f.bytes) return fail(PI_ERR_WORKSPACE, "folded model of %zu bytes needed, %zu given", f.bytes,
                                          folded_bytes);
  PI_TRY(check_device());
  hipStream_t s = (hipStream_t)stream;
  const ModelArgs a = model_args(m);
  hipError_t e = launch_fold_direct(m->dtype, a, (char *)folded + f.direct_off, s);
  if (e == hipSuccess && f.has_mfma)
    e = launch_fold_mfma(m->dtype, a, mfma_layout(m->d, m->n_out, m->L_off), (char *)folded + f.mfma_off, s);
  return launched(e, "pi_model_fold");
}

pi_status pi_rollout_describe(const pi_problem *p, const pi_lwpr *m, int32_t *out) {
  PI_TRY(check_pair(p, m));
  if (!out) return fail(PI_ERR_NULL, "out must be non-NULL");
  {
    const RolloutPlan pl = rollout_plan(p, m);
    if (pl.mfma && (p->dtype != PI_F32 || !mfma_model_ok(m)))
      return fail(PI_ERR_UNSUPPORTED, "MFMA rollout needs float32, d in {4,6,16} and folded tiles under 2 GiB");
    PI_TRY(check_pieces(p, m, pl));
  }
  PI_TRY(check_device());
  const RolloutLaunch rl = rollout_launch(p, m);
  const RolloutPlan &pl = rl.pl;
  out[0] = pl.pf == kPfF16x2    ? PI_VARIANT_MFMA_F16X2
           : pl.pf == kPfBf16x3 ? PI_VARIANT_MFMA_BF16X3
           : pl.mfma            ? PI_VARIANT_MFMA
                                : PI_VARIANT_DIRECT;
  out[1] = pl.mfma ? pl.spw : 1;
  out[2] = pl.mfma ? pl.waves : 1;
  out[3] = rl.pair ? 2 : 1;
  return ok();
}

size_t pi_workspace_bytes(int32_t op, const pi_problem *p, const pi_lwpr *m) {
  switch (op) {
    case PI_OP_PREDICT:
      if (check_model(m) != PI_OK) return (size_t)-1;
      return mfma_model_ok(m) ? std::max(fold_bytes(m, true), fold_bytes(m, false))
                                     : fold_bytes(m, false);
    case PI_OP_ROLLOUT:
      if (check_pair(p, m) != PI_OK) return (size_t)-1;
      return rollout_ws(p, m);
    case PI_OP_UPDATE:
      if (check_problem(p) != PI_OK) return (size_t)-1;
      return update_ws_bytes(p->K, p->T);
    case PI_OP_RH_SHIFT:
      if (check_pair(p, m) != PI_OK) return (size_t)-1;
      return fold_bytes(m, false) + shift_partial_bytes(model_args(m), m->dtype);
    case PI_OP_ADJOINT:
      if (check_pair(p, m) != PI_OK) return (size_t)-1;
      return adjoint_ws_bytes(p->dtype, p->dyn, p->K, p->M, p->T, m->L_off[m->n_out], m->d,
                              adjoint_default_ckpt(p->T), adjoint_mfma_bytes(p, m));
  }
  fail(PI_ERR_VALUE, "unknown op %d", op);
  return (size_t)-1;
}

pi_status lwpr_predict(const pi_lwpr *m, const void *Z, int64_t N, void *mean, void *var,
                       int32_t variant, void *ws, size_t ws_bytes, void *stream) {
  PI_TRY(check_model(m));
  if (N < 0) return fail(PI_ERR_SHAPE, "N=%lld must be >= 0", (long long)N);
  if (N > 0 && (!Z || !mean || !var)) return fail(PI_ERR_NULL, "Z, mean and var must be non-NULL");
  if (variant == PI_VARIANT_MFMA_BF16X3 || variant == PI_VARIANT_MFMA_F16X2)
    return fail(PI_ERR_UNSUPPORTED, "prediction has no pieces form (use PI_VARIANT_MFMA)");
  if (variant < PI_VARIANT_AUTO || variant > PI_VARIANT_MFMA) return fail(PI_ERR_VALUE, "unknown variant %d", variant);
  const bool use_mfma = variant == PI_VARIANT_MFMA || (variant == PI_VARIANT_AUTO && mfma_model_ok(m));
  if (use_mfma && !mfma_model_ok(m))
    return fail(PI_ERR_UNSUPPORTED, "MFMA prediction needs float32, d in {4,6,16} and folded tiles under 2 GiB");
  PI_TRY(check_folded(m, use_mfma));
  if (!m->folded) PI_TRY(check_ws(ws, ws_bytes, fold_bytes(m, use_mfma)));
  PI_TRY(check_device());
  if (N == 0) return ok();
  hipStream_t s = (hipStream_t)stream;
  const ModelArgs a = model_args(m);
  const void *base = nullptr;
  hipError_t e = folded_base(m, use_mfma, ws, s, &base);
  if (e == hipSuccess) {
    if (use_mfma)
      e = launch_predict_mfma(a, mfma_layout(m->d, m->n_out, m->L_off), base, Z, N, mean, var, s);
    else
      e = launch_predict_direct(m->dtype, a, base, Z, N, mean, var, s);
  }
  return launched(e, "lwpr_predict");
}

pi_status pi_rollout_cost(const pi_problem *p, const pi_lwpr *m, const void *x0, const void *u_nom,
                          const uint32_t *iter, void *cost, void *ws, size_t ws_bytes, void *stream) {
  PI_TRY(check_rollout(p, m, x0, u_nom, iter, cost));
  PI_TRY(check_ws(ws, ws_bytes, rollout_ws(p, m)));
  PI_TRY(check_device());
  return launched(run_rollout(p, m, x0, u_nom, iter, cost, ws, (hipStream_t)stream), "pi_rollout_cost");
}

pi_status pi_rollout_cost_noalloc(const pi_problem *p, const pi_lwpr *m, const void *x0, const void *u_nom,
                                  const uint32_t *iter, void *cost, void *stream) {
  PI_TRY(check_rollout(p, m, x0, u_nom, iter, cost));
  const size_t need = rollout_ws(p, m);
  const size_t cap = (size_t)PI_NOALLOC_SCRATCH_BYTES;
  if (need > cap)
    return fail(PI_ERR_WORKSPACE,
                "this rollout needs %zu bytes of scratch; the allocation-free entry point holds %zu "
                "(pass a folded model, fewer sub-rollouts, or use pi_rollout_cost with a workspace)",
                need, cap);
  PI_TRY(check_device());
  void *ptr = nullptr;
  PI_TRY(noalloc_scratch(&ptr));
  return launched(run_rollout(p, m, x0, u_nom, iter, cost, ptr, (hipStream_t)stream), "pi_rollout_cost_noalloc");
}

pi_status pi_update(const pi_problem *p, const void *cost, const uint32_t *iter, void *u_nom,
                    void *weights, void *ws, size_t ws_bytes, void *stream) {
  PI_TRY(check_problem(p));
  if (!cost || !iter || !u_nom) return fail(PI_ERR_NULL, "cost, iter and u_nom must be non-NULL");
  PI_TRY(check_ws(ws, ws_bytes, update_ws_bytes(p->K, p->T)));
  PI_TRY(check_device());
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (p->dtype == PI_F64) {
    const ProbDev<double> d = prob_dev<double>(p);
    e = launch_update(PI_F64, &d, cost, iter, u_nom, (double *)weights, ws, 1, p->lambda, p->weighting, s);
  } else {
    const ProbDev<float> d = prob_dev<float>(p);
    e = launch_update(PI_F32, &d, cost, iter, u_nom, (double *)weights, ws, 1, p->lambda, p->weighting, s);
  }
  return launched(e, "pi_update");
}

pi_status pi_rh_shift(const pi_problem *p, const pi_lwpr *m, void *x0, void *u_nom,
                      const uint32_t *iter, void *ws, size_t ws_bytes, void *stream) {
  PI_TRY(check_pair(p, m));
  if (!x0 || !u_nom || !iter) return fail(PI_ERR_NULL, "x0, u_nom and iter must be non-NULL");
  const ModelArgs a = model_args(m);
  const size_t fb = fold_bytes(m, false);
  PI_TRY(check_folded(m, false));
  PI_TRY(check_ws(ws, ws_bytes, fb + shift_partial_bytes(a, m->dtype)));
  PI_TRY(check_device());
  hipStream_t s = (hipStream_t)stream;
  void *part = (char *)ws + fb;
  const void *base = nullptr;
  hipError_t e = folded_base(m, false, ws, s, &base);
  if (e == hipSuccess) {
    if (p->dtype == PI_F64) {
      const ProbDev<double> d = prob_dev<double>(p);
      e = launch_rh_shift(PI_F64, &d, a, base, part, x0, u_nom, iter, s);
    } else {
      const ProbDev<float> d = prob_dev<float>(p);
      e = launch_rh_shift(PI_F32, &d, a, base, part, x0, u_nom, iter, s);
    }
  }
  return launched(e, "pi_rh_shift");
}

size_t pi_adjoint_workspace_bytes(const pi_problem *p, const pi_lwpr *m, int32_t ckpt_every) {
  int ckpt = 0;
  if (check_adjoint(p, m, ckpt_every, &ckpt) != PI_OK) return (size_t)-1;
  return adjoint_ws(p, m, ckpt);
}

pi_status pi_rollout_adjoint(const pi_problem *p, const pi_lwpr *m, const void *x0, const void *u_nom,
                             const uint32_t *iter, int32_t ckpt_every, const void *gJ, void *J, void *g_u_nom,
                             void *g_centre, void *g_metric, void *ws, size_t ws_bytes, void *stream) {
  int ckpt = 0;
  PI_TRY(check_adjoint(p, m, ckpt_every, &ckpt));
  if (!x0 || !u_nom || !iter || !J || !g_u_nom || !g_centre || !g_metric)
    return fail(PI_ERR_NULL, "x0, u_nom, iter, J and the gradient outputs must be non-NULL");
  PI_TRY(check_ws(ws, ws_bytes, adjoint_ws(p, m, ckpt)));
  PI_TRY(check_device());
  hipStream_t s = (hipStream_t)stream;
  const ModelArgs a = model_args(m);
  hipError_t e;
  if (p->dtype == PI_F64) {
    const ProbDev<double> d = prob_dev<double>(p);
    e = launch_adjoint(PI_F64, &d, a, x0, u_nom, iter, ckpt, (const double *)gJ, (double *)J, g_u_nom, g_centre,
                       g_metric, ws, nullptr, kPfF32, s);
  } else {
    const ProbDev<float> d = prob_dev<float>(p);
    const MfmaLayout l = mfma_layout(m->d, m->n_out, m->L_off);
    const bool mf = adjoint_mfma_bytes(p, m) != 0;
    e = launch_adjoint(PI_F32, &d, a, x0, u_nom, iter, ckpt, (const double *)gJ, (double *)J, g_u_nom, g_centre,
                       g_metric, ws, mf ? &l : nullptr, mf ? variant_pf(p->variant) : kPfF32, s);
  }
  return launched(e, "pi_rollout_adjoint");
}

pi_status pi_pair_give_ups(uint64_t *count, void *stream) {
  if (!count) return fail(PI_ERR_NULL, "count must be non-NULL");
  PI_TRY(check_device());
  return launched(launch_read_give_ups(count, (hipStream_t)stream), "pi_pair_give_ups");
}

pi_status pi_philox4x32_10(const uint32_t *ctr, uint64_t key, uint32_t *out, int64_t N,
                           void *stream) {
  if (N < 0) return fail(PI_ERR_SHAPE, "N must be >= 0");
  if (N > 0 && (!ctr || !out)) return fail(PI_ERR_NULL, "ctr and out must be non-NULL");
  PI_TRY(check_device());
  return launched(launch_philox(ctr, (uint32_t)key, (uint32_t)(key >> 32), out, N, (hipStream_t)stream),
                  "pi_philox4x32_10");
}

pi_status pi_noise(const pi_problem *p, int32_t tag, const uint32_t *iter, int32_t k0, int32_t nk,
                   int32_t m, void *out, void *stream) {
  PI_TRY(check_problem(p));
  if (tag != PI_TAG_CTRL && tag != PI_TAG_DYN && tag != PI_TAG_PLANT) return fail(PI_ERR_VALUE, "unknown tag %d", tag);
  if (!iter || !out) return fail(PI_ERR_NULL, "iter and out must be non-NULL");
  if (tag != PI_TAG_PLANT && (k0 < 0 || nk < 0 || m < 0 || (int64_t)k0 + nk > (int64_t)UINT32_MAX))
    return fail(PI_ERR_SHAPE, "bad rollout range");
  PI_TRY(check_device());
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (p->dtype == PI_F64) {
    const ProbDev<double> d = prob_dev<double>(p);
    e = launch_noise(PI_F64, &d, tag, iter, k0, nk, m, out, s);
  } else {
    const ProbDev<float> d = prob_dev<float>(p);
    e = launch_noise(PI_F32, &d, tag, iter, k0, nk, m, out, s);
  }
  return launched(e, "pi_noise");
}

size_t pi_batched_workspace_bytes(int32_t B, const pi_problem *p, const pi_lwpr *m) {
  BatchLayout L;
  if (batch_layout(B, p, m, &L) != PI_OK) return (size_t)-1;
  return L.bytes;
}

pi_status pi_rollout_cost_batched(int32_t B, const pi_problem *p, const pi_lwpr *m, const void *const *x0,
                                  const void *const *u_nom, const uint32_t *const *iter, void *const *cost,
                                  void *ws, size_t ws_bytes, void *stream) {
  BatchLayout L;
  PI_TRY(batch_layout(B, p, m, &L));
  PI_TRY(check_batched_args(B, x0, u_nom, iter, cost));
  PI_TRY(check_ws(ws, ws_bytes, L.bytes));
  PI_TRY(check_device());
  return launched(run_batched_rollouts(B, p, m, x0, u_nom, iter, cost, L, (char *)ws, (hipStream_t)stream),
                  "pi_rollout_cost_batched");
}

pi_status pi_control_step_batched(int32_t B, const pi_problem *p, const pi_lwpr *m, void *const *x0,
                                  void *const *u_nom, uint32_t *const *iter, void *const *cost, void *ws,
                                  size_t ws_bytes, void *stream) {
  BatchLayout L;
  PI_TRY(batch_layout(B, p, m, &L));
  PI_TRY(check_batched_args(B, (const void *const *)x0, (const void *const *)u_nom,
                            (const uint32_t *const *)iter, cost));
  PI_TRY(check_ws(ws, ws_bytes, L.bytes));
  PI_TRY(check_device());
  hipStream_t s = (hipStream_t)stream;
  char *w = (char *)ws;
  hipError_t e = run_batched_rollouts(B, p, m, (const void *const *)x0, (const void *const *)u_nom,
                                      (const uint32_t *const *)iter, cost, L, w, s);
  // each problem's update (Eq. 2) and receding-horizon advance, in problem
  // order, sharing one update and one shift scratch area
  for (int b = 0; b < B && e == hipSuccess; ++b) {
    const ProbDev<float> d = prob_dev<float>(&p[b]);
    e = launch_update(PI_F32, &d, cost[b], iter[b], u_nom[b], nullptr, w + L.upd_off, 1, p[b].lambda,
                      p[b].weighting, s);
    if (e != hipSuccess) break;
    const ModelArgs a = model_args(&m[b]);
    const void *base;
    char *part = w + L.shift_off;
    if (m[b].folded) {
      base = (const char *)m[b].folded + folded_layout(&m[b]).direct_off;
    } else {
      base = w + L.shift_off;
      part += align_up(fold_bytes(&m[b], false), 256);
      e = launch_fold_direct(PI_F32, a, w + L.shift_off, s);
      if (e != hipSuccess) break;
    }
    e = launch_rh_shift(PI_F32, &d, a, base, part, x0[b], u_nom[b], iter[b], s);
  }
  return launched(e, "pi_control_step_batched");
}

}  // extern "C"
