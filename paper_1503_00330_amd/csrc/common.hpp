// Device-side building blocks shared by the gfx950 kernels: problem parameters
// passed by value, the counter-based random stream, explicit Euler dynamics and
// the state cost.  (PI^2-RH with LWPR dynamics, arXiv:1503.00330.)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pi2rh {

constexpr int kMaxOut = 8;
constexpr int kMaxU = 4;
constexpr int kMaxD = 16;
constexpr int kMaxX = 12;
constexpr int kMaxObs = 64;
constexpr int kMaxR = 16;

enum { kDynPointMass2D = 0, kDynQuad12 = 1, kDynQuadHybrid = 2 };
// First-order response of the attitude rates to their commands (Sec. 4.1):
// d(angles)/dt = kRateGain (commanded - actual).
constexpr double kRateGain = 25.0;
enum { kObsIndicator = 0, kObsSmooth = 1 };
enum { kTagCtrl = 0u, kTagDyn = 1u, kTagPlant = 2u };

// Everything a rollout kernel needs about one problem, by value (< 1 KB).
template <typename Real>
struct ProbDev {
  int dyn, K, T, M, Ms;        // Ms = max(M, 1) sub-rollouts per rollout
  int n_x, n_u, n_out, d;
  Real dt;
  Real noise_std[kMaxU];
  Real goal[3], w_pos[3], w_ang, w_vel;
  int obs_kind, n_obs;
  const Real *obs;             // dev [n_obs][3]
  Real obs_penalty, obs_decay;
  uint32_t key0, key1, problem_id;
  int ctrl_cost;               // 1: add the control terms of the cost-to-go (hybrid model)
  Real ctrl_w[3];              // lambda / sigma_a^2 of the commanded-rate channels
};

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with the published multipliers, the high halves mixed
// into the odd words with the round key, key bumped by the Weyl constants.
struct Philox4 {
  uint32_t v[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
    const uint32_t p0lo = m0 * c0, p0hi = __umulhi(m0, c0);
    const uint32_t p1lo = m1 * c2, p1hi = __umulhi(m1, c2);
    const uint32_t n0 = p1hi ^ c1 ^ k0;
    const uint32_t n2 = p0hi ^ c3 ^ k1;
    c0 = n0;
    c1 = p1lo;
    c2 = n2;
    c3 = p0lo;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  Philox4 out;
  out.v[0] = c0;
  out.v[1] = c1;
  out.v[2] = c2;
  out.v[3] = c3;
  return out;
}

__device__ __forceinline__ uint32_t stream_word(uint32_t tag, uint32_t problem, uint32_t iter) {
  return (tag << 30) | ((problem & 0x3FFu) << 20) | (iter & 0xFFFFFu);
}

// Uniform in (0,1) from the top 23 bits: exact in float and double.
template <typename Real>
__device__ __forceinline__ Real unit_open(uint32_t r) {
  return ((Real)(r >> 9) + (Real)0.5) * (Real)(1.0 / 8388608.0);
}

__device__ __forceinline__ void sincos_2pi(float u, float *s, float *c) { sincospif(2.0f * u, s, c); }
__device__ __forceinline__ void sincos_2pi(double u, double *s, double *c) { sincospi(2.0 * u, s, c); }
__device__ __forceinline__ float log_(float x) { return logf(x); }
__device__ __forceinline__ double log_(double x) { return log(x); }
__device__ __forceinline__ float sqrt_(float x) { return sqrtf(x); }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float exp_(float x) { return expf(x); }
__device__ __forceinline__ double exp_(double x) { return exp(x); }

// n (<= 8) standard normals of draw (tag, k, m, t); normal i is lane i%4 of
// counter block i/4; Box-Muller on the uniform pairs (0,1) and (2,3).
template <typename Real, int N>
__device__ __forceinline__ void normals(uint32_t key0, uint32_t key1, uint32_t word3, uint32_t k,
                                        uint32_t m, uint32_t t, Real *out) {
#pragma unroll
  for (int blk = 0; blk * 4 < N; ++blk) {
    Philox4 r = philox4x32_10(t, k, (m << 4) | (uint32_t)blk, word3, key0, key1);
    Real s0, c0, s1, c1;
    const Real rad0 = sqrt_((Real)-2 * log_(unit_open<Real>(r.v[0])));
    const Real rad1 = sqrt_((Real)-2 * log_(unit_open<Real>(r.v[2])));
    sincos_2pi(unit_open<Real>(r.v[1]), &s0, &c0);
    sincos_2pi(unit_open<Real>(r.v[3]), &s1, &c1);
    const Real v[4] = {rad0 * c0, rad0 * s0, rad1 * c1, rad1 * s1};
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (blk * 4 + i < N) out[blk * 4 + i] = v[i];
  }
}

// Runtime-count wrapper (n <= 8).
template <typename Real>
__device__ __forceinline__ void normals_n(int n, uint32_t key0, uint32_t key1, uint32_t word3,
                                          uint32_t k, uint32_t m, uint32_t t, Real *out) {
  if (n <= 4)
    normals<Real, 4>(key0, key1, word3, k, m, t, out);
  else
    normals<Real, 8>(key0, key1, word3, k, m, t, out);
}

// ---------------------------------------------------------------- dynamics
// The LWPR input of a state and an applied control: z = [x ; u] for the point
// mass and the 12-state quadrotor; for the hybrid quadrotor (Sec. 4.1: the
// learned models take the three euler angles and the total thrust) z =
// [phi, theta, psi, F] = [x_6, x_7, x_8, u_3].
template <int DYN, typename Real>
__device__ __forceinline__ void lwpr_input(const Real *x, const Real *u, Real *z) {
  if constexpr (DYN == kDynQuadHybrid) {
    z[0] = x[6];
    z[1] = x[7];
    z[2] = x[8];
    z[3] = u[3];
  } else {
    constexpr int NX = DYN == kDynPointMass2D ? 4 : 12, NU = DYN == kDynPointMass2D ? 2 : 4;
#pragma unroll
    for (int a = 0; a < NX; ++a) z[a] = x[a];
#pragma unroll
    for (int a = 0; a < NU; ++a) z[NX + a] = u[a];
  }
}

// Explicit Euler: positions integrate velocities, velocities the linear
// accelerations; for the 12-state quadrotor euler angles integrate the body
// rates and rates integrate the angular accelerations; for the hybrid
// quadrotor the angles follow their commanded rates u_0..2 through the
// first-order response (Sec. 4.1) and the learned models give the linear
// accelerations.  Right-hand sides use x_t and the applied control u.
template <typename Real>
__device__ __forceinline__ void euler_step(int dyn, Real dt, const Real *x, const Real *acc, const Real *u,
                                           Real *xn) {
  if (dyn == kDynPointMass2D) {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      xn[a] = x[a] + dt * x[2 + a];
      xn[2 + a] = x[2 + a] + dt * acc[a];
    }
  } else if (dyn == kDynQuadHybrid) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      xn[a] = x[a] + dt * x[3 + a];
      xn[3 + a] = x[3 + a] + dt * acc[a];
      xn[6 + a] = x[6 + a] + dt * ((Real)kRateGain * (u[a] - x[6 + a]));
    }
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      xn[a] = x[a] + dt * x[3 + a];
      xn[3 + a] = x[3 + a] + dt * acc[a];
      xn[6 + a] = x[6 + a] + dt * x[9 + a];
      xn[9 + a] = x[9 + a] + dt * acc[3 + a];
    }
  }
}

// State cost q(x) (Sec. 5): weighted squared goal error, |euler|^2 and |v|^2
// penalties, plus the obstacle term over obstacles in `obs` (LDS or global).
template <typename Real>
__device__ __forceinline__ Real state_cost(const ProbDev<Real> &p, const Real *obs, const Real *x) {
  const int np = p.dyn == kDynPointMass2D ? 2 : 3;
  Real c = 0;
  for (int a = 0; a < np; ++a) {
    const Real e = x[a] - p.goal[a];
    c += p.w_pos[a] * e * e;
  }
  for (int a = 0; a < np; ++a) c += p.w_vel * x[np + a] * x[np + a];
  if (p.dyn != kDynPointMass2D)
    for (int a = 0; a < 3; ++a) c += p.w_ang * x[6 + a] * x[6 + a];
  if (p.obs_kind == kObsIndicator) {
    bool inside = false;
    for (int i = 0; i < p.n_obs; ++i) {
      const Real dx = x[0] - obs[3 * i], dy = x[1] - obs[3 * i + 1], r = obs[3 * i + 2];
      inside |= (dx * dx + dy * dy < r * r);
    }
    if (inside) c += p.obs_penalty;
  } else {
    for (int i = 0; i < p.n_obs; ++i) {
      const Real dx = x[0] - obs[3 * i], dy = x[1] - obs[3 * i + 1];
      c += p.obs_penalty * exp_(-p.obs_decay * (dx * dx + dy * dy));
    }
  }
  return c;
}

// Control terms of the cost-to-go S-tilde (Sec. 3.1, below Eq. 2) for one step
// of the hybrid model, whose commanded rates are its control-affine channel:
// G_c = kRateGain I and the noise enters through the same channel, B dw =
// G_c eps dt.  Then G_c^T H^-1 G_c = R with H = G_c R^-1 G_c^T, and
// B B^T = lambda G_c R^-1 G_c^T with eps ~ N(0, diag(sigma^2)) per step gives
// R = lambda diag(1/sigma^2) / dt, so
//   u^T G_c^T H^-1 G_c u dt + u^T G_c^T H^-1 B dw = sum_a lambda/sigma_a^2 u_a (u_a + eps_a)
// over the three commanded rates; u is the nominal control, eps its sampled
// perturbation.
template <typename Real>
__device__ __forceinline__ Real control_cost(const ProbDev<Real> &p, const Real *u_nom_t, const Real *pert) {
  Real c = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) c += p.ctrl_w[a] * u_nom_t[a] * (u_nom_t[a] + pert[a]);
  return c;
}

// d q / d x into g[n_x] (the indicator has zero derivative almost everywhere).
template <typename Real>
__device__ __forceinline__ void state_cost_grad(const ProbDev<Real> &p, const Real *obs,
                                                const Real *x, Real *g) {
  const int np = p.dyn == kDynPointMass2D ? 2 : 3;
  for (int a = 0; a < p.n_x; ++a) g[a] = 0;
  for (int a = 0; a < np; ++a) g[a] = 2 * p.w_pos[a] * (x[a] - p.goal[a]);
  for (int a = 0; a < np; ++a) g[np + a] = 2 * p.w_vel * x[np + a];
  if (p.dyn != kDynPointMass2D)
    for (int a = 0; a < 3; ++a) g[6 + a] = 2 * p.w_ang * x[6 + a];
  if (p.obs_kind == kObsSmooth) {
    for (int i = 0; i < p.n_obs; ++i) {
      const Real dx = x[0] - obs[3 * i], dy = x[1] - obs[3 * i + 1];
      const Real e = p.obs_penalty * exp_(-p.obs_decay * (dx * dx + dy * dy));
      g[0] -= 2 * p.obs_decay * dx * e;
      g[1] -= 2 * p.obs_decay * dy * e;
    }
  }
}

// ------------------------------------------------------- mixture statistics
// Running statistics of one softmax-weighted Gaussian mixture over a subset
// of its local models, in a shifted exponent domain:
//   m  = largest activation seen (natural log units for the direct form,
//        base-2 units for the MFMA form),
//   Z  = sum_j exp(a_j - m),     mu = sum_j e_j y_j / Z,
//   M2 = sum_j e_j (y_j - mu)^2, S2 = sum_j e_j sigma_j^2.
// Adding one model is a weighted Welford step; merging two sets is Chan's
// parallel update.  The variance is (M2 + S2) / Z: this avoids the
// cancellation of E[y^2] - mu^2 (law of total variance, Eq. 1).
template <typename Real>
struct MixStat {
  Real m, Z, mu, M2, S2;
};

template <typename Real>
__device__ __forceinline__ MixStat<Real> mix_empty() {
  MixStat<Real> s;
  s.m = (Real)-3.0e38;
  s.Z = 0;
  s.mu = 0;
  s.M2 = 0;
  s.S2 = 0;
  return s;
}

// exp(x) (Base2 = false) or 2^x (Base2 = true) in the working precision.
template <bool Base2>
__device__ __forceinline__ float expb(float x) { return Base2 ? exp2f(x) : expf(x); }
template <bool Base2>
__device__ __forceinline__ double expb(double x) { return Base2 ? exp2(x) : exp(x); }

template <bool Base2, typename Real>
__device__ __forceinline__ MixStat<Real> mix_merge(const MixStat<Real> &a, const MixStat<Real> &b) {
  MixStat<Real> r;
  r.m = a.m > b.m ? a.m : b.m;
  const Real sa = expb<Base2>(a.m - r.m), sb = expb<Base2>(b.m - r.m);
  const Real Za = a.Z * sa, Zb = b.Z * sb;
  r.Z = Za + Zb;
  const Real fb = r.Z > 0 ? Zb / r.Z : (Real)0;
  const Real dmu = b.mu - a.mu;
  r.mu = a.mu + dmu * fb;
  r.M2 = a.M2 * sa + b.M2 * sb + dmu * dmu * Za * fb;
  r.S2 = a.S2 * sa + b.S2 * sb;
  return r;
}

// e / Z for the running mean: exact division in double, the hardware
// reciprocal (1 ulp) in float.
__device__ __forceinline__ float ratio(float e, float Z) { return e * __builtin_amdgcn_rcpf(Z); }
__device__ __forceinline__ double ratio(double e, double Z) { return e / Z; }

// Adds one local model (activation act, prediction y, noise variance s2).
// One exponential per model: the larger of (m, act) becomes the new shift.
template <bool Base2, typename Real>
__device__ __forceinline__ void mix_add(MixStat<Real> &s, Real act, Real y, Real s2) {
  const bool up = act > s.m;
  const Real t = expb<Base2>(up ? s.m - act : act - s.m);
  const Real sc = up ? t : (Real)1, e = up ? (Real)1 : t;
  s.m = up ? act : s.m;
  const Real Zn = s.Z * sc + e;
  const Real dy = y - s.mu;
  const Real mun = s.mu + dy * ratio(e, Zn);
  s.M2 = s.M2 * sc + e * dy * (y - mun);
  s.S2 = s.S2 * sc + e * s2;
  s.Z = Zn;
  s.mu = mun;
}

// M2 (the spread of the local predictions) is non-negative in exact
// arithmetic; when a new leading model takes over, e/Z can round to just above
// one and leave a negative M2 of order eps * (y - mu)^2, which in float can
// exceed the noise term, so it is clamped at zero.
template <typename Real>
__device__ __forceinline__ void mix_finish(const MixStat<Real> &s, Real *mean, Real *var) {
  *mean = s.mu;
  *var = ((s.M2 > (Real)0 ? s.M2 : (Real)0) + s.S2) / s.Z;
}

}  // namespace pi2rh
