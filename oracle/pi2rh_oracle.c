/*
 * FP64 CPU oracle for PI^2-RH rollouts through a learned LWPR dynamics model.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP implementation: it is a plain, slow,
 * literal transcription of the method's definitions, written for a reader to
 * check against the paper by eye.
 *
 * Paper: Williams, Rombokas, Daniel, "GPU based Path Integral Control with
 * Learned Dynamics" (arXiv:1503.00330).
 *
 *   - LWPR mixture mean/variance ........ Sec. 2, Eq. (1); local models are PLS
 *                                           regressions (Sec. 2, first paragraph)
 *   - control-affine noise, u_L = eps ... Sec. 3.1 (dynamics form and u_L)
 *   - cost-to-go S(tau_i) ............... Sec. 3.1 (definition of S below Eq. 2)
 *   - path-integral update .............. Sec. 3.1, Eq. (2); iterative PI^2
 *   - receding horizon warm start ....... Sec. 3.1 (last paragraph)
 *   - sub-rollouts, averaged cost ....... Sec. 3.2
 *   - state cost, phi = 0 ............... Sec. 5 (q(x) and the terminal cost)
 *   - Euler integration ................. Table 1 caption
 *
 * Readings where the paper is silent or garbled:
 *   R1  Eq. (1) mixes indices; read as the normalised Gaussian mixture:
 *       w_j = softmax_j(-q_j/2), mu = sum w_j y_j,
 *       var = sum w_j ((mu - y_j)^2 + sigma_j^2).
 *   R2  local model: centred input delta = z - c_j, PLS deflation
 *       s_r = u_r . r_r, r_{r+1} = r_r - s_r p_r, y_j = beta_0 + sum_r beta_r s_r.
 *   R3  z = [x ; u], outputs are accelerations, explicit Euler on the state.
 *   R4  noise: eps_{k,t} = sigma_u * N(0, I) shared by the M sub-rollouts of
 *       rollout k; the next state uses a = mu + sqrt(var) * xi_{k,m,t}
 *       (a = mu when M = 0, "mean prediction only").
 *   R5  cost c_{k,m,t} = dt * q(x_{t+1}); cbar_{k,t} = mean over m; phi = 0 and
 *       the control-cost terms of S-tilde are dropped (Sec. 5).
 *   R6  update: S_{k,i} = sum_{t >= i} cbar_{k,t}; P = softmax_k(-S/lambda);
 *       u_i += sum_k P_{k,i} eps_{k,i}.  TRAJECTORY weighting uses S_{k,0}.
 *   R7  random stream: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 *       key = seed, counter = (t, k, (m << 4) | blk,
 *       tag << 30 | (problem & 0x3FF) << 20 | (iter & 0xFFFFF)),
 *       uniforms ((r >> 9) + 0.5) * 2^-23 (exact in single and double
 *       precision), Box-Muller pairs (u0,u1), (u2,u3).
 *   R8  adjoint: J = (1/(K max(M,1))) sum_{k,m,t} c_{k,m,t} with all noise
 *       held fixed; derivatives w.r.t. u_nom, c_j and every entry of D_j.
 *   R9  the paper's own quadrotor model (Sec. 4.1, "hybrid"): controls are
 *       commanded euler rates and the total thrust F; the angles follow the
 *       first-order response dr/dt = 25 (r_commanded - r); three LWPR models
 *       with inputs (phi, theta, psi, F) give the cartesian accelerations.
 *       State [p, v, r] (9), integrated by explicit Euler like the others.
 *   R10 the control terms of S-tilde (Sec. 3.1, below Eq. 2), which the
 *       experiments drop (Sec. 5), as an option: per step of rollout k
 *       u^T G_c^T H^-1 G_c u dt + u^T G_c^T H^-1 B dw with H = G_c R^-1 G_c^T,
 *       u the nominal control.  The control-affine channel is the hybrid
 *       model's commanded rates, G_c = 25 I on those three controls (R9); the
 *       noise enters through the same channel, B dw = G_c eps dt with eps the
 *       step's sampled perturbation; B B^T = lambda G_c R^-1 G_c^T (Sec. 3.1)
 *       with eps ~ N(0, diag(sigma^2)) per step fixes R = lambda
 *       diag(1/sigma^2) / dt.  The sum over steps runs from the step i on,
 *       like S, so the term is added to every step's cost (the paper's lower
 *       index of that sum is garbled).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_POINTMASS2D 0
#define ORC_QUAD12 1
#define ORC_QUAD_HYBRID 2
#define ORC_RATE_GAIN 25.0
#define ORC_OBS_INDICATOR 0
#define ORC_OBS_SMOOTH 1
#define ORC_W_COST_TO_GO 0
#define ORC_W_TRAJECTORY 1
#define ORC_TAG_CTRL 0u
#define ORC_TAG_DYN 1u
#define ORC_TAG_PLANT 2u

typedef struct {
  int32_t d, n_out, R;
  const int64_t *L_off;   /* [n_out+1] */
  const double *centre;   /* [Ltot][d] */
  const double *metric;   /* [Ltot][d][d] */
  const double *proj_u;   /* [Ltot][R][d] */
  const double *proj_p;   /* [Ltot][R][d] or NULL (p = u) */
  const double *beta;     /* [Ltot][R+1] */
  const double *sigma2;   /* [Ltot] */
} orc_model;

typedef struct {
  int32_t dyn, K, T, M;
  double dt, lam, noise_std[4];
  double goal[3], w_pos[3], w_ang, w_vel;
  int32_t obs_kind, n_obs;
  const double *obs;      /* [n_obs][3] = (cx, cy, r) */
  double obs_penalty, obs_decay;
  int32_t weighting;
  uint64_t seed;
  uint32_t problem_id;
  int32_t ctrl_cost;      /* 1: add the control terms of S-tilde (reading R10) */
} orc_problem;

/* ------------------------------------------------------------------ Philox */

/* Philox4x32 with 10 rounds: each round multiplies counter words 0 and 2 by
 * two fixed 32-bit constants, splits the 64-bit products into high and low
 * halves and mixes them with the other words and the round key; the key is
 * advanced by two Weyl increments between rounds. */
void orc_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* n standard normals of the draw (tag, k, m, t) under (seed, problem, iter). */
void orc_normals(uint64_t seed, uint32_t tag, uint32_t problem_id, uint32_t iter,
                 uint32_t k, uint32_t m, uint32_t t, int32_t n, double *out) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  const double two_pi = 6.283185307179586476925286766559;
  for (int32_t blk = 0; blk * 4 < n; ++blk) {
    uint32_t ctr[4], r[4];
    ctr[0] = t;
    ctr[1] = k;
    ctr[2] = (m << 4) | (uint32_t)blk;
    ctr[3] = (tag << 30) | ((problem_id & 0x3FFu) << 20) | (iter & 0xFFFFFu);
    orc_philox(ctr, key, r);
    double u[4];
    for (int i = 0; i < 4; ++i) u[i] = ((double)(r[i] >> 9) + 0.5) * (1.0 / 8388608.0);
    double rad0 = sqrt(-2.0 * log(u[0])), rad1 = sqrt(-2.0 * log(u[2]));
    double nv[4] = {rad0 * cos(two_pi * u[1]), rad0 * sin(two_pi * u[1]),
                    rad1 * cos(two_pi * u[3]), rad1 * sin(two_pi * u[3])};
    for (int i = 0; i < 4 && blk * 4 + i < n; ++i) out[blk * 4 + i] = nv[i];
  }
}

/* -------------------------------------------------------------------- LWPR */

/* Local PLS prediction of model j at centred input delta (reading R2). */
static double local_prediction(const orc_model *md, int64_t j, const double *delta, double *work) {
  const int d = md->d, R = md->R;
  const double *U = md->proj_u + j * R * d;
  const double *P = md->proj_p ? md->proj_p + j * R * d : U;
  const double *B = md->beta + j * (R + 1);
  for (int a = 0; a < d; ++a) work[a] = delta[a];
  double y = B[0];
  for (int r = 0; r < R; ++r) {
    double s = 0.0;
    for (int a = 0; a < d; ++a) s += U[r * d + a] * work[a];
    for (int a = 0; a < d; ++a) work[a] -= s * P[r * d + a];
    y += B[r + 1] * s;
  }
  return y;
}

/* Quadratic form (z - c_j)^T D_j (z - c_j), full matrix product. */
static double kernel_distance(const orc_model *md, int64_t j, const double *z, double *delta) {
  const int d = md->d;
  const double *c = md->centre + j * d;
  const double *D = md->metric + j * d * d;
  for (int a = 0; a < d; ++a) delta[a] = z[a] - c[a];
  double q = 0.0;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) q += delta[a] * D[a * d + b] * delta[b];
  return q;
}

/* Eq. (1) for output o: weights, local predictions, mean and variance.
 * w and y must hold L_o entries; work must hold 2*d. */
static void mixture(const orc_model *md, int o, const double *z, double *w, double *y,
                    double *mean, double *var, double *work) {
  const int64_t j0 = md->L_off[o], j1 = md->L_off[o + 1];
  const int64_t L = j1 - j0;
  double *delta = work, *tmp = work + md->d;
  double amax = -INFINITY;
  for (int64_t i = 0; i < L; ++i) {
    double q = kernel_distance(md, j0 + i, z, delta);
    w[i] = -0.5 * q;                       /* activation a_j */
    if (w[i] > amax) amax = w[i];
    y[i] = local_prediction(md, j0 + i, delta, tmp);
  }
  double Z = 0.0;
  for (int64_t i = 0; i < L; ++i) { w[i] = exp(w[i] - amax); Z += w[i]; }
  for (int64_t i = 0; i < L; ++i) w[i] /= Z;
  double mu = 0.0;                          /* pass 1: mean */
  for (int64_t i = 0; i < L; ++i) mu += w[i] * y[i];
  double v = 0.0;                           /* pass 2: variance */
  for (int64_t i = 0; i < L; ++i) {
    double e = mu - y[i];
    v += w[i] * (e * e + md->sigma2[j0 + i]);
  }
  *mean = mu;
  *var = v;
}

static int64_t max_L(const orc_model *md) {
  int64_t m = 1;
  for (int o = 0; o < md->n_out; ++o) {
    int64_t L = md->L_off[o + 1] - md->L_off[o];
    if (L > m) m = L;
  }
  return m;
}

/* mean, var: [N][n_out]; weights (nullable): [N][Ltot] normalised per output. */
void orc_lwpr_predict(const orc_model *md, const double *Z, int64_t N, double *mean,
                      double *var, double *weights, int32_t nthreads) {
  const int64_t Lm = max_L(md), Lt = md->L_off[md->n_out];
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    double *w = malloc(sizeof(double) * Lm), *y = malloc(sizeof(double) * Lm);
    double *work = malloc(sizeof(double) * 2 * md->d);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
    for (int64_t n = 0; n < N; ++n) {
      for (int o = 0; o < md->n_out; ++o) {
        mixture(md, o, Z + n * md->d, w, y, &mean[n * md->n_out + o], &var[n * md->n_out + o],
                work);
        if (weights) {
          int64_t L = md->L_off[o + 1] - md->L_off[o];
          memcpy(weights + n * Lt + md->L_off[o], w, sizeof(double) * L);
        }
      }
    }
    free(w); free(y); free(work);
  }
}

/* ---------------------------------------------------------------- dynamics */

static int n_state(int dyn) { return dyn == ORC_POINTMASS2D ? 4 : (dyn == ORC_QUAD_HYBRID ? 9 : 12); }
static int n_control(int dyn) { return dyn == ORC_POINTMASS2D ? 2 : 4; }
static int n_pos(int dyn) { return dyn == ORC_POINTMASS2D ? 2 : 3; }

/* The LWPR input for state x and applied control u (readings R3, R9). */
static void model_input(int dyn, const double *x, const double *u, double *z) {
  if (dyn == ORC_QUAD_HYBRID) {
    /* euler angles phi, theta, psi and the thrust F */
    z[0] = x[6];
    z[1] = x[7];
    z[2] = x[8];
    z[3] = u[3];
    return;
  }
  const int nx = n_state(dyn), nu = n_control(dyn);
  for (int a = 0; a < nx; ++a) z[a] = x[a];
  for (int a = 0; a < nu; ++a) z[nx + a] = u[a];
}

/* Explicit Euler (Table 1 caption): positions integrate velocities, velocities
 * integrate the sampled linear accelerations; for the 12-state quadrotor the
 * Euler angles integrate the body rates and the rates integrate the angular
 * accelerations; for the hybrid model the angles relax towards the commanded
 * rates u[0..2] (reading R9).  All right-hand sides use the old state. */
static void euler_step(int dyn, double dt, const double *x, const double *acc, const double *u,
                       double *xn) {
  const int np = n_pos(dyn);
  for (int a = 0; a < np; ++a) {
    xn[a] = x[a] + dt * x[np + a];
    xn[np + a] = x[np + a] + dt * acc[a];
  }
  if (dyn == ORC_QUAD12) {
    for (int a = 0; a < 3; ++a) {
      xn[6 + a] = x[6 + a] + dt * x[9 + a];
      xn[9 + a] = x[9 + a] + dt * acc[3 + a];
    }
  } else if (dyn == ORC_QUAD_HYBRID) {
    for (int a = 0; a < 3; ++a) {
      double rate = ORC_RATE_GAIN * (u[a] - x[6 + a]);
      xn[6 + a] = x[6 + a] + dt * rate;
    }
  }
}

/* State cost q(x) of Sec. 5: weighted goal distance, angle and velocity
 * penalties, and an obstacle term (indicator with a fixed penalty, or the
 * smooth sum of Gaussian bumps in the horizontal distances). */
static double state_cost(const orc_problem *p, const double *x) {
  const int np = n_pos(p->dyn);
  double c = 0.0;
  for (int a = 0; a < np; ++a) {
    double e = x[a] - p->goal[a];
    c += p->w_pos[a] * e * e;
  }
  for (int a = 0; a < np; ++a) c += p->w_vel * x[np + a] * x[np + a];
  if (p->dyn != ORC_POINTMASS2D) /* the three euler angles */
    for (int a = 0; a < 3; ++a) c += p->w_ang * x[6 + a] * x[6 + a];
  if (p->obs_kind == ORC_OBS_INDICATOR) {
    int inside = 0;
    for (int i = 0; i < p->n_obs; ++i) {
      double dx = x[0] - p->obs[3 * i], dy = x[1] - p->obs[3 * i + 1], r = p->obs[3 * i + 2];
      if (dx * dx + dy * dy < r * r) inside = 1;
    }
    if (inside) c += p->obs_penalty;
  } else {
    for (int i = 0; i < p->n_obs; ++i) {
      double dx = x[0] - p->obs[3 * i], dy = x[1] - p->obs[3 * i + 1];
      c += p->obs_penalty * exp(-p->obs_decay * (dx * dx + dy * dy));
    }
  }
  return c;
}

/* d q / d x (the indicator contributes nothing almost everywhere). */
static void state_cost_grad(const orc_problem *p, const double *x, double *g) {
  const int np = n_pos(p->dyn), nx = n_state(p->dyn);
  for (int a = 0; a < nx; ++a) g[a] = 0.0;
  for (int a = 0; a < np; ++a) g[a] += 2.0 * p->w_pos[a] * (x[a] - p->goal[a]);
  for (int a = 0; a < np; ++a) g[np + a] += 2.0 * p->w_vel * x[np + a];
  if (p->dyn != ORC_POINTMASS2D)
    for (int a = 0; a < 3; ++a) g[6 + a] += 2.0 * p->w_ang * x[6 + a];
  if (p->obs_kind == ORC_OBS_SMOOTH) {
    for (int i = 0; i < p->n_obs; ++i) {
      double dx = x[0] - p->obs[3 * i], dy = x[1] - p->obs[3 * i + 1];
      double e = p->obs_penalty * exp(-p->obs_decay * (dx * dx + dy * dy));
      g[0] += -2.0 * p->obs_decay * dx * e;
      g[1] += -2.0 * p->obs_decay * dy * e;
    }
  }
}

/* Control terms of S-tilde for one step (reading R10): u the nominal
 * control, eps the step's sampled perturbation of it (both [n_u]). */
static double control_cost(const orc_problem *p, const double *u, const double *eps) {
  if (!p->ctrl_cost) return 0.0;
  double G[3][3] = {{0}}, Rinv[3][3] = {{0}}, H[3][3] = {{0}}, Hinv[3][3] = {{0}};
  for (int a = 0; a < 3; ++a) {
    G[a][a] = ORC_RATE_GAIN;
    Rinv[a][a] = p->noise_std[a] * p->noise_std[a] * p->dt / p->lam;
  }
  /* H = G R^-1 G^T (diagonal here, since G and R are) */
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c)
        for (int e = 0; e < 3; ++e) H[a][b] += G[a][c] * Rinv[c][e] * G[b][e];
  for (int a = 0; a < 3; ++a) Hinv[a][a] = 1.0 / H[a][a];
  /* M = G^T H^-1 G */
  double M[3][3] = {{0}};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c)
        for (int e = 0; e < 3; ++e) M[a][b] += G[c][a] * Hinv[c][e] * G[e][b];
  /* B dw = G eps dt */
  double Bdw[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Bdw[a] += G[a][b] * eps[b] * p->dt;
  double quad = 0.0, cross = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) quad += u[a] * M[a][b] * u[b];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) cross += u[a] * G[b][a] * Hinv[b][c] * Bdw[c];
  return quad * p->dt + cross;
}

/* Per-rollout scratch for the step function. */
typedef struct {
  double *w, *y, *work;
} step_scratch;

/* One sampled step of sub-rollout m of rollout k (readings R3, R4). */
static void rollout_step(const orc_problem *p, const orc_model *md, const double *x,
                         const double *u_nom_t, uint32_t iter, int64_t k, int m, int t,
                         step_scratch *s, double *xn, double *mean_out, double *var_out,
                         double *ctrl_out) {
  const int nx = n_state(p->dyn), nu = n_control(p->dyn), no = md->n_out;
  double eps[4], xi[8], z[32], acc[8], u[4], pert[4];
  (void)nx;
  orc_normals(p->seed, ORC_TAG_CTRL, p->problem_id, iter, (uint32_t)k, 0u, (uint32_t)t, nu, eps);
  if (p->M > 0)
    orc_normals(p->seed, ORC_TAG_DYN, p->problem_id, iter, (uint32_t)k, (uint32_t)m,
                (uint32_t)t, no, xi);
  for (int a = 0; a < nu; ++a) {
    pert[a] = p->noise_std[a] * eps[a];
    u[a] = u_nom_t[a] + pert[a];
  }
  if (ctrl_out) *ctrl_out = control_cost(p, u_nom_t, pert);
  model_input(p->dyn, x, u, z);
  for (int o = 0; o < no; ++o) {
    double mu, v;
    mixture(md, o, z, s->w, s->y, &mu, &v, s->work);
    acc[o] = (p->M > 0) ? mu + sqrt(v) * xi[o] : mu;
    if (mean_out) mean_out[o] = mu;
    if (var_out) var_out[o] = v;
  }
  euler_step(p->dyn, p->dt, x, acc, u, xn);
}

/* cost: [(k1-k0)][T] = cbar_{k,t}; states (nullable): [(k1-k0)][max(M,1)][T+1][n_x]. */
void orc_rollout_cost(const orc_problem *p, const orc_model *md, const double *x0,
                      const double *u_nom, uint32_t iter, int64_t k0, int64_t k1, double *cost,
                      double *states, int32_t nthreads) {
  const int nx = n_state(p->dyn), nu = n_control(p->dyn), T = p->T;
  const int Ms = p->M > 0 ? p->M : 1;
  const int64_t Lm = max_L(md);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    step_scratch s;
    s.w = malloc(sizeof(double) * Lm);
    s.y = malloc(sizeof(double) * Lm);
    s.work = malloc(sizeof(double) * 2 * md->d);
    double *xs = malloc(sizeof(double) * (T + 1) * nx);
    double *csum = malloc(sizeof(double) * T);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
    for (int64_t k = k0; k < k1; ++k) {
      for (int t = 0; t < T; ++t) csum[t] = 0.0;
      for (int m = 0; m < Ms; ++m) {
        for (int a = 0; a < nx; ++a) xs[a] = x0[a];
        for (int t = 0; t < T; ++t) {
          double ctrl = 0.0;
          rollout_step(p, md, xs + t * nx, u_nom + t * nu, iter, k, m, t, &s, xs + (t + 1) * nx,
                       NULL, NULL, &ctrl);
          csum[t] += p->dt * state_cost(p, xs + (t + 1) * nx) + ctrl;
        }
        if (states)
          memcpy(states + ((k - k0) * Ms + m) * (int64_t)(T + 1) * nx, xs,
                 sizeof(double) * (T + 1) * nx);
      }
      for (int t = 0; t < T; ++t) cost[(k - k0) * T + t] = csum[t] / Ms;
    }
    free(s.w); free(s.y); free(s.work); free(xs); free(csum);
  }
}

/* ------------------------------------------------------------------ update */

/* Eq. (2) with the cost-to-go of Sec. 3.1 (reading R6). cost: [K][T];
 * u_nom: [T][n_u] updated in place; weights (nullable): [T][K]. */
void orc_update(const orc_problem *p, const double *cost, uint32_t iter, double *u_nom,
                double *weights) {
  const int K = p->K, T = p->T, nu = n_control(p->dyn);
  double *S = malloc(sizeof(double) * (size_t)K * T);
  for (int k = 0; k < K; ++k) {
    for (int i = 0; i < T; ++i) {
      double s = 0.0;
      int from = (p->weighting == ORC_W_TRAJECTORY) ? 0 : i;
      for (int t = from; t < T; ++t) s += cost[(int64_t)k * T + t];
      S[(int64_t)k * T + i] = s;
    }
  }
  double *omega = malloc(sizeof(double) * K);
  for (int i = 0; i < T; ++i) {
    double smin = INFINITY;
    for (int k = 0; k < K; ++k)
      if (S[(int64_t)k * T + i] < smin) smin = S[(int64_t)k * T + i];
    double Zs = 0.0;
    for (int k = 0; k < K; ++k) {
      omega[k] = exp(-(S[(int64_t)k * T + i] - smin) / p->lam);
      Zs += omega[k];
    }
    double du[4] = {0, 0, 0, 0};
    for (int k = 0; k < K; ++k) {
      double eps[4];
      orc_normals(p->seed, ORC_TAG_CTRL, p->problem_id, iter, (uint32_t)k, 0u, (uint32_t)i, nu,
                  eps);
      double P = omega[k] / Zs;
      if (weights) weights[(int64_t)i * K + k] = P;
      for (int a = 0; a < nu; ++a) du[a] += P * p->noise_std[a] * eps[a];
    }
    for (int a = 0; a < nu; ++a) u_nom[i * nu + a] += du[a];
  }
  free(S);
  free(omega);
}

/* Receding-horizon advance (Sec. 3.1, last paragraph): execute u_0 on the
 * plant (here a draw from the learned model under the PLANT stream at the
 * current iteration word), shift the plan left by one step repeating the last
 * control.  The iteration word counts PI^2 iterations; it advances after each
 * update, so every iteration of a control step draws fresh noise. */
void orc_rh_shift(const orc_problem *p, const orc_model *md, double *x0, double *u_nom,
                  const uint32_t *iter) {
  const int nx = n_state(p->dyn), nu = n_control(p->dyn), no = md->n_out, T = p->T;
  const int64_t Lm = max_L(md);
  double *w = malloc(sizeof(double) * Lm), *y = malloc(sizeof(double) * Lm);
  double *work = malloc(sizeof(double) * 2 * md->d);
  double z[32], acc[8], xi[8], xn[16];
  orc_normals(p->seed, ORC_TAG_PLANT, p->problem_id, *iter, 0u, 0u, 0u, no, xi);
  model_input(p->dyn, x0, u_nom, z);
  for (int o = 0; o < no; ++o) {
    double mu, v;
    mixture(md, o, z, w, y, &mu, &v, work);
    acc[o] = mu + sqrt(v) * xi[o];
  }
  euler_step(p->dyn, p->dt, x0, acc, u_nom, xn);
  for (int a = 0; a < nx; ++a) x0[a] = xn[a];
  for (int t = 0; t + 1 < T; ++t)
    for (int a = 0; a < nu; ++a) u_nom[t * nu + a] = u_nom[(t + 1) * nu + a];
  free(w); free(y); free(work);
}

/* ----------------------------------------------------------------- adjoint */

/* Reverse-mode derivative of J = (1/(K max(M,1))) sum_{k,m,t} c_{k,m,t} with
 * eps and xi held fixed (reading R8).  Each sub-rollout stores its whole state
 * trajectory and is swept backwards; every quantity of Eq. (1) is recomputed
 * per step.  Gradients are accumulated per thread and summed in thread order.
 * g_u: [T][n_u], g_c: [Ltot][d], g_D: [Ltot][d][d].  Returns J. */
double orc_adjoint(const orc_problem *p, const orc_model *md, const double *x0,
                   const double *u_nom, uint32_t iter, double *g_u, double *g_c, double *g_D,
                   int32_t nthreads) {
  if (p->dyn == ORC_QUAD_HYBRID) return NAN; /* the adjoint covers the other two families */
  const int nx = n_state(p->dyn), nu = n_control(p->dyn), no = md->n_out, T = p->T;
  const int d = md->d, R = md->R;
  const int Ms = p->M > 0 ? p->M : 1;
  const int64_t Lt = md->L_off[no], Lm = max_L(md);
  const double scale = 1.0 / ((double)p->K * Ms);
  int nth = 1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  nth = omp_get_max_threads();
#endif
  double *acc_u = calloc((size_t)nth * T * nu, sizeof(double));
  double *acc_c = calloc((size_t)nth * Lt * d, sizeof(double));
  double *acc_D = calloc((size_t)nth * Lt * d * d, sizeof(double));
  double *acc_J = calloc((size_t)nth, sizeof(double));
#ifdef _OPENMP
#pragma omp parallel
#endif
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    double *gu = acc_u + (size_t)tid * T * nu, *gc = acc_c + (size_t)tid * Lt * d;
    double *gD = acc_D + (size_t)tid * Lt * d * d;
    double *xs = malloc(sizeof(double) * (T + 1) * nx);
    double *w = malloc(sizeof(double) * Lm), *y = malloc(sizeof(double) * Lm);
    double *work = malloc(sizeof(double) * 2 * d);
    double *delta = malloc(sizeof(double) * d), *rbar = malloc(sizeof(double) * d);
    double *dq = malloc(sizeof(double) * d);
    double *svals = malloc(sizeof(double) * (R > 0 ? R : 1));
    step_scratch s = {w, y, work};
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
    for (int64_t k = 0; k < p->K; ++k) {
      for (int m = 0; m < Ms; ++m) {
        /* forward sweep, storing every state */
        for (int a = 0; a < nx; ++a) xs[a] = x0[a];
        for (int t = 0; t < T; ++t) {
          rollout_step(p, md, xs + t * nx, u_nom + t * nu, iter, k, m, t, &s, xs + (t + 1) * nx,
                       NULL, NULL, NULL);
          acc_J[tid] += p->dt * state_cost(p, xs + (t + 1) * nx);
        }
        /* backward sweep; xbar is the adjoint of x_{t+1} */
        double xbar[16], gq[16];
        for (int a = 0; a < nx; ++a) xbar[a] = 0.0;
        for (int t = T - 1; t >= 0; --t) {
          const double *x = xs + t * nx, *x1 = xs + (t + 1) * nx;
          state_cost_grad(p, x1, gq);
          for (int a = 0; a < nx; ++a) xbar[a] += p->dt * gq[a];
          /* rebuild z_t and the noise of this step */
          double eps[4], xi[8], z[32], zbar[32], abar[8];
          orc_normals(p->seed, ORC_TAG_CTRL, p->problem_id, iter, (uint32_t)k, 0u, (uint32_t)t,
                      nu, eps);
          if (p->M > 0)
            orc_normals(p->seed, ORC_TAG_DYN, p->problem_id, iter, (uint32_t)k, (uint32_t)m,
                        (uint32_t)t, no, xi);
          for (int a = 0; a < nx; ++a) z[a] = x[a];
          for (int a = 0; a < nu; ++a) z[nx + a] = u_nom[t * nu + a] + p->noise_std[a] * eps[a];
          for (int a = 0; a < d; ++a) zbar[a] = 0.0;
          /* Euler transpose: abar from the velocity/rate slots of xbar */
          const int np = n_pos(p->dyn);
          for (int a = 0; a < np; ++a) abar[a] = p->dt * xbar[np + a];
          if (p->dyn == ORC_QUAD12)
            for (int a = 0; a < 3; ++a) abar[3 + a] = p->dt * xbar[9 + a];
          double xprev[16];
          for (int a = 0; a < nx; ++a) xprev[a] = xbar[a];
          for (int a = 0; a < np; ++a) xprev[np + a] += p->dt * xbar[a];
          if (p->dyn == ORC_QUAD12)
            for (int a = 0; a < 3; ++a) xprev[9 + a] += p->dt * xbar[6 + a];
          /* through the mixture of every output */
          for (int o = 0; o < no; ++o) {
            double mu, v;
            mixture(md, o, z, w, y, &mu, &v, work);
            double mubar = abar[o];
            double vbar = (p->M > 0 && v > 0.0) ? abar[o] * xi[o] / (2.0 * sqrt(v)) : 0.0;
            const int64_t j0 = md->L_off[o], L = md->L_off[o + 1] - j0;
            for (int64_t i = 0; i < L; ++i) {
              const int64_t j = j0 + i;
              const double e = y[i] - mu;
              const double ybar = w[i] * (mubar + 2.0 * vbar * e);
              const double actbar = w[i] * (mubar * e + vbar * (e * e + md->sigma2[j] - v));
              const double qbar = -0.5 * actbar;
              const double *c = md->centre + j * d, *D = md->metric + j * d * d;
              const double *U = md->proj_u + j * R * d;
              const double *P = md->proj_p ? md->proj_p + j * R * d : U;
              const double *B = md->beta + j * (R + 1);
              for (int a = 0; a < d; ++a) delta[a] = z[a] - c[a];
              /* PLS deflation, forward then reverse */
              for (int a = 0; a < d; ++a) work[a] = delta[a];
              for (int r = 0; r < R; ++r) {
                double sv = 0.0;
                for (int a = 0; a < d; ++a) sv += U[r * d + a] * work[a];
                svals[r] = sv;
                for (int a = 0; a < d; ++a) work[a] -= sv * P[r * d + a];
              }
              for (int a = 0; a < d; ++a) rbar[a] = 0.0;
              for (int r = R - 1; r >= 0; --r) {
                double pr = 0.0;
                for (int a = 0; a < d; ++a) pr += P[r * d + a] * rbar[a];
                double sbar = B[r + 1] * ybar - pr;
                for (int a = 0; a < d; ++a) rbar[a] += sbar * U[r * d + a];
              }
              /* quadratic form: dq/ddelta = (D + D^T) delta, dq/dD = delta delta^T */
              for (int a = 0; a < d; ++a) {
                double sv = 0.0;
                for (int b = 0; b < d; ++b) sv += (D[a * d + b] + D[b * d + a]) * delta[b];
                dq[a] = sv;
              }
              for (int a = 0; a < d; ++a) {
                const double db = rbar[a] + qbar * dq[a];
                zbar[a] += db;
                gc[j * d + a] -= db;
              }
              for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) gD[(j * d + a) * d + b] += qbar * delta[a] * delta[b];
            }
          }
          for (int a = 0; a < nu; ++a) gu[t * nu + a] += zbar[nx + a];
          for (int a = 0; a < nx; ++a) xbar[a] = xprev[a] + zbar[a];
        }
      }
    }
    free(xs); free(w); free(y); free(work); free(delta); free(rbar); free(dq); free(svals);
  }
  double J = 0.0;
  for (int th = 0; th < nth; ++th) J += acc_J[th];
  for (int64_t i = 0; i < (int64_t)T * nu; ++i) {
    double sv = 0.0;
    for (int th = 0; th < nth; ++th) sv += acc_u[(size_t)th * T * nu + i];
    g_u[i] = sv * scale;
  }
  for (int64_t i = 0; i < Lt * d; ++i) {
    double sv = 0.0;
    for (int th = 0; th < nth; ++th) sv += acc_c[(size_t)th * Lt * d + i];
    g_c[i] = sv * scale;
  }
  for (int64_t i = 0; i < Lt * d * d; ++i) {
    double sv = 0.0;
    for (int th = 0; th < nth; ++th) sv += acc_D[(size_t)th * Lt * d * d + i];
    g_D[i] = sv * scale;
  }
  free(acc_u); free(acc_c); free(acc_D); free(acc_J);
  return J * scale;
}

int32_t orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Batch helpers for the tests (loops over the functions above). */
void orc_philox_many(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out) {
  for (int64_t i = 0; i < n; ++i) orc_philox(ctr + 4 * i, key, out + 4 * i);
}

/* out[(k - k0)][t][0..n) = normals of draw (tag, k, m, t) for k0 <= k < k0 + nk. */
void orc_noise_block(uint64_t seed, uint32_t tag, uint32_t problem_id, uint32_t iter, int64_t k0,
                     int64_t nk, uint32_t m, int32_t T, int32_t n, double *out) {
  for (int64_t kk = 0; kk < nk; ++kk)
    for (int32_t t = 0; t < T; ++t)
      orc_normals(seed, tag, problem_id, iter, (uint32_t)(k0 + kk), m, (uint32_t)t, n,
                  out + (kk * T + t) * n);
}
