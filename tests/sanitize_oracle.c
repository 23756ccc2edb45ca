/* Drives every entry point of the FP64 oracle on small instances of each
 * dynamics family, so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer checks its memory accesses and arithmetic
 * (tests/test_sanitizers.py builds and runs it on the CPU).  Exits 0 after
 * printing "ok" when every call completed and returned finite values. */
#include "../oracle/pi2rh_oracle.c"

#include <stdio.h>

static uint64_t state = 0x9E3779B97F4A7C15ULL;
static double urand(void) { /* 53-bit uniform in [0, 1) from a 64-bit LCG */
  state = state * 6364136223846793005ULL + 1442695040888963407ULL;
  return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}
static double sym(void) { return 2.0 * urand() - 1.0; }

static int finite_all(const double *a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(a[i])) return 0;
  return 1;
}

static int run_case(int dyn, int M, int obs_kind, int ctrl, int with_p) {
  const int n_out = dyn == ORC_POINTMASS2D ? 2 : dyn == ORC_QUAD12 ? 6 : 3;
  const int d = dyn == ORC_POINTMASS2D ? 6 : dyn == ORC_QUAD12 ? 16 : 4;
  const int nx = dyn == ORC_POINTMASS2D ? 4 : dyn == ORC_QUAD12 ? 12 : 9;
  const int nu = dyn == ORC_POINTMASS2D ? 2 : 4;
  const int R = 2, K = 3, T = 5, N = 7;
  int64_t L_off[9];
  L_off[0] = 0;
  for (int o = 0; o < n_out; ++o) L_off[o + 1] = L_off[o] + 1 + (o % 3);
  const int64_t Lt = L_off[n_out];
  double *c = malloc(sizeof(double) * Lt * d), *D = malloc(sizeof(double) * Lt * d * d);
  double *U = malloc(sizeof(double) * Lt * R * d), *P = malloc(sizeof(double) * Lt * R * d);
  double *B = malloc(sizeof(double) * Lt * (R + 1)), *s2 = malloc(sizeof(double) * Lt);
  for (int64_t j = 0; j < Lt; ++j) {
    for (int a = 0; a < d; ++a) c[j * d + a] = sym();
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) D[(j * d + a) * d + b] = (a == b ? 0.8 : 0.0) + 0.05 * (a + b) / (double)d;
    for (int r = 0; r < R; ++r)
      for (int a = 0; a < d; ++a) {
        U[(j * R + r) * d + a] = sym() / sqrt((double)d);
        P[(j * R + r) * d + a] = sym() / sqrt((double)d);
      }
    for (int r = 0; r <= R; ++r) B[j * (R + 1) + r] = sym();
    s2[j] = 0.01 + 0.01 * urand();
  }
  orc_model md = {d, n_out, R, L_off, c, D, U, with_p ? P : NULL, B, s2};
  double obs[3 * 3];
  for (int i = 0; i < 3; ++i) {
    obs[3 * i] = sym();
    obs[3 * i + 1] = sym();
    obs[3 * i + 2] = 0.2;
  }
  orc_problem p;
  memset(&p, 0, sizeof(p));
  p.dyn = dyn;
  p.K = K;
  p.T = T;
  p.M = M;
  p.dt = 0.02;
  p.lam = 1.0;
  for (int a = 0; a < 4; ++a) p.noise_std[a] = 0.3 + 0.1 * a;
  for (int a = 0; a < 3; ++a) {
    p.goal[a] = sym();
    p.w_pos[a] = 1.0 + a;
  }
  p.w_ang = 0.2;
  p.w_vel = 0.1;
  p.obs_kind = obs_kind;
  p.n_obs = 3;
  p.obs = obs;
  p.obs_penalty = obs_kind == ORC_OBS_SMOOTH ? 100.0 : 1000.0;
  p.obs_decay = 10.0;
  p.weighting = ORC_W_COST_TO_GO;
  p.seed = 0xC0FFEE00ULL + (uint64_t)dyn;
  p.problem_id = 3;
  p.ctrl_cost = ctrl;
  const int Ms = M > 0 ? M : 1;
  double *Z = malloc(sizeof(double) * N * d), *mean = malloc(sizeof(double) * N * n_out);
  double *var = malloc(sizeof(double) * N * n_out), *w = malloc(sizeof(double) * N * Lt);
  for (int i = 0; i < N * d; ++i) Z[i] = sym();
  double *x0 = calloc(nx, sizeof(double)), *u = malloc(sizeof(double) * T * nu);
  for (int a = 0; a < 3 && a < nx; ++a) x0[a] = sym();
  for (int i = 0; i < T * nu; ++i) u[i] = 0.3 * sym();
  double *cost = malloc(sizeof(double) * K * T), *st = malloc(sizeof(double) * K * Ms * (T + 1) * nx);
  double *W = malloc(sizeof(double) * T * K);
  double *gu = malloc(sizeof(double) * T * nu), *gc = malloc(sizeof(double) * Lt * d);
  double *gD = malloc(sizeof(double) * Lt * d * d);
  double nz[16];
  uint32_t it = 2;
  orc_lwpr_predict(&md, Z, N, mean, var, w, 1);
  orc_rollout_cost(&p, &md, x0, u, it, 0, K, cost, st, 1);
  orc_update(&p, cost, it, u, W);
  orc_rh_shift(&p, &md, x0, u, &it);
  orc_normals(p.seed, ORC_TAG_DYN, p.problem_id, it, 1, 0, 2, n_out, nz);
  int ok = finite_all(mean, N * n_out) && finite_all(var, N * n_out) && finite_all(w, N * Lt) &&
           finite_all(cost, K * T) && finite_all(st, K * Ms * (T + 1) * nx) && finite_all(W, T * K) &&
           finite_all(u, T * nu) && finite_all(x0, nx) && finite_all(nz, n_out);
  if (dyn != ORC_QUAD_HYBRID && !ctrl) {
    const double J = orc_adjoint(&p, &md, x0, u, it, gu, gc, gD, 1);
    ok = ok && isfinite(J) && finite_all(gu, T * nu) && finite_all(gc, Lt * d) && finite_all(gD, Lt * d * d);
  }
  free(c), free(D), free(U), free(P), free(B), free(s2), free(Z), free(mean), free(var), free(w);
  free(x0), free(u), free(cost), free(st), free(W), free(gu), free(gc), free(gD);
  if (!ok) fprintf(stderr, "non-finite result: dyn %d M %d obs %d ctrl %d p %d\n", dyn, M, obs_kind, ctrl, with_p);
  return ok;
}

int main(void) {
  int ok = 1;
  for (int dyn = 0; dyn < 3; ++dyn)
    for (int M = 0; M <= 2; M += 2)
      for (int obs = 0; obs < 2; ++obs)
        ok = run_case(dyn, M, obs, 0, (dyn + M + obs) % 2) && ok;
  ok = run_case(ORC_QUAD_HYBRID, 1, ORC_OBS_SMOOTH, 1, 0) && ok;
  uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4], many[8];
  orc_philox(ctr, key, out);
  uint32_t ctrs[8] = {0, 1, 2, 3, 4, 5, 6, 7};
  orc_philox_many(2, ctrs, key, many);
  printf(ok ? "ok\n" : "FAILED\n");
  return ok ? 0 : 1;
}
