// Drives the host side of the C ABI -- argument validation, workspace and
// layout arithmetic, the batched work list -- on a machine without a GPU, so
// that a build whose host code carries AddressSanitizer and
// UndefinedBehaviorSanitizer checks it (tests/test_sanitizers.py builds and
// runs it on the CPU).  Every call either fails validation with the expected
// status or reaches the device check (PI_ERR_DEVICE).  Prints "ok".
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include <hip/hip_runtime_api.h>

#include "../include/pi2rh.h"

static int failures = 0;
#define EXPECT(cond)                                                     \
  do {                                                                   \
    if (!(cond)) {                                                       \
      fprintf(stderr, "line %d: %s (%s)\n", __LINE__, #cond, pi_last_error()); \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

static char fake_mem[64];
static void *const FAKE = fake_mem;   // never dereferenced: no device work happens

static pi_lwpr model(int dtype, int d, int n_out, int per_out) {
  pi_lwpr m;
  memset(&m, 0, sizeof(m));
  m.dtype = dtype;
  m.d = d;
  m.n_out = n_out;
  m.R = 2;
  for (int o = 0; o <= PI_MAX_OUT; ++o) m.L_off[o] = (o <= n_out ? o : n_out) * per_out;
  m.centre = m.metric = m.proj_u = m.beta = m.sigma2 = FAKE;
  return m;
}

static pi_problem problem(int dtype, int dyn, int K, int T, int M) {
  pi_problem p;
  memset(&p, 0, sizeof(p));
  p.dtype = dtype;
  p.dyn = dyn;
  p.K = K;
  p.T = T;
  p.M = M;
  p.dt = 0.02;
  p.lambda = 1.0;
  for (int a = 0; a < PI_MAX_U; ++a) p.noise_std[a] = 0.5;
  p.n_obs = 3;
  p.obs = FAKE;
  p.obs_penalty = 1000.0;
  p.obs_decay = 10.0;
  p.seed = 7;
  return p;
}

int main() {
  // valid requests below would reach a device with fake pointers: run only
  // where no GPU is visible
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) == hipSuccess && n_dev > 0) {
    printf("skip: a GPU is visible\n");
    return 77;
  }
  const int dyns[3] = {PI_DYN_POINTMASS2D, PI_DYN_QUAD12, PI_DYN_QUAD_HYBRID};
  const int ds[3] = {6, 16, 4}, nos[3] = {2, 6, 3};
  for (int i = 0; i < 3; ++i)
    for (int dtype = PI_F32; dtype <= PI_F64; ++dtype)
      for (int M = 0; M <= 3; M += 3) {
        pi_problem p = problem(dtype, dyns[i], 1000 + 37 * i, 50, M);
        pi_lwpr m = model(dtype, ds[i], nos[i], 40 + i);
        for (int op = PI_OP_PREDICT; op <= PI_OP_RH_SHIFT; ++op) {
          const size_t n = pi_workspace_bytes(op, &p, &m);
          if (op == PI_OP_ADJOINT && dyns[i] == PI_DYN_QUAD_HYBRID) continue;
          EXPECT(n != (size_t)-1 && n < ((size_t)1 << 40));
        }
        for (int ck = 0; ck <= 60; ck += 7) {
          const size_t a = pi_adjoint_workspace_bytes(&p, &m, ck);
          EXPECT(dyns[i] == PI_DYN_QUAD_HYBRID ? a == (size_t)-1 : a < ((size_t)1 << 40));
        }
        EXPECT(pi_model_fold_bytes(&m) < ((size_t)1 << 40));
        for (int split = 0; split <= 2; ++split) {
          p.tile_split = split;
          EXPECT(pi_rollout_cost(&p, &m, FAKE, FAKE, (const uint32_t *)FAKE, FAKE, FAKE, (size_t)1 << 40,
                                 NULL) == PI_ERR_DEVICE);
          EXPECT(pi_rollout_cost_noalloc(&p, &m, FAKE, FAKE, (const uint32_t *)FAKE, FAKE, NULL) ==
                 (pi_workspace_bytes(PI_OP_ROLLOUT, &p, &m) > PI_NOALLOC_SCRATCH_BYTES ? PI_ERR_WORKSPACE
                                                                                        : PI_ERR_DEVICE));
          int32_t out[4];
          EXPECT(pi_rollout_describe(&p, &m, out) == PI_ERR_DEVICE);
        }
        EXPECT(pi_update(&p, FAKE, (const uint32_t *)FAKE, FAKE, NULL, FAKE, (size_t)1 << 40, NULL) ==
               PI_ERR_DEVICE);
        EXPECT(pi_rh_shift(&p, &m, FAKE, FAKE, (const uint32_t *)FAKE, FAKE, (size_t)1 << 40, NULL) ==
               PI_ERR_DEVICE);
        EXPECT(lwpr_predict(&m, FAKE, 33, FAKE, FAKE, PI_VARIANT_AUTO, FAKE, (size_t)1 << 40, NULL) ==
               PI_ERR_DEVICE);
        // invalid requests fail before the device
        p.K = 0;
        EXPECT(pi_rollout_cost(&p, &m, FAKE, FAKE, (const uint32_t *)FAKE, FAKE, FAKE, 1, NULL) == PI_ERR_SHAPE);
        p.K = 5;
        EXPECT(pi_rollout_cost(&p, &m, FAKE, FAKE, (const uint32_t *)FAKE, FAKE, FAKE, 0, NULL) ==
               PI_ERR_WORKSPACE);
        m.L_off[1] = 0;
        EXPECT(pi_rollout_cost(&p, &m, FAKE, FAKE, (const uint32_t *)FAKE, FAKE, FAKE, 1, NULL) == PI_ERR_SHAPE);
      }
  // batched: uneven problems, per-problem tiles, a pre-folded model
  const int B = 5;
  std::vector<pi_problem> ps;
  std::vector<pi_lwpr> ms;
  std::vector<void *> ptrs(B, FAKE);
  std::vector<uint32_t *> iters(B, (uint32_t *)FAKE);
  for (int b = 0; b < B; ++b) {
    ps.push_back(problem(PI_F32, PI_DYN_QUAD12, 100 + 997 * b, 20 + 13 * b, b % 3));
    ps.back().tile_samples = (b % 2) ? 8 : 32;
    ms.push_back(model(PI_F32, 16, 6, 16 + 9 * b));
  }
  const size_t fb = pi_model_fold_bytes(&ms[1]);
  ms[1].folded = FAKE;
  ms[1].folded_bytes = fb;
  const size_t wb = pi_batched_workspace_bytes(B, ps.data(), ms.data());
  EXPECT(wb != (size_t)-1 && wb > 0);
  EXPECT(pi_rollout_cost_batched(B, ps.data(), ms.data(), (const void *const *)ptrs.data(),
                                 (const void *const *)ptrs.data(), (const uint32_t *const *)iters.data(),
                                 ptrs.data(), FAKE, wb, NULL) == PI_ERR_DEVICE);
  EXPECT(pi_control_step_batched(B, ps.data(), ms.data(), ptrs.data(), ptrs.data(), iters.data(), ptrs.data(),
                                 FAKE, wb, NULL) == PI_ERR_DEVICE);
  EXPECT(pi_control_step_batched(B, ps.data(), ms.data(), ptrs.data(), ptrs.data(), iters.data(), ptrs.data(),
                                 FAKE, wb - 1, NULL) == PI_ERR_WORKSPACE);
  ps[0].tile_waves = 8;   // 8 waves need tiles of at most 16
  EXPECT(pi_batched_workspace_bytes(B, ps.data(), ms.data()) == (size_t)-1);
  ps[0].tile_waves = 0;
  ps[2].dyn = PI_DYN_POINTMASS2D;
  EXPECT(pi_batched_workspace_bytes(B, ps.data(), ms.data()) == (size_t)-1);
  EXPECT(pi_rollout_cost_batched(0, ps.data(), ms.data(), NULL, NULL, NULL, NULL, NULL, 0, NULL) == PI_ERR_SHAPE);
  EXPECT(pi_philox4x32_10(NULL, 1, NULL, -1, NULL) == PI_ERR_SHAPE);
  uint64_t cnt;
  EXPECT(pi_pair_give_ups(&cnt, NULL) == PI_ERR_DEVICE);
  EXPECT(strlen(pi_version()) > 0);
  printf(failures ? "FAILED\n" : "ok\n");
  return failures ? 1 : 0;
}
