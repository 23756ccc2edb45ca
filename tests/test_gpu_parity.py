"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (each follows from the working precision of the path it checks):
  * LWPR mean/variance: normwise per output, max|g-o| / max|o| <= 1e-5 for
    FP32 (in-distribution inputs), 1e-11 for FP64;
  * trajectory costs S_k = sum_t cbar_{k,t}: relative 1e-4 per rollout for
    FP32 outside indicator flips (flips counted, <= 0.1 %), 1e-10 for FP64;
  * control updates: 1e-4 absolute (teacher-forced on identical costs),
    1e-10 for FP64 end to end;
  * random stream: Philox blocks bit-exact; normals to rounding.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import DYN_POINTMASS2D, DYN_QUAD12, OBS_SMOOTH, W_TRAJECTORY

torch = pytest.importorskip("torch")
pi = pytest.importorskip("paper_1503_00330_amd")

pytestmark = pytest.mark.gpu

F32, F64 = np.float32, np.float64


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    pi.load()
    yield
    torch.cuda.synchronize()


def nrel(g, o):
    """Normwise error per output column: max|g - o| / max|o|, worst column."""
    g, o = np.asarray(g, np.float64).reshape(len(g), -1), np.asarray(o, np.float64).reshape(len(o), -1)
    return float(np.max(np.abs(g - o).max(0) / np.maximum(np.abs(o).max(0), 1e-300)))


def c16(g, o):
    """Elementwise relative error with a floor for elements near zero:
    |g - o| / max(|o|, 1e-3 max|o|), worst element of the array."""
    g, o = np.asarray(g, np.float64).ravel(), np.asarray(o, np.float64).ravel()
    return float(np.max(np.abs(g - o) / np.maximum(np.abs(o), 1e-3 * max(np.abs(o).max(), 1e-300))))


def cost_check(g, o, prob, tol):
    """S_k relative errors outside rows whose obstacle indicator flips."""
    g, o = np.asarray(g, np.float64), np.asarray(o, np.float64)
    flip = np.abs(g - o).max(1) > 0.25 * prob.dt * prob.obs_penalty
    Sg, So = g.sum(1), o.sum(1)
    r = np.abs(Sg - So) / np.maximum(np.abs(So), 1e-30)
    ok = ~flip
    assert flip.sum() <= max(1, int(0.001 * len(g))), "indicator flips in %d rows" % flip.sum()
    assert r[ok].max(initial=0.0) <= tol, (r[ok].max(), np.argmax(np.where(ok, r, 0)))
    return r[ok].max(initial=0.0), int(flip.sum())


# ------------------------------------------------------------- random stream

def test_philox_blocks_bit_exact():
    rng = np.random.default_rng(1)
    n = 1 << 20
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = 0x0123456789ABCDEF
    g = pi.philox4x32_10(torch.from_numpy(ctr.view(np.int32)).cuda(), key)
    g = g.cpu().numpy().view(np.uint32)
    ref = oracle.philox_many(ctr, [key & 0xFFFFFFFF, key >> 32])
    assert np.array_equal(g, ref)


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("tag", [oracle.TAG_CTRL, oracle.TAG_DYN])
def test_noise_matches_oracle(dtype, tag):
    prob, _ = synth.tiny_problem(3, dyn=DYN_QUAD12, K=300, T=11, dtype=dtype)
    dp = pi.DeviceProblem(prob)
    dp.iter.fill_(7)
    m = 2 if tag == oracle.TAG_DYN else 0
    g = pi.noise(dp, tag, m=m).cpu().numpy()
    o = oracle.noise_block(prob, tag, it=7, m=m)
    if tag == oracle.TAG_CTRL:
        o = o * np.asarray(prob.noise_std, np.float64)
    tol = 1e-13 if dtype == F64 else 4e-6
    assert np.max(np.abs(g - o)) <= tol


# ------------------------------------------------------------ LWPR, Eq. (1)

def _models():
    rng = np.random.default_rng(77)
    return {
        "cfg1": synth.config(1)[1].astype(F64),
        "ragged16": synth.make_lwpr(rng, 16, [1, 17, 33, 5, 16, 40], 4),
        "pm6": synth.make_lwpr(rng, 6, [16, 16], 2),
        "d3": synth.make_lwpr(rng, 3, [7, 2], 2, loadings_equal_u=False),
        # deflation loadings p != u at the quadrotor's d = 16: the fold's
        # reverse accumulation through the deflation chain on the matrix-core form
        "pu16": synth.make_lwpr(rng, 16, [23, 16, 9, 31, 16, 40], 4, loadings_equal_u=False),
        "paper4": synth.paper_shape()[1].astype(F64),     # d = 4, 15/15/24 models
    }


MODELS = _models()
PRED_CASES = [("cfg1", pi.PI_VARIANT_MFMA, F32), ("cfg1", pi.PI_VARIANT_DIRECT, F32),
              ("cfg1", pi.PI_VARIANT_DIRECT, F64), ("ragged16", pi.PI_VARIANT_MFMA, F32),
              ("ragged16", pi.PI_VARIANT_DIRECT, F64), ("pm6", pi.PI_VARIANT_MFMA, F32),
              ("pm6", pi.PI_VARIANT_DIRECT, F64), ("d3", pi.PI_VARIANT_DIRECT, F32),
              ("d3", pi.PI_VARIANT_DIRECT, F64), ("paper4", pi.PI_VARIANT_MFMA, F32),
              ("paper4", pi.PI_VARIANT_DIRECT, F32), ("paper4", pi.PI_VARIANT_DIRECT, F64),
              ("cfg2", pi.PI_VARIANT_MFMA, F32), ("cfg2", pi.PI_VARIANT_DIRECT, F64),
              ("pu16", pi.PI_VARIANT_MFMA, F32), ("pu16", pi.PI_VARIANT_DIRECT, F32),
              ("pu16", pi.PI_VARIANT_DIRECT, F64)]


def _model(name):
    # the 6 x 1024-model set of the 65536-rollout workload is built on first use
    if name == "cfg2":
        return synth.config(2)[1].astype(F64)
    return MODELS[name]


@pytest.mark.parametrize("name,variant,dtype", PRED_CASES)
def test_lwpr_predict_parity(name, variant, dtype):
    model = _model(name).astype(dtype)
    N = 16 * 37 + 5
    Z = np.random.default_rng(5).uniform(-1, 1, (N, model.d)).astype(dtype)
    dm = pi.DeviceModel(model)
    mean, var = pi.lwpr_predict(dm, torch.from_numpy(Z).cuda(), variant)
    om, ov = oracle.lwpr_predict(model, Z)
    tol = 1e-11 if dtype == F64 else 1e-5
    gm, gv = mean.cpu().numpy(), var.cpu().numpy()
    assert nrel(gm, om) <= tol
    assert nrel(gv, ov) <= tol
    assert np.all(gv > 0)
    # elementwise (each output's array under the 1e-3 max|o| floor): reported,
    # and held to the bound that FP32 weights of a diffuse mixture allow (a
    # correctly rounded q already moves small means by ~2e-5 of max|o|)
    ew = max(max(c16(gm[:, o], om[:, o]), c16(gv[:, o], ov[:, o])) for o in range(model.n_out))
    print("%s %s %s: normwise %.2e / %.2e, elementwise %.2e" % (
        name, variant, np.dtype(dtype).name, nrel(gm, om), nrel(gv, ov), ew))
    assert ew <= (1e-10 if dtype == F64 else 1e-3)


def test_lwpr_predict_far_inputs_reported():
    # outside the model's support the FP32 weights lose relative accuracy
    # (error grows with q); finite and bounded is what is required there
    model = MODELS["cfg1"].astype(F32)
    Z = np.random.default_rng(6).uniform(-4, 4, (97, 16)).astype(F32)
    mean, var = pi.lwpr_predict(pi.DeviceModel(model), torch.from_numpy(Z).cuda())
    om, ov = oracle.lwpr_predict(model, Z)
    e = nrel(mean.cpu().numpy(), om)
    print("far-input normwise error %.2e" % e)
    assert np.all(np.isfinite(mean.cpu().numpy())) and e < 1e-3


@pytest.mark.parametrize("variant", [pi.PI_VARIANT_DIRECT, pi.PI_VARIANT_MFMA])
def test_lwpr_predict_variance_lower_bound(variant):
    # Eq. (1): var = sum w (y - mu)^2 + sum w sigma^2 >= min_j sigma_j^2 of the
    # output, at any input; far from the centres the local predictions differ
    # by hundreds, which in FP32 cancels the spread term to rounding noise
    model = MODELS["cfg1"].astype(F32)
    Z = np.random.default_rng(16).uniform(-40, 40, (301, 16)).astype(F32)
    mean, var = pi.lwpr_predict(pi.DeviceModel(model), torch.from_numpy(Z).cuda(), variant=variant)
    v = var.cpu().numpy()
    lo = np.array([model.sigma2[model.L_off[o]:model.L_off[o + 1]].min() for o in range(model.n_out)])
    assert np.all(np.isfinite(v)) and np.all(np.isfinite(mean.cpu().numpy()))
    assert np.all(v >= lo[None, :] * (1 - 1e-4))


@pytest.mark.parametrize("variant", [pi.PI_VARIANT_DIRECT, pi.PI_VARIANT_MFMA])
def test_long_horizon_fp32_rollout_stays_finite(variant):
    # the adjoint workload's horizon (T = 400): trajectories leave the models'
    # support, where FP32 rounding once made the sampled variance negative
    prob, model, _ = synth.config(4, obs_kind=synth.OBS_SMOOTH, K=64)
    dp, dm = pi.DeviceProblem(prob, variant=variant), pi.DeviceModel(model)
    c = pi.rollout_cost(dp, dm).cpu().numpy()
    assert np.all(np.isfinite(c))


def test_lwpr_predict_empty_and_single():
    model = MODELS["pm6"].astype(F32)
    dm = pi.DeviceModel(model)
    z = torch.zeros((0, 6), device="cuda")
    m, v = pi.lwpr_predict(dm, z)
    assert m.shape == (0, 2)
    z1 = np.full((1, 6), 0.25, F32)
    m, v = pi.lwpr_predict(dm, torch.from_numpy(z1).cuda())
    om, ov = oracle.lwpr_predict(model, z1)
    assert nrel(m.cpu().numpy(), om) <= 1e-5


# ----------------------------------------------------------------- rollouts

def test_rollout_fp64_config0_strict():
    prob, model, _ = synth.config(0)
    cost = pi.rollout_cost(pi.DeviceProblem(prob), pi.DeviceModel(model)).cpu().numpy()
    ref = oracle.rollout_cost(prob, model)
    r, flips = cost_check(cost, ref, prob, 1e-10)
    assert flips == 0
    assert np.max(np.abs(cost - ref)) <= 1e-10 * np.abs(ref).max()


# (variant, samples per workgroup, workgroups per tile, waves per workgroup);
# 0 = library's choice.  MFMA tiles of 16 rows on a pair of workgroups (split
# 0 = library's choice, which pairs these small problems, or 2 = forced) or on
# one (split 1), 8 rows, 32 rows; the same with the products in three bf16
# pieces (one or two 16-row tiles per wave, and the shared-tile launch of 128
# or 64 rows on 4 waves, 128 on 8); the same launches with the products in two
# fp16 pieces; and the direct kernel
BF3 = pi.PI_VARIANT_MFMA_BF16X3
HF2 = pi.PI_VARIANT_MFMA_F16X2
ROLLOUT_SHAPES = [(pi.PI_VARIANT_MFMA, 0, 0, 0), (pi.PI_VARIANT_MFMA, 16, 2, 4), (pi.PI_VARIANT_MFMA, 16, 2, 8),
                  (pi.PI_VARIANT_MFMA, 16, 1, 4), (pi.PI_VARIANT_MFMA, 16, 1, 8), (pi.PI_VARIANT_MFMA, 8, 1, 0),
                  (pi.PI_VARIANT_MFMA, 32, 0, 0), (BF3, 0, 0, 0), (BF3, 16, 2, 4), (BF3, 16, 1, 4),
                  (BF3, 16, 1, 8), (BF3, 8, 1, 8), (BF3, 32, 1, 4), (BF3, 128, 1, 4), (BF3, 64, 1, 4), (BF3, 128, 1, 8),
                  (HF2, 0, 0, 0), (HF2, 16, 2, 4), (HF2, 16, 1, 8), (HF2, 8, 1, 8), (HF2, 32, 1, 4),
                  (HF2, 128, 1, 4), (HF2, 64, 1, 4), (HF2, 128, 1, 8),
                  (pi.PI_VARIANT_DIRECT, 0, 0, 0)]


@pytest.mark.parametrize("shape", ROLLOUT_SHAPES)
@pytest.mark.parametrize("M", [0, 1, 3])
def test_rollout_fp32_ragged(shape, M):
    variant, spw, split, waves = shape
    prob, model = synth.tiny_problem(11, dyn=DYN_QUAD12, L=[20, 17, 33, 16, 1, 40], R=4, K=37, T=9,
                                     M=M, dtype=F32, n_obs=6)
    dp = pi.DeviceProblem(prob, variant=variant, tile_samples=spw, tile_split=split, tile_waves=waves)
    cost = pi.rollout_cost(dp, pi.DeviceModel(model)).cpu().numpy()
    ref = oracle.rollout_cost(prob, model)
    cost_check(cost, ref, prob, 1e-4)
    assert nrel(cost, ref) <= 1e-4


@pytest.mark.parametrize("variant,split,spw", [(pi.PI_VARIANT_MFMA, 1, 0), (pi.PI_VARIANT_MFMA, 2, 0),
                                               (BF3, 2, 0), (BF3, 1, 32), (BF3, 1, 128), (HF2, 2, 0), (HF2, 1, 32),
                                               (HF2, 1, 128)])
def test_rollout_loadings_differ_from_directions(variant, split, spw):
    # local models whose PLS deflation loadings p differ from the projection
    # directions u (d = 16, matrix-core tiles)
    prob, _ = synth.tiny_problem(19, dyn=DYN_QUAD12, L=3, R=4, K=53, T=13, M=1, dtype=F32, n_obs=5)
    model = MODELS["pu16"].astype(F32)
    dp = pi.DeviceProblem(prob, variant=variant, tile_split=split, tile_samples=spw)
    cost = pi.rollout_cost(dp, pi.DeviceModel(model)).cpu().numpy()
    ref = oracle.rollout_cost(prob, model)
    cost_check(cost, ref, prob, 1e-4)
    assert nrel(cost, ref) <= 1e-4


@pytest.mark.parametrize("variant,spw,split,waves", [(HF2, 0, 0, 0), (HF2, 16, 1, 8), (HF2, 32, 1, 4), (HF2, 128, 1, 8),
                                                     (HF2, 128, 1, 4), (BF3, 128, 1, 8), (pi.PI_VARIANT_MFMA, 0, 0, 0),
                                                     (pi.PI_VARIANT_DIRECT, 0, 0, 0)])
@pytest.mark.parametrize("far", [False, True])
def test_f16x2_power_of_two_scales(variant, spw, split, waves, far):
    # The fp16 form's powers of two.  Near: every third model's metric scaled
    # by 3000, so that its quadratic-form values pass 2^14 and its tile runs
    # the epilogue with the models' scales (the other models of those tiles
    # keep scale 1 and carry the weight).  Far: the plant starts 200 m out and
    # each output's first model is centred there, so that every row's
    # features z_a z_b pass 2^14 (row scales) and the models that carry the
    # weight have scaled values (c^T D c past 2^14).  The other contractions
    # run the same instances for comparison.
    prob, model = synth.tiny_problem(23, dyn=DYN_QUAD12, L=[20, 17, 33, 16, 1, 40], R=4, K=37, T=9, M=1,
                                     dtype=F32, n_obs=6)
    if far:   # goal and obstacles moved with the plant: costs of the dynamics, not of the offset
        prob.x0[:3] += np.float32(200.0)
        prob.goal[:3] += prob.goal.dtype.type(200.0)
        prob.obs[:, :2] += prob.obs.dtype.type(200.0)
        model.centre[model.L_off[:-1], :3] += np.float32(200.0)
    else:
        model.metric[::3] *= np.float32(3000.0)
    dp = pi.DeviceProblem(prob, variant=variant, tile_samples=spw, tile_split=split, tile_waves=waves)
    cost = pi.rollout_cost(dp, pi.DeviceModel(model)).cpu().numpy()
    ref = oracle.rollout_cost(prob, model)
    r, _ = cost_check(cost, ref, prob, 1e-4)
    print("f16x2 scales (far %s, %s): max S rel %.2e" % (far, (variant, spw, split, waves), r))
    assert nrel(cost, ref) <= 1e-4


@pytest.mark.parametrize("dtype,split", [(F32, 1), (F32, 2), (F64, 0)])
def test_rollout_pointmass(dtype, split):
    prob, model = synth.tiny_problem(12, dyn=DYN_POINTMASS2D, L=[9, 23], R=2, K=70, T=15, M=2,
                                     dtype=dtype, n_obs=3, obs_kind=OBS_SMOOTH)
    cost = pi.rollout_cost(pi.DeviceProblem(prob, tile_split=split), pi.DeviceModel(model)).cpu().numpy()
    ref = oracle.rollout_cost(prob, model)
    cost_check(cost, ref, prob, 1e-10 if dtype == F64 else 1e-4)


# (variant, samples per workgroup, split) for the paper's hybrid quadrotor
HYBRID_SHAPES = [(pi.PI_VARIANT_MFMA, 0, 0), (pi.PI_VARIANT_MFMA, 16, 1), (pi.PI_VARIANT_MFMA, 32, 0),
                 (pi.PI_VARIANT_DIRECT, 0, 0)]


@pytest.mark.parametrize("shape", HYBRID_SHAPES)
@pytest.mark.parametrize("M", [0, 1, 4])
def test_rollout_hybrid_quadrotor(shape, M):
    # the paper's model (Sec. 4.1): angles follow commanded rates, three
    # LWPR models of (angles, thrust) give the accelerations
    variant, spw, split = shape
    prob, model = synth.paper_shape(M=M, K=150, T=21)
    prob.u_nom = np.random.default_rng(M).normal(0.0, 0.3, prob.u_nom.shape).astype(F32)
    dp = pi.DeviceProblem(prob, variant=variant, tile_samples=spw, tile_split=split)
    cost = pi.rollout_cost(dp, pi.DeviceModel(model)).cpu().numpy()
    ref = oracle.rollout_cost(prob, model)
    cost_check(cost, ref, prob, 1e-4)
    assert nrel(cost, ref) <= 1e-4


# the control terms of S-tilde on the hybrid model: the matrix-core tiles
# (paired, single, 32 rows), the 16-lane direct kernel and, past 8192
# sub-rollouts, the lane-per-sub-rollout direct kernel
CTRL_SHAPES = HYBRID_SHAPES + [(pi.PI_VARIANT_DIRECT, 0, 0, 2100)]


@pytest.mark.parametrize("shape", CTRL_SHAPES)
@pytest.mark.parametrize("M", [0, 1, 4])
def test_rollout_control_terms(shape, M):
    variant, spw, split = shape[:3]
    K = shape[3] if len(shape) > 3 else 150
    prob, model = synth.paper_shape(M=M, K=K, T=37)
    prob.u_nom = np.random.default_rng(7 + M).normal(0.0, 0.3, prob.u_nom.shape).astype(F32)
    prob.ctrl_cost = 1
    dp = pi.DeviceProblem(prob, variant=variant, tile_samples=spw, tile_split=split)
    cost = pi.rollout_cost(dp, pi.DeviceModel(model)).cpu().numpy()
    ref = oracle.rollout_cost(prob, model)
    off = prob.copy()
    off.ctrl_cost = 0
    ctrl = ref - oracle.rollout_cost(off, model)
    assert np.abs(ctrl).max() > 0.1 * np.abs(ref).max()    # the terms matter here
    cost_check(cost, ref, prob, 1e-4)


def test_control_terms_fp64_iteration():
    # end to end in double: rollouts with the control terms, then the update
    # weighting by S-tilde
    prob, model = synth.paper_shape(M=1, K=96, T=17, dtype=F64)
    prob.u_nom = np.random.default_rng(3).normal(0.0, 0.3, prob.u_nom.shape)
    prob.ctrl_cost = 1
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    cost = pi.rollout_cost(dp, dm)
    ref_cost, ref_u = oracle.iteration(prob, model)
    assert np.max(np.abs(cost.cpu().numpy() - ref_cost)) <= 1e-10 * np.abs(ref_cost).max()
    pi.update(dp, cost)
    assert np.max(np.abs(dp.u_nom.cpu().numpy() - ref_u)) <= 1e-10


@pytest.mark.parametrize("M", [0, 1, 4, 8, 16, 32])
def test_rollout_paper_shapes_full(M):
    # the paper's timing shapes at full size (1000 rollouts x 50 steps, M
    # sub-rollouts each) in the launch the timing uses; every rollout against
    # the oracle
    prob, model = synth.paper_shape(M=M)
    assert (prob.K, prob.T) == (1000, 50)
    prob.u_nom = np.random.default_rng(100 + M).normal(0.0, 0.3, prob.u_nom.shape).astype(F32)
    cost = pi.rollout_cost(pi.DeviceProblem(prob), pi.DeviceModel(model)).cpu().numpy()
    ref = oracle.rollout_cost(prob, model)
    r, flips = cost_check(cost, ref, prob, 1e-4)
    print("paper shape M=%d: max S rel %.2e, flips %d" % (M, r, flips))


def test_hybrid_fp64_iteration_and_shift():
    prob, model = synth.paper_shape(M=2, K=64, T=15, dtype=F64)
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    cost = pi.rollout_cost(dp, dm).cpu().numpy()
    assert np.max(np.abs(cost - oracle.rollout_cost(prob, model))) <= 1e-10 * np.abs(cost).max()
    pi.iteration(dp, dm)
    pi.rh_shift(dp, dm)
    x, u, it = oracle.rh_loop(prob, model, steps=1, iterations=1)
    assert int(dp.iter.item()) == it
    assert np.max(np.abs(dp.u_nom.cpu().numpy() - u)) <= 1e-10
    assert np.max(np.abs(dp.x0.cpu().numpy() - x)) <= 1e-10


def test_hybrid_adjoint_is_refused():
    prob, model = synth.paper_shape(K=4, T=3)
    with pytest.raises(pi.PiError):
        pi.rollout_adjoint(pi.DeviceProblem(prob), pi.DeviceModel(model))


@pytest.mark.parametrize("dtype", [F32, F64])
def test_rollout_direct_both_grids(dtype):
    # the direct kernels: 16 lanes per sub-rollout below 8192 sub-rollouts, one
    # lane each above; both against the oracle on sampled rollouts
    for K in (300, 9000):
        prob, model = synth.tiny_problem(17, dyn=DYN_QUAD12, L=[9, 3, 40, 2, 17, 5], R=3, K=K, T=5,
                                         M=1, dtype=dtype, n_obs=4, obs_kind=OBS_SMOOTH)
        dp = pi.DeviceProblem(prob, variant=pi.PI_VARIANT_DIRECT)
        cost = pi.rollout_cost(dp, pi.DeviceModel(model)).cpu().numpy()
        rows = list(range(0, 40)) + list(range(K - 40, K))
        ref = np.concatenate([oracle.rollout_cost(prob, model, k_range=(0, 40)),
                              oracle.rollout_cost(prob, model, k_range=(K - 40, K))])
        tol = 1e-10 if dtype == F64 else 1e-4
        assert nrel(cost[rows], ref) <= tol


def test_rollout_edge_sizes():
    for K, T in ((1, 1), (1, 5), (17, 1)):
        prob, model = synth.tiny_problem(13, dyn=DYN_QUAD12, L=3, R=2, K=K, T=T, M=1, dtype=F32)
        cost = pi.rollout_cost(pi.DeviceProblem(prob), pi.DeviceModel(model)).cpu().numpy()
        ref = oracle.rollout_cost(prob, model)
        assert cost.shape == (K, T)
        cost_check(cost, ref, prob, 1e-4)


@pytest.fixture(scope="module")
def config1_oracle():
    """The oracle's per-step costs of all 2048 x 100 rollouts of the
    quadrotor workload (6 x 256 models) and its end-to-end update."""
    prob, model, _ = synth.config(1)
    cost, u = oracle.iteration(prob, model)
    return prob, model, cost, u


@pytest.mark.parametrize("variant,split,spw", [(pi.PI_VARIANT_AUTO, 0, 0), (pi.PI_VARIANT_AUTO, 1, 0),
                                               (BF3, 0, 0), (BF3, 1, 32), (BF3, 1, 128), (HF2, 0, 0), (HF2, 1, 32),
                                               (HF2, 1, 128)])
def test_rollout_config1_full_launch_all_rows(variant, split, spw, config1_oracle):
    # the benchmarked 2048-rollout launch (split 0: 128 tiles of 16 rollouts
    # on 256 paired workgroups) and the one-workgroup-per-tile form, with
    # float32 products and in three bf16 pieces: every rollout's S_k, and
    # every per-step cost elementwise
    prob, model, ref, _ = config1_oracle
    dp = pi.DeviceProblem(prob, variant=variant, tile_split=split, tile_samples=spw)
    cost = pi.rollout_cost(dp, pi.DeviceModel(model)).cpu().numpy()
    assert cost.shape == (2048, 100) and np.all(np.isfinite(cost))
    r, flips = cost_check(cost, ref, prob, 1e-4)
    keep = np.abs(cost - ref).max(1) <= 0.25 * prob.dt * prob.obs_penalty
    ew = c16(cost[keep], ref[keep])
    print("config 1 all rows (variant %d, split %d, spw %d): max S rel %.2e, per-step elementwise %.2e, flips %d"
          % (variant, split, spw, r, ew, flips))
    assert ew <= 1e-4


@pytest.mark.parametrize("variant", [pi.PI_VARIANT_AUTO, BF3, HF2])
def test_iteration_config1_fp32_end_to_end(variant, config1_oracle):
    # rollouts and update on the GPU in FP32 against the oracle's FP64
    # iteration; an error dS in the costs moves the update by about
    # max_k |dS_k| spread(eps) / lambda
    prob, model, ref_cost, ref_u = config1_oracle
    dp, dm = pi.DeviceProblem(prob, variant=variant), pi.DeviceModel(model)
    cost = pi.rollout_cost(dp, dm)
    pi.update(dp, cost)
    du = np.max(np.abs(dp.u_nom.cpu().numpy() - ref_u))
    dS = np.max(np.abs(cost.cpu().numpy().astype(np.float64).sum(1) - ref_cost.sum(1)))
    print("config 1 end-to-end FP32 update: max |du| %.2e (max |dS| %.2e)" % (du, dS))
    assert int(dp.iter.item()) == 1
    assert du <= 1e-4


@pytest.mark.parametrize("variant,spw", [(pi.PI_VARIANT_AUTO, 0), (BF3, 32), (BF3, 128), (HF2, 0), (HF2, 32)])
def test_rollout_config2_full_launch_sampled_rows(variant, spw):
    # 65536 rollouts over T = 200 against 6 x 1024 models: 4096 one-workgroup
    # tiles, two workgroups per compute unit (or, bf16 pieces, 2048 tiles of
    # 32 rows, or 512 shared-tile workgroups of 128); sampled rows at both
    # ends and across tile boundaries
    prob, model, _ = synth.config(2)
    dp, dm = pi.DeviceProblem(prob, variant=variant, tile_samples=spw), pi.DeviceModel(model)
    assert pi.rollout_describe(dp, dm)["tile_split"] == 1
    cost = pi.rollout_cost(dp, dm).cpu().numpy()
    assert cost.shape == (65536, 200) and np.all(np.isfinite(cost))
    # 16 runs of 16 rows spread over the whole grid, the run starts offset
    # from the tile boundaries so that most runs straddle two tiles
    starts = [int(a) for a in np.linspace(0, 65536 - 16, 16).round()]
    starts = [a - (a % 16) + (8 if 0 < a < 65520 else 0) for a in starts]
    rows = [a + i for a in starts for i in range(16)]
    assert len(set(rows)) == 256
    ref = np.concatenate([oracle.rollout_cost(prob, model, k_range=(a, a + 16)) for a in starts])
    r, flips = cost_check(cost[rows], ref, prob, 1e-4)
    keep = np.abs(cost[rows] - ref).max(1) <= 0.25 * prob.dt * prob.obs_penalty
    ew = c16(cost[rows][keep], ref[keep])
    print("config 2 sampled rows (256, variant %d, spw %d): max S rel %.2e, per-step elementwise %.2e, flips %d"
          % (variant, spw, r, ew, flips))
    assert ew <= 1e-4


def test_prefolded_model_gives_identical_results():
    # pi_model_fold once, then every entry point reads the folded buffer: the
    # same kernels on the same folded values, so results are bitwise equal
    prob, model, _ = synth.config(1, K=300, T=12)
    dm, df = pi.DeviceModel(model), pi.DeviceModel(model).fold()
    Z = torch.from_numpy(np.random.default_rng(8).uniform(-1, 1, (77, 16)).astype(F32)).cuda()
    for variant in (pi.PI_VARIANT_DIRECT, pi.PI_VARIANT_MFMA):
        a, b = pi.lwpr_predict(dm, Z, variant=variant), pi.lwpr_predict(df, Z, variant=variant)
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    for split in (1, 2):
        dp = pi.DeviceProblem(prob, tile_split=split)
        assert torch.equal(pi.rollout_cost(dp, dm), pi.rollout_cost(dp, df))
    d1, d2 = pi.DeviceProblem(prob), pi.DeviceProblem(prob)
    pi.rh_shift(d1, dm)
    pi.rh_shift(d2, df)
    assert torch.equal(d1.x0, d2.x0) and torch.equal(d1.u_nom, d2.u_nom)
    p64, _, _ = synth.config(0)
    m64 = synth.config(0)[1]
    a = pi.rollout_cost(pi.DeviceProblem(p64), pi.DeviceModel(m64))
    b = pi.rollout_cost(pi.DeviceProblem(p64), pi.DeviceModel(m64).fold())
    assert torch.equal(a, b)


def test_rollout_describe_reports_the_launch():
    prob, model, _ = synth.config(1)
    dm = pi.DeviceModel(model)
    d = pi.rollout_describe(pi.DeviceProblem(prob), dm)
    # 128 tiles of 16 rollouts leave compute units idle: pairs of workgroups,
    # with 8 waves when the 256 workgroups fit one per compute unit
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    assert d == {"variant": "mfma", "tile_samples": 16, "tile_waves": 8 if n_cu >= 256 else 4,
                 "tile_split": 2, "kernel": "rollout_pair_kernel"}
    assert pi.rollout_describe(pi.DeviceProblem(prob, tile_waves=4), dm)["tile_waves"] == 4
    assert pi.rollout_describe(pi.DeviceProblem(prob, tile_split=1), dm)["tile_split"] == 1
    big, _, _ = synth.config(1, K=65536, T=2)
    db = pi.rollout_describe(pi.DeviceProblem(big), dm)
    assert db["tile_split"] == 1 and db["tile_waves"] == 4
    p64 = pi.DeviceProblem(prob, dtype=torch.float64)
    assert pi.rollout_describe(p64, pi.DeviceModel(model, dtype=torch.float64))["kernel"] == \
        "rollout_direct_kernel"


def test_bf16x3_describe_and_refusals():
    # the three-piece bf16 form: reported as such; refused (PI_ERR_UNSUPPORTED)
    # for 8 waves with 32-row tiles, float64, other plants and d != 16, and
    # by the prediction entry point
    prob, model, _ = synth.config(1)
    dm = pi.DeviceModel(model)
    d = pi.rollout_describe(pi.DeviceProblem(prob, variant=BF3, tile_samples=32, tile_split=1), dm)
    assert d == {"variant": "mfma-bf16x3", "tile_samples": 32, "tile_waves": 4, "tile_split": 1,
                 "kernel": "rollout_mfma_kernel"}
    assert pi.rollout_describe(pi.DeviceProblem(prob, variant=BF3), dm)["kernel"] == "rollout_pair_kernel"
    d = pi.rollout_describe(pi.DeviceProblem(prob, variant=BF3, tile_samples=128, tile_split=1), dm)
    assert d["tile_samples"] == 128 and d["tile_waves"] == 4 and d["kernel"] == "rollout_mfma_kernel"
    with pytest.raises(pi.PiError) as e:      # 128-row tiles: the bf16 form only
        pi.rollout_cost(pi.DeviceProblem(prob, variant=pi.PI_VARIANT_MFMA, tile_samples=128), dm)
    assert "tile_samples=128 outside [0,32]" in str(e.value)
    d = pi.rollout_describe(pi.DeviceProblem(prob, variant=BF3, tile_samples=128, tile_waves=8), dm)
    assert d["tile_samples"] == 128 and d["tile_waves"] == 8 and d["tile_split"] == 1
    # the fp16 form: the bf16 form's launches; by default 16-row tiles on
    # pairs here, the shared tile (128 rows, 8 waves) from 32768 rollouts on
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    d = pi.rollout_describe(pi.DeviceProblem(prob, variant=HF2), dm)
    assert d == {"variant": "mfma-f16x2", "tile_samples": 16, "tile_waves": 8 if n_cu >= 256 else 4,
                 "tile_split": 2, "kernel": "rollout_pair_kernel"}
    big, _, _ = synth.config(1, K=32768, T=2)
    for v in (BF3, HF2):
        d = pi.rollout_describe(pi.DeviceProblem(big, variant=v), dm)
        assert (d["tile_samples"], d["tile_waves"], d["tile_split"]) == (128, 8, 1)
    with pytest.raises(pi.PiError) as e:
        pi.rollout_describe(pi.DeviceProblem(prob, variant=HF2, tile_samples=32, tile_waves=8), dm)
    assert e.value.status == 7 and "f16x2" in str(e.value)
    refused = [(pi.DeviceProblem(prob, variant=BF3, tile_samples=32, tile_waves=8, tile_split=1), dm),
               (pi.DeviceProblem(prob, variant=BF3, dtype=torch.float64),
                pi.DeviceModel(model, dtype=torch.float64))]
    pm, pmodel = synth.tiny_problem(5, dyn=DYN_POINTMASS2D, L=4, R=2, K=16, T=3, M=1, dtype=F32)
    refused.append((pi.DeviceProblem(pm, variant=BF3), pi.DeviceModel(pmodel)))
    for dp, m in refused:
        with pytest.raises(pi.PiError) as e:
            pi.rollout_cost(dp, m)
        assert e.value.status == 7
    for v in (BF3, HF2):
        with pytest.raises(pi.PiError) as e:
            pi.lwpr_predict(dm, torch.zeros((4, 16), dtype=torch.float32, device="cuda"), variant=v)
        assert e.value.status == 7


@pytest.mark.parametrize("variant,split,spw", [(pi.PI_VARIANT_AUTO, 1, 0), (pi.PI_VARIANT_AUTO, 2, 0),
                                               (BF3, 2, 0), (BF3, 1, 32), (BF3, 1, 128), (HF2, 2, 0), (HF2, 1, 128)])
def test_rollout_bitwise_repeatable(variant, split, spw):
    prob, model, _ = synth.config(1, K=512, T=20)
    dp = pi.DeviceProblem(prob, variant=variant, tile_split=split, tile_samples=spw)
    dm = pi.DeviceModel(model)
    a = pi.rollout_cost(dp, dm).clone()
    for _ in range(3):
        assert torch.equal(a, pi.rollout_cost(dp, dm))


# ------------------------------------------------------------------- update

@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("weighting", [0, W_TRAJECTORY])
@pytest.mark.parametrize("K", [1, 333, 4100])
def test_update_teacher_forced(dtype, weighting, K):
    prob, _ = synth.tiny_problem(14, dyn=DYN_QUAD12, K=K, T=23, dtype=dtype)
    prob.weighting = weighting
    prob.lam = 0.3
    cost = np.random.default_rng(K).uniform(0.0, 1.0, (K, prob.T)).astype(dtype)
    dp = pi.DeviceProblem(prob)
    dp.iter.fill_(4)
    u, W = pi.update(dp, torch.from_numpy(cost).cuda(), weights=True)
    ou, oW = oracle.update(prob, cost, it=4, weights=True)
    assert int(dp.iter.item()) == 5
    tol = 1e-12 if dtype == F64 else 1e-4
    assert np.max(np.abs(u.cpu().numpy() - ou)) <= tol
    assert np.max(np.abs(W.cpu().numpy() - oW)) <= 1e-12


@pytest.mark.parametrize("cfg", [1, 2])
def test_update_teacher_forced_full_size(cfg):
    # the benchmarked update sizes (2048 x 100 and 65536 x 200) from seeded costs
    prob, _, _ = synth.config(cfg)
    cost = np.random.default_rng(cfg).uniform(0.0, 1.0, (prob.K, prob.T)).astype(F32)
    dp = pi.DeviceProblem(prob)
    u, W = pi.update(dp, torch.from_numpy(cost).cuda(), weights=True)
    ou, oW = oracle.update(prob, cost, it=0, weights=True)
    assert np.max(np.abs(u.cpu().numpy() - ou)) <= 1e-4
    assert np.max(np.abs(W.cpu().numpy() - oW)) <= 1e-12


def test_iteration_fp64_end_to_end():
    prob, model, _ = synth.config(0)
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    pi.iteration(dp, dm)
    _, ou = oracle.iteration(prob, model)
    assert np.max(np.abs(dp.u_nom.cpu().numpy() - ou)) <= 1e-10


# ------------------------------------------------------------------ RH shift

@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("dyn", [DYN_POINTMASS2D, DYN_QUAD12])
def test_rh_shift_matches_oracle(dtype, dyn):
    prob, model = synth.tiny_problem(15, dyn=dyn, L=[30, 40, 7, 9, 12, 3][:(2 if dyn == 0 else 6)],
                                     R=2, K=4, T=300, dtype=dtype)
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    dp.iter.fill_(5)
    pi.rh_shift(dp, dm)
    ox, ou = oracle.rh_shift(prob, model, prob.x0, prob.u_nom, 5)
    assert int(dp.iter.item()) == 5
    assert np.array_equal(dp.u_nom.cpu().numpy(), ou.astype(dtype))
    tol = 1e-12 if dtype == F64 else 1e-6
    assert np.max(np.abs(dp.x0.cpu().numpy() - ox)) <= tol * max(1.0, np.abs(ox).max())
