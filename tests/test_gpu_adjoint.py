"""Adjoint of the expected rollout cost on the GPU (noise held fixed):
FP64 against the oracle's hand-derived adjoint (strict), FP32 to tolerance,
autograd wiring, and a directional-derivative check at the full adjoint
workload size."""
import numpy as np
import pytest

import oracle
import synth
from synth import DYN_POINTMASS2D, DYN_QUAD12, OBS_SMOOTH

torch = pytest.importorskip("torch")
pi = pytest.importorskip("paper_1503_00330_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    yield
    torch.cuda.synchronize()


def nrel(g, o):
    g, o = np.asarray(g, np.float64).ravel(), np.asarray(o, np.float64).ravel()
    return float(np.abs(g - o).max() / max(np.abs(o).max(), 1e-300))


def _case(dyn, M, dtype, seed=30, K=9, T=11, L=None, ckpt=0):
    L = L or ([5, 7] if dyn == DYN_POINTMASS2D else [5, 3, 7, 2, 6, 4])
    prob, model = synth.tiny_problem(seed, dyn=dyn, L=L, R=2, K=K, T=T, M=M, dtype=dtype, n_obs=3,
                                     obs_kind=OBS_SMOOTH)
    prob.obs[:, :2] = prob.x0[:2] + np.array([0.12, -0.1])   # obstacles near the path
    return prob, model


@pytest.mark.parametrize("dyn", [DYN_POINTMASS2D, DYN_QUAD12])
@pytest.mark.parametrize("M", [0, 1, 2])
@pytest.mark.parametrize("ckpt", [0, 1, 4, 11])
def test_adjoint_fp64_matches_oracle(dyn, M, ckpt):
    prob, model = _case(dyn, M, np.float64)
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    J, gu, gc, gD = pi.rollout_adjoint(dp, dm, ckpt_every=ckpt)
    oJ, ogu, ogc, ogD = oracle.adjoint(prob, model)
    assert abs(J.item() - oJ) <= 1e-12 * abs(oJ)
    for g, o in ((gu, ogu), (gc, ogc), (gD, ogD)):
        assert nrel(g.cpu().numpy(), o) <= 1e-10


# float32: the matrix-core forward that keeps every step (variant AUTO) and the
# checkpointed direct forward (variant DIRECT)
@pytest.mark.parametrize("variant", [pi.PI_VARIANT_AUTO, pi.PI_VARIANT_DIRECT])
@pytest.mark.parametrize("M", [0, 1, 3])
@pytest.mark.parametrize("dyn", [DYN_POINTMASS2D, DYN_QUAD12])
def test_adjoint_fp32_matches_oracle(dyn, M, variant):
    prob, model = _case(dyn, M, np.float32, K=40, T=16)
    dp, dm = pi.DeviceProblem(prob, variant=variant), pi.DeviceModel(model)
    J, gu, gc, gD = pi.rollout_adjoint(dp, dm)
    oJ, ogu, ogc, ogD = oracle.adjoint(prob, model)
    assert abs(J.item() - oJ) <= 1e-5 * abs(oJ)
    for g, o in ((gu, ogu), (gc, ogc), (gD, ogD)):
        assert nrel(g.cpu().numpy(), o) <= 1e-4


@pytest.mark.parametrize("ckpt", [1, 5, 7, 16])
def test_adjoint_fp32_matrix_core_checkpoints(ckpt):
    # the matrix-core adjoint recomputes every segment of `ckpt` steps from
    # its checkpoints (ragged last segment at 5 and 7; one segment at 16)
    prob, model = _case(DYN_QUAD12, 1, np.float32, K=40, T=16)
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    J, gu, gc, gD = pi.rollout_adjoint(dp, dm, ckpt_every=ckpt)
    oJ, ogu, ogc, ogD = oracle.adjoint(prob, model)
    assert abs(J.item() - oJ) <= 1e-5 * abs(oJ)
    for g, o in ((gu, ogu), (gc, ogc), (gD, ogD)):
        assert nrel(g.cpu().numpy(), o) <= 1e-4


@pytest.mark.parametrize("variant", [pi.PI_VARIANT_MFMA_F16X2, pi.PI_VARIANT_MFMA_BF16X3])
@pytest.mark.parametrize("M,ckpt,K,T", [(0, 0, 40, 16), (1, 5, 40, 16), (3, 16, 40, 16), (1, 1, 40, 16),
                                        (1, 3, 4096, 8)])
def test_adjoint_pieces_forward_matches_oracle(variant, M, ckpt, K, T):
    # the forward and the segment recomputes in the fp16 (bf16) pieces, the
    # reverse sweep and the parameter pass in float32 with the forward's
    # traced anchors and normalisers (4096 rollouts: the 32-row tiles)
    prob, model = _case(DYN_QUAD12, M, np.float32, K=K, T=T)
    dp, dm = pi.DeviceProblem(prob, variant=variant), pi.DeviceModel(model)
    J, gu, gc, gD = pi.rollout_adjoint(dp, dm, ckpt_every=ckpt)
    oJ, ogu, ogc, ogD = oracle.adjoint(prob, model)
    assert abs(J.item() - oJ) <= 1e-5 * abs(oJ)
    for g, o in ((gu, ogu), (gc, ogc), (gD, ogD)):
        assert nrel(g.cpu().numpy(), o) <= 1e-4


def test_adjoint_seed_scales_the_gradients():
    # gJ seeds the reverse pass: gradients of gJ * J, J itself unscaled
    prob, model = _case(DYN_QUAD12, 1, np.float64, K=12, T=9)
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    a = [t.clone() for t in pi.rollout_adjoint(dp, dm)]
    b = pi.rollout_adjoint(dp, dm, gJ=torch.tensor([-2.5], dtype=torch.float64))
    assert torch.equal(a[0], b[0])
    for x, y in zip(a[1:], b[1:]):
        assert torch.allclose(-2.5 * x, y, rtol=1e-15, atol=0)
    p32, m32 = _case(DYN_QUAD12, 1, np.float32, K=40, T=16)
    d32, dm32 = pi.DeviceProblem(p32), pi.DeviceModel(m32)
    a = [t.clone() for t in pi.rollout_adjoint(d32, dm32)]
    b = pi.rollout_adjoint(d32, dm32, gJ=torch.tensor([4.0], dtype=torch.float64))
    for x, y in zip(a[1:], b[1:]):
        assert torch.equal(4.0 * x, y)


def test_adjoint_fp32_odd_tile_count():
    # 7 model tiles: in the matrix-core parameter pass one wave holds a valid
    # and an absent tile (its prefetch must return to the valid one)
    prob, model = _case(DYN_QUAD12, 1, np.float32, K=37, T=13, L=[5, 3, 7, 2, 6, 20])
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    J, gu, gc, gD = pi.rollout_adjoint(dp, dm)
    oJ, ogu, ogc, ogD = oracle.adjoint(prob, model)
    assert abs(J.item() - oJ) <= 1e-5 * abs(oJ)
    for g, o in ((gu, ogu), (gc, ogc), (gD, ogD)):
        assert nrel(g.cpu().numpy(), o) <= 1e-4


def test_adjoint_J_matches_forward_rollout():
    prob, model = _case(DYN_QUAD12, 1, np.float64, K=20, T=9)
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    J, *_ = pi.rollout_adjoint(dp, dm)
    cost = pi.rollout_cost(dp, dm)
    assert abs(J.item() - cost.sum(1).mean().item()) <= 1e-12 * abs(J.item())


def test_autograd_function():
    from paper_1503_00330_amd.autograd import PI2RHAdjoint
    prob, model = _case(DYN_QUAD12, 1, np.float64, K=6, T=7)
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    u = dp.u_nom.clone().requires_grad_(True)
    c = dm.centre.clone().requires_grad_(True)
    D = dm.metric.clone().requires_grad_(True)
    J = PI2RHAdjoint.apply(u, c, D, dp, dm)
    (2.0 * J).backward()
    _, ogu, ogc, ogD = oracle.adjoint(prob, model)
    assert nrel(u.grad.cpu().numpy(), 2 * ogu) <= 1e-10
    assert nrel(c.grad.cpu().numpy(), 2 * ogc) <= 1e-10
    assert nrel(D.grad.cpu().numpy(), 2 * ogD) <= 1e-10


def test_adjoint_repeatable():
    prob, model = _case(DYN_QUAD12, 1, np.float32, K=50, T=12)
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    a = [t.clone() for t in pi.rollout_adjoint(dp, dm)]
    b = pi.rollout_adjoint(dp, dm)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_adjoint_full_batch_directional_derivative():
    # The adjoint workload's batch (K = 8192 rollouts, 6 x 256 models) over a
    # 100-step horizon, where the trajectories stay near the models' support
    # and J is smooth in u: FP64 g_u . v against central differences of the
    # FP64 forward kernel (h = 1e-5; truncation O(h^2) and rounding both well
    # under 1e-8 relative), and the FP32 gradients against the FP64 ones.
    prob, model, _ = synth.config(4, obs_kind=OBS_SMOOTH, T=100)
    dp = pi.DeviceProblem(prob, dtype=torch.float64)
    dm = pi.DeviceModel(model, dtype=torch.float64)
    J, gu, gc, gD = pi.rollout_adjoint(dp, dm)
    v = torch.from_numpy(np.random.default_rng(0).standard_normal(prob.u_nom.shape)).to(dp.u_nom)
    h = 1e-5
    u0 = dp.u_nom.clone()
    Js = []
    for sgn in (1.0, -1.0):
        dp.u_nom.copy_(u0 + sgn * h * v)
        Js.append(pi.rollout_cost(dp, dm).sum(1).mean().item())
    dp.u_nom.copy_(u0)
    fd = (Js[0] - Js[1]) / (2 * h)
    an = float((gu * v).sum().item())
    assert abs(fd - an) <= 1e-8 * abs(an), (fd, an)
    J32, gu32, gc32, gD32 = pi.rollout_adjoint(pi.DeviceProblem(prob), pi.DeviceModel(model))
    for g32, g64 in ((gu32, gu), (gc32, gc), (gD32, gD)):
        assert nrel(g32.cpu().numpy(), g64.cpu().numpy()) <= 1e-5
    assert abs(J32.item() - J.item()) <= 1e-6 * abs(J.item())


def test_adjoint_full_size_fp64():
    # The adjoint workload itself (K = 8192, T = 400, checkpoints every 20
    # steps, smooth obstacle cost).  Over 400 steps many sampled trajectories
    # leave the models' support; far from every centre the weights switch
    # between local models over distances of ~1e-5 and derivatives with
    # respect to early controls grow like exp(lambda (T - t)) (mean
    # directional derivatives of 1e17), beyond what finite differences resolve
    # even in FP64 (the oracle's own differences do not converge at 256
    # rollouts).  What holds at this size: finite gradients, J of the adjoint's
    # forward sweep against the forward kernel (two FP64 summation orders whose
    # rounding the chaotic rollouts amplify to ~1e-5), and the gradients of the
    # first 16 rollouts -- whose differences converge (5e-6 at h = 1e-7 on the
    # last 40 controls) -- against the FP64 oracle's adjoint (4e-7 measured,
    # the rounding of 400 chaotic steps).
    prob, model, _ = synth.config(4, obs_kind=OBS_SMOOTH)
    dp = pi.DeviceProblem(prob, dtype=torch.float64)
    dm = pi.DeviceModel(model, dtype=torch.float64)
    J, gu, gc, gD = pi.rollout_adjoint(dp, dm, ckpt_every=20)
    for g in (gu, gc, gD):
        assert torch.isfinite(g).all()
    Jf = pi.rollout_cost(dp, dm).sum(1).mean().item()
    assert abs(J.item() - Jf) <= 1e-4 * abs(Jf)
    p16, _, _ = synth.config(4, obs_kind=OBS_SMOOTH, K=16)
    J16, gu16, gc16, gD16 = pi.rollout_adjoint(pi.DeviceProblem(p16, dtype=torch.float64), dm, ckpt_every=20)
    oJ, ogu, ogc, ogD = oracle.adjoint(p16, model)
    assert abs(J16.item() - oJ) <= 1e-10 * abs(oJ)
    for g, o in ((gu16, ogu), (gc16, ogc), (gD16, ogD)):
        assert nrel(g.cpu().numpy(), o) <= 1e-5


def _x0_envelope(prob, model, rel=2.0 ** -24):
    """FP64 sensitivity of the rollout costs to one FP32 unit roundoff in the
    start position: per-rollout relative cost changes (max over the two signs)
    and the change of the mean cost, with the unperturbed costs."""
    m64 = pi.DeviceModel(model, dtype=torch.float64)
    S = pi.rollout_cost(pi.DeviceProblem(prob, dtype=torch.float64), m64).sum(1).cpu().numpy()
    env, envJ = np.zeros_like(S), 0.0
    for sgn in (1.0, -1.0):
        dp = pi.DeviceProblem(prob, dtype=torch.float64)
        dp.x0[:3] *= 1.0 + sgn * rel
        Sp = pi.rollout_cost(dp, m64).sum(1).cpu().numpy()
        env = np.maximum(env, np.abs(Sp - S) / np.abs(S))
        envJ = max(envJ, abs(Sp.mean() - S.mean()) / abs(S.mean()))
    return S, env, envJ


def test_adjoint_full_size_fp32():
    # The adjoint workload in FP32 (K = 8192, T = 400, checkpoints every 20,
    # smooth obstacles).  Over 400 steps many trajectories leave the models'
    # support; the FP64 path itself then moves its per-rollout costs by up to
    # O(1) under a single FP32 unit roundoff in the start position, while FP32
    # rounds at every step.  So FP32 is held to that envelope, measured here in
    # FP64: the mean cost (J of the adjoint's own forward) within 10x the
    # envelope's change of the mean, the non-chaotic majority of rollouts
    # (median) within the 1e-4 cost tolerance, and the 90th percentile within
    # 10x the envelope's.  Gradients must be finite (FP32 gradients are
    # compared with FP64 where the trajectories stay well-conditioned: T <= 200).
    prob, model, _ = synth.config(4, obs_kind=OBS_SMOOTH)
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    J, gu, gc, gD = pi.rollout_adjoint(dp, dm, ckpt_every=20)
    for g in (gu, gc, gD):
        assert torch.isfinite(g).all()
    S64, env, envJ = _x0_envelope(prob, model)
    Jrel = abs(J.item() - S64.mean()) / abs(S64.mean())
    S32 = pi.rollout_cost(dp, dm).double().sum(1).cpu().numpy()
    e = np.abs(S32 - S64) / np.abs(S64)
    print("T=400 FP32: J rel %.2e (envelope %.2e); per-rollout median %.2e, p90 %.2e (envelope p90 %.2e)"
          % (Jrel, envJ, np.median(e), np.percentile(e, 90), np.percentile(env, 90)))
    assert Jrel <= 10 * envJ
    assert np.median(e) <= 1e-4
    assert np.percentile(e, 90) <= 10 * np.percentile(env, 90)


@pytest.mark.parametrize("variant", [pi.PI_VARIANT_AUTO, pi.PI_VARIANT_DIRECT, pi.PI_VARIANT_MFMA_F16X2])
def test_adjoint_fp32_gradients_over_200_steps(variant):
    # the adjoint workload's batch over 200 steps, where trajectories stay near
    # the models' support: FP32 gradients (matrix-core and direct) against the
    # FP64 ones at full size (2.5e-4 measured for both: the sensitivity of the
    # map grows like exp(0.04 T), 2.4e-7 at T = 100), and per rollout on the
    # first 16 rollouts
    for K in (8192, 16):
        prob, model, _ = synth.config(4, obs_kind=OBS_SMOOTH, T=200, K=K)
        r64 = pi.rollout_adjoint(pi.DeviceProblem(prob, dtype=torch.float64),
                                 pi.DeviceModel(model, dtype=torch.float64), ckpt_every=20)
        r32 = pi.rollout_adjoint(pi.DeviceProblem(prob, variant=variant), pi.DeviceModel(model), ckpt_every=20)
        assert abs(r32[0].item() - r64[0].item()) <= 1e-6 * abs(r64[0].item())
        errs = [nrel(a.cpu().numpy(), b.cpu().numpy()) for a, b in zip(r32[1:], r64[1:])]
        print("T=200 K=%d variant %d: gradient errors %s" % (K, variant, ["%.2e" % x for x in errs]))
        assert max(errs) <= 1e-3
