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


# FP32 against FP64 for the mean cost at the 400-step adjoint workload, where
# rounding differences grow chaotically (2.8e-3 measured)
FP32_LONG_J_TOL = 1e-2


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


def test_adjoint_full_size_fp32():
    # the same workload in FP32: every gradient finite (the variance of
    # Eq. (1) is clamped against rounding), and J consistent with the FP64
    # forward kernel to the spread FP32 trajectories reach over 400 chaotic
    # steps (per-rollout cost differences: median 3e-5, 99th percentile 0.12;
    # mean cost 2.8e-3 measured)
    prob, model, _ = synth.config(4, obs_kind=OBS_SMOOTH)
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    J, gu, gc, gD = pi.rollout_adjoint(dp, dm, ckpt_every=20)
    for g in (gu, gc, gD):
        assert torch.isfinite(g).all()
    d64 = pi.DeviceProblem(prob, dtype=torch.float64)
    J64 = pi.rollout_cost(d64, pi.DeviceModel(model, dtype=torch.float64)).sum(1).mean().item()
    assert abs(J.item() - J64) <= FP32_LONG_J_TOL * abs(J64)
