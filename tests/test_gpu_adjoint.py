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


@pytest.mark.parametrize("dyn", [DYN_POINTMASS2D, DYN_QUAD12])
def test_adjoint_fp32_matches_oracle(dyn):
    prob, model = _case(dyn, 1, np.float32, K=40, T=16)
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


def test_adjoint_full_size_directional_derivative():
    # the adjoint workload (K = 8192, T = 400, checkpoints every 20 steps) with
    # the smooth obstacle cost: g_u . v against central differences of J from
    # the forward rollout kernel
    prob, model, _ = synth.config(4, obs_kind=OBS_SMOOTH)
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    J, gu, gc, gD = pi.rollout_adjoint(dp, dm, ckpt_every=20)
    assert np.all(np.isfinite(gu.cpu().numpy())) and np.all(np.isfinite(gD.cpu().numpy()))
    cost = pi.rollout_cost(dp, dm)
    Jf = cost.double().sum(1).mean().item()
    assert abs(J.item() - Jf) <= 2e-4 * abs(Jf)
    v = torch.zeros_like(dp.u_nom)
    v[:40] = torch.randn(40, 4, generator=torch.Generator().manual_seed(0)).to(v)
    h = 2e-2
    u0 = dp.u_nom.clone()
    Js = []
    for sgn in (1.0, -1.0):
        dp.u_nom.copy_(u0 + sgn * h * v)
        Js.append(pi.rollout_cost(dp, dm).double().sum(1).mean().item())
    dp.u_nom.copy_(u0)
    fd = (Js[0] - Js[1]) / (2 * h)
    an = float((gu.double() * v.double()).sum().item())
    assert abs(fd - an) <= 0.05 * abs(an) + 1e-3 * abs(Jf), (fd, an)
