"""The allocation-free rollout entry point (pi_rollout_cost_noalloc): the same
costs as pi_rollout_cost with a caller workspace, bit for bit, on consecutive
calls of different sizes sharing the library's static scratch."""
import ctypes as C

import numpy as np
import pytest

import synth
from synth import DYN_POINTMASS2D, DYN_QUAD12, DYN_QUAD_HYBRID

torch = pytest.importorskip("torch")
pi = pytest.importorskip("paper_1503_00330_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    yield
    torch.cuda.synchronize()


def _noalloc(dp, dm):
    """pi_rollout_cost_noalloc through the C ABI into a NaN-filled cost array."""
    cost = torch.full((dp.K, dp.T), float("nan"), dtype=dp.dtype, device="cuda")
    ps, ms = dp.struct(), dm.struct()
    st = pi.load().pi_rollout_cost_noalloc(C.byref(ps), C.byref(ms), dp.x0.data_ptr(),
                                            dp.u_nom.data_ptr(), dp.iter.data_ptr(), cost.data_ptr(),
                                            torch.cuda.current_stream().cuda_stream)
    assert st == 0, pi.last_error()
    return cost


def _with_workspace(dp, dm):
    return pi.rollout_cost(dp, dm).clone()


def _pair(first, second):
    """Two noalloc calls in a row (the second smaller), each against the
    workspace entry point on the same inputs."""
    a = _noalloc(*first)
    b = _noalloc(*second)
    torch.cuda.synchronize()
    ra, rb = _with_workspace(*first), _with_workspace(*second)
    assert torch.equal(a, ra)
    assert torch.equal(b, rb)
    assert torch.isfinite(a).all() and torch.isfinite(b).all()


def test_noalloc_quadrotor_then_smaller():
    # 2048 x 100 quadrotor rollouts over 6 x 256 models (paired workgroups,
    # model folded into the scratch), then a smaller ragged problem with 3
    # sub-rollouts (sub-rollout costs in the scratch over the first call's)
    prob, model, _ = synth.config(1)
    first = (pi.DeviceProblem(prob), pi.DeviceModel(model))
    assert pi.rollout_describe(*first)["tile_split"] == 2
    p2, m2 = synth.tiny_problem(5, dyn=DYN_QUAD12, L=[19, 16, 33, 8, 16, 17], R=4, K=301, T=37, M=3,
                                dtype=np.float32, n_obs=7)
    second = (pi.DeviceProblem(p2), pi.DeviceModel(m2))
    _pair(first, second)


def test_noalloc_folded_models_and_other_families():
    # a pre-folded model (no fold region), then the hybrid model with the
    # control terms of the cost-to-go, then a float64 point mass on the direct
    # kernels
    prob, model, _ = synth.config(1, K=1024, T=60)
    first = (pi.DeviceProblem(prob, tile_split=1), pi.DeviceModel(model).fold())
    p2, m2 = synth.paper_shape(M=4, K=200, T=30)
    p2.ctrl_cost = 1
    second = (pi.DeviceProblem(p2), pi.DeviceModel(m2))
    _pair(first, second)
    p3, m3 = synth.tiny_problem(9, dyn=DYN_POINTMASS2D, L=[7, 5], R=2, K=40, T=9, M=2,
                                dtype=np.float64, n_obs=3)
    c3 = _noalloc(pi.DeviceProblem(p3), pi.DeviceModel(m3))
    assert torch.equal(c3, _with_workspace(pi.DeviceProblem(p3), pi.DeviceModel(m3)))


def test_noalloc_bf16x3_launches():
    # the three-piece bf16 contraction (model pieces folded into the scratch):
    # the paired 2048-rollout launch, then a smaller ragged problem on the
    # 128-row shared-tile launch with 8 waves
    prob, model, _ = synth.config(1)
    bf = pi.PI_VARIANT_MFMA_BF16X3
    first = (pi.DeviceProblem(prob, variant=bf), pi.DeviceModel(model))
    assert pi.rollout_describe(*first)["variant"] == "mfma-bf16x3"
    p2, m2 = synth.tiny_problem(6, dyn=DYN_QUAD12, L=[19, 16, 33, 8, 16, 17], R=4, K=301, T=37, M=1,
                                dtype=np.float32, n_obs=7)
    second = (pi.DeviceProblem(p2, variant=bf, tile_samples=128, tile_waves=8), pi.DeviceModel(m2))
    assert pi.rollout_describe(*second)["tile_samples"] == 128
    _pair(first, second)


def test_noalloc_f16x2_launch():
    # the two-piece fp16 contraction on the shared tile (its pieces and scales
    # folded into the scratch), then a smaller ragged problem on 4 waves
    prob, model, _ = synth.config(1, K=1024, T=40)
    hf = pi.PI_VARIANT_MFMA_F16X2
    first = (pi.DeviceProblem(prob, variant=hf), pi.DeviceModel(model))
    assert pi.rollout_describe(*first)["variant"] == "mfma-f16x2"
    p2, m2 = synth.tiny_problem(7, dyn=DYN_QUAD12, L=[19, 16, 33, 8, 16, 17], R=4, K=301, T=37, M=1,
                                dtype=np.float32, n_obs=7)
    second = (pi.DeviceProblem(p2, variant=hf, tile_samples=64, tile_waves=4), pi.DeviceModel(m2))
    _pair(first, second)


def test_noalloc_rejects_requests_past_the_scratch():
    # 4096 rollouts x 120 sub-rollouts x 20 steps need 39 MB of sub-rollout
    # costs (and the 6 x 1024-model fold, float32 tiles and bf16 pieces,
    # 16 MB): refused before any device work, the output untouched
    prob, model, _ = synth.config(2, K=4096, T=20)
    prob.M = 120
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    need = pi.workspace_bytes(pi.PI_OP_ROLLOUT, dp, dm)
    assert need > 32 << 20
    cost = torch.zeros((dp.K, dp.T), dtype=torch.float32, device="cuda")
    ps, ms = dp.struct(), dm.struct()
    st = pi.load().pi_rollout_cost_noalloc(C.byref(ps), C.byref(ms), dp.x0.data_ptr(), dp.u_nom.data_ptr(),
                                            dp.iter.data_ptr(), cost.data_ptr(),
                                            torch.cuda.current_stream().cuda_stream)
    assert st == 5     # PI_ERR_WORKSPACE
    assert "allocation-free" in pi.last_error()
    torch.cuda.synchronize()
    assert (cost == 0).all()
