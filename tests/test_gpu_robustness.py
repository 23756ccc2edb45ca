"""Failure handling of the HIP path, forced from the host so that every kernel
still exits normally.

* Paired workgroups: the bounded wait on the partner is forced to give up at
  once (PI2RH_PAIR_SPIN_LIMIT=0).  Every cost row must then be the normal
  launch's row up to some chunk and NaN from there on -- never a finite value
  computed from a half whose state went stale -- and the give-ups are counted.
* Non-finite inputs (NaN or Inf in the start state, a nominal control, a local
  model's centre, prediction inputs) propagate: the GPU and the oracle have
  the same non-finite entries and agree on the finite ones.
"""

import numpy as np
import pytest

import oracle
import synth
from synth import DYN_QUAD12

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


def _prefix_then_nan(got, ref):
    """Rows equal to ref bitwise up to their first NaN, NaN from there on."""
    bad = 0
    for g, r in zip(got, ref):
        nan = np.isnan(g)
        f = int(np.argmax(nan)) if nan.any() else len(g)
        assert np.array_equal(g[:f], r[:f])
        assert nan[f:].all()
        bad += f < len(g)
    return bad


@pytest.mark.parametrize("waves,variant", [(4, pi.PI_VARIANT_AUTO), (8, pi.PI_VARIANT_AUTO),
                                           (4, pi.PI_VARIANT_MFMA_F16X2)])
def test_forced_pair_give_up_never_leaves_finite_wrong_costs(waves, variant, monkeypatch):
    prob, model, _ = synth.config(1, T=40)
    prob.u_nom = np.random.default_rng(9).normal(0.0, 0.2, prob.u_nom.shape).astype(F32)
    dp = pi.DeviceProblem(prob, tile_split=2, tile_waves=waves, variant=variant)
    dm = pi.DeviceModel(model).fold()
    assert pi.rollout_describe(dp, dm)["tile_split"] == 2
    ref = pi.rollout_cost(dp, dm).cpu().numpy()
    assert np.isfinite(ref).all()
    before = pi.pair_give_ups()
    monkeypatch.setenv("PI2RH_PAIR_SPIN_LIMIT", "0")
    got = pi.rollout_cost(dp, dm).cpu().numpy()
    monkeypatch.delenv("PI2RH_PAIR_SPIN_LIMIT")
    given_up = pi.pair_give_ups() - before
    bad_rows = _prefix_then_nan(got, ref)
    print("waves %d: %d workgroups gave up, %d of %d rows abandoned" % (waves, given_up, bad_rows, len(got)))
    assert given_up > 0 and bad_rows > 0
    # the library's own limit again: the next launch is whole
    assert np.array_equal(pi.rollout_cost(dp, dm).cpu().numpy(), ref)
    assert pi.pair_give_ups() == before + given_up


def _nonfinite_match(g, o, tol):
    g, o = np.asarray(g, np.float64), np.asarray(o, np.float64)
    assert np.array_equal(~np.isfinite(g), ~np.isfinite(o))
    fin = np.isfinite(o)
    if fin.any():
        err = np.abs(g[fin] - o[fin]) / np.maximum(np.abs(o[fin]), 1e-3 * np.abs(o[fin]).max())
        assert err.max() <= tol, err.max()


INJECT = ["x0_nan", "u_nan", "u_inf", "centre_nan"]
# (dtype, variant, split, samples per tile): matrix-core paired and single,
# the pieces forms (fp16 pairs and shared tile, bf16 shared tile), direct
# float32, float64
FORMS = [(F32, pi.PI_VARIANT_MFMA, 2, 0), (F32, pi.PI_VARIANT_MFMA, 1, 0),
         (F32, pi.PI_VARIANT_MFMA_F16X2, 2, 0), (F32, pi.PI_VARIANT_MFMA_F16X2, 1, 128),
         (F32, pi.PI_VARIANT_MFMA_BF16X3, 1, 128), (F32, pi.PI_VARIANT_DIRECT, 0, 0),
         (F64, pi.PI_VARIANT_DIRECT, 0, 0)]


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("inject", INJECT)
def test_nonfinite_inputs_propagate_like_the_oracle(inject, form):
    dtype, variant, split, spw = form
    prob, model = synth.tiny_problem(31, dyn=DYN_QUAD12, L=[17, 12, 20, 9, 16, 11], R=3, K=40, T=23,
                                     M=1, dtype=dtype, n_obs=4)
    prob.u_nom = np.random.default_rng(2).normal(0.0, 0.2, prob.u_nom.shape).astype(dtype)
    if inject == "x0_nan":
        prob.x0[4] = np.nan
    elif inject == "u_nan":
        prob.u_nom[9, 1] = np.nan
    elif inject == "u_inf":
        prob.u_nom[14, 3] = np.inf
    else:
        model.centre[model.L_off[2] + 3, 5] = np.nan
    dp = pi.DeviceProblem(prob, variant=variant, tile_split=split, tile_samples=spw)
    got = pi.rollout_cost(dp, pi.DeviceModel(model)).cpu().numpy()
    ref = oracle.rollout_cost(prob, model)
    assert not np.isfinite(ref).all()
    _nonfinite_match(got, ref, 1e-10 if dtype == F64 else 1e-4)


@pytest.mark.parametrize("variant", [pi.PI_VARIANT_MFMA, pi.PI_VARIANT_DIRECT])
def test_nonfinite_prediction_inputs_stay_in_their_rows(variant):
    _, model = synth.tiny_problem(8, dyn=DYN_QUAD12, L=[40, 33, 18, 25, 30, 21], R=4, dtype=F32)
    Z = np.random.default_rng(4).uniform(-1, 1, (70, 16)).astype(F32)
    Z[3, 2] = np.nan
    Z[21, 0] = np.inf
    Z[40, 15] = -np.inf
    mean, var = pi.lwpr_predict(pi.DeviceModel(model), torch.from_numpy(Z).cuda(), variant=variant)
    om, ov = oracle.lwpr_predict(model, Z)
    bad = np.zeros(len(Z), bool)
    bad[[3, 21, 40]] = True
    for g, o in ((mean.cpu().numpy(), om), (var.cpu().numpy(), ov)):
        assert np.array_equal(~np.isfinite(g), ~np.isfinite(o))
        assert (~np.isfinite(o[bad])).all() and np.isfinite(o[~bad]).all()
        err = np.abs(g[~bad] - o[~bad]).max(0) / np.abs(o[~bad]).max(0)
        assert err.max() <= 1e-5
