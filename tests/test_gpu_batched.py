"""Batched controllers in one persistent launch: each problem of an uneven
batch gives exactly (bitwise) the costs of its own plain launch with one
workgroup per tile and matches the oracle; a batched control step (rollouts,
updates, receding-horizon advances) leaves every problem's state exactly as
its own plain control step does, eagerly and replayed from a HIP graph."""
import numpy as np
import pytest

import oracle
import synth
from synth import DYN_QUAD12

torch = pytest.importorskip("torch")
pi = pytest.importorskip("paper_1503_00330_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    yield
    torch.cuda.synchronize()


def _batch(spw=0, waves=0, variant=0):
    specs = [(33, 9, [20, 17, 33, 16, 1, 40], 1), (70, 5, 16, 2), (17, 12, 7, 1),
             (128, 3, [64, 3, 9, 12, 30, 2], 0), (5, 7, 48, 1)]
    out = []
    for b, (K, T, L, M) in enumerate(specs):
        prob, model = synth.tiny_problem(40 + b, dyn=DYN_QUAD12, L=L, R=4, K=K, T=T, M=M,
                                         dtype=np.float32, n_obs=4 + b)
        prob.problem_id = b
        out.append((prob, model))
    # plain launches of the same problems keep one workgroup per tile (a pair of
    # workgroups sums the model halves in another order) and the persistent
    # launch's waves per workgroup (4 unless given; the waves' partial sums are
    # added in order, so another wave count groups them differently)
    dps = [pi.DeviceProblem(p, tile_samples=spw, tile_waves=waves or 4, tile_split=1, variant=variant)
           for p, _ in out]
    dms = [pi.DeviceModel(m) for _, m in out]
    return out, dps, dms


BF3 = 3   # PI_VARIANT_MFMA_BF16X3: the contraction in three bf16 pieces
HF2 = 4   # PI_VARIANT_MFMA_F16X2: in two fp16 pieces


@pytest.mark.parametrize("spw,waves,variant", [(0, 0, 0), (8, 4, 0), (16, 8, 0), (32, 4, 0),
                                               (0, 0, BF3), (16, 8, BF3), (32, 4, BF3), (128, 8, BF3),
                                               (128, 4, BF3), (0, 0, HF2), (16, 8, HF2), (32, 4, HF2), (128, 8, HF2),
                                               (64, 4, HF2)])
def test_batched_equals_plain_launches(spw, waves, variant):
    host, dps, dms = _batch(spw, waves, variant)
    for dp in dps:
        dp.iter.fill_(3)
    br = pi.BatchedRollout(dps, dms)
    costs = [c.clone() for c in br.run()]
    for b, (dp, dm) in enumerate(zip(dps, dms)):
        plain = pi.rollout_cost(dp, dm)
        assert torch.equal(plain, costs[b]), b
    # and against the oracle
    for b, (prob, model) in enumerate(host):
        ref = oracle.rollout_cost(prob, model, it=3)
        g = costs[b].cpu().numpy().astype(np.float64)
        r = np.abs(g.sum(1) - ref.sum(1)) / np.abs(ref.sum(1))
        flips = np.abs(g - ref).max(1) > 0.25 * prob.dt * prob.obs_penalty
        assert flips.sum() <= 1 and r[~flips].max() <= 1e-4, (b, r.max())


def test_batched_rerun_is_repeatable():
    _, dps, dms = _batch()
    br = pi.BatchedRollout(dps, dms)
    a = [c.clone() for c in br.run()]
    b = br.run()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_batched_full_workload():
    # the 64 uneven quadrotor problems (K 512..16384, 6 x (64..1024) models,
    # T 50..200) in one persistent launch: bitwise equal to each problem's
    # plain 4-wave one-workgroup-per-tile launch, and sampled rollouts of the
    # first, the largest and the last problem against the oracle
    batch = synth.batched_config()
    dps = [pi.DeviceProblem(p, tile_split=1, tile_waves=4) for p, _ in batch]
    dms = [pi.DeviceModel(m) for _, m in batch]
    br = pi.BatchedRollout(dps, dms)
    costs = [c.clone() for c in br.run()]
    for b, (dp, dm) in enumerate(zip(dps, dms)):
        assert torch.equal(pi.rollout_cost(dp, dm), costs[b]), b
    big = max(range(len(batch)), key=lambda b: batch[b][0].K * batch[b][1].centre.shape[0])
    for b in sorted({0, big, len(batch) - 1}):
        prob, model = batch[b]
        g = costs[b].cpu().numpy().astype(np.float64)
        assert g.shape == (prob.K, prob.T) and np.all(np.isfinite(g))
        starts = (0, prob.K - 16)
        rows = [a + i for a in starts for i in range(16)]
        ref = np.concatenate([oracle.rollout_cost(prob, model, k_range=(a, a + 16)) for a in starts])
        r = np.abs(g[rows].sum(1) - ref.sum(1)) / np.abs(ref.sum(1))
        flips = np.abs(g[rows] - ref).max(1) > 0.25 * prob.dt * prob.obs_penalty
        assert flips.sum() <= 1 and r[~flips].max() <= 1e-4, (b, r.max())
        print("batched problem %d (K=%d, T=%d): max S rel %.2e, flips %d"
              % (b, prob.K, prob.T, r[~flips].max(), flips.sum()))


def _state(dps):
    return [(d.x0.clone(), d.u_nom.clone(), d.iter.clone()) for d in dps]


def _plain_control_step(dp, dm):
    cost = pi.rollout_cost(dp, dm)
    pi.update(dp, cost)
    pi.rh_shift(dp, dm)
    return cost


@pytest.mark.parametrize("variant", [0, BF3, HF2])
def test_batched_tiles_per_problem(variant):
    # every problem keeps its own tile size (8, 16, 32 and the default) in one launch
    host, dps, dms = _batch(variant=variant)
    for dp, spw in zip(dps, (8, 32, 16, 0, 8)):
        dp.tile_samples = spw
    br = pi.BatchedRollout(dps, dms)
    costs = [c.clone() for c in br.run()]
    for b, (dp, dm) in enumerate(zip(dps, dms)):
        if variant != HF2:
            assert torch.equal(pi.rollout_cost(dp, dm), costs[b]), b
            continue
        # the fp16 form's 8- and 16-row problems run on the batch's 32-row
        # instantiation, whose scale products the compiler rounds in another
        # order than the 16-row one: not bitwise, so against the oracle
        prob, model = host[b]
        got, ref = costs[b].double().cpu().numpy(), oracle.rollout_cost(prob, model)
        flip = np.abs(got - ref).max(1) > 0.25 * prob.dt * prob.obs_penalty
        r = np.abs(got.sum(1) - ref.sum(1)) / np.abs(ref.sum(1))
        assert flip.sum() <= 1 and r[~flip].max(initial=0.0) <= 1e-4, (b, r.max())


@pytest.mark.parametrize("prefold,launch", [(False, (0, 0, 0)), (True, (0, 0, 0)), (False, (128, 8, BF3)),
                                            (False, (128, 8, HF2))])
def test_batched_control_step_equals_plain_control_steps(prefold, launch):
    host, dps, dms = _batch(*launch)
    if prefold:          # models read in place from their pi_model_fold buffers
        for dm in dms[::2]:
            dm.fold()
    for b, dp in enumerate(dps):
        dp.iter.fill_(b)
    start = _state(dps)
    br = pi.BatchedRollout(dps, dms)
    br.control_step()
    after = _state(dps)
    costs = [c.clone() for c in br.costs]
    for dp, (x, u, it) in zip(dps, start):
        dp.x0.copy_(x), dp.u_nom.copy_(u), dp.iter.copy_(it)
    for b, (dp, dm) in enumerate(zip(dps, dms)):
        cost = _plain_control_step(dp, dm)
        assert torch.equal(cost, costs[b]), b
        assert torch.equal(dp.x0, after[b][0]) and torch.equal(dp.u_nom, after[b][1]), b
        assert int(dp.iter.item()) == b + 1 == int(after[b][2].item())
    # against the oracle's control step (rollouts, update, plant step, shift)
    for b, (prob, model) in enumerate(host):
        p = prob.copy()
        x, u, it = oracle.rh_loop(p, model, steps=1, iterations=1, it=b)
        assert it == b + 1
        assert np.max(np.abs(after[b][1].cpu().numpy() - u)) <= 1e-4, b
        assert np.max(np.abs(after[b][0].cpu().numpy() - x)) <= 1e-4 * max(1.0, np.abs(x).max()), b


@pytest.mark.parametrize("launch", [(0, 0, 0), (128, 8, BF3), (128, 8, HF2)])
def test_batched_control_step_graph_replays(launch):
    # one batched control step captured once and replayed three times, each
    # replay checked against the same step run eagerly from the same state
    # (the library's default tiles, and the bf16 form's shared tile)
    _, dps, dms = _batch(*launch)
    br = pi.BatchedRollout(dps, dms)
    br.capture()
    for rep in range(3):
        start = _state(dps)
        br.step(graph=True)
        torch.cuda.synchronize()
        replay = _state(dps)
        for dp, (x, u, it) in zip(dps, start):
            dp.x0.copy_(x), dp.u_nom.copy_(u), dp.iter.copy_(it)
        br.step(graph=False)
        torch.cuda.synchronize()
        eager = _state(dps)
        for a, b in zip(replay, eager):
            for x, y in zip(a, b):
                assert torch.equal(x, y), rep
        assert int(dps[0].iter.item()) == rep + 1


def test_batched_control_step_full_workload():
    # the 64 uneven problems of the batched workload: one batched control step
    # leaves every (x0, u_nom, iter) exactly as 64 plain control steps do
    batch = synth.batched_config()
    dps = [pi.DeviceProblem(p, tile_split=1, tile_waves=4) for p, _ in batch]
    dms = [pi.DeviceModel(m).fold() for _, m in batch]
    start = _state(dps)
    br = pi.BatchedRollout(dps, dms)
    br.control_step()
    after = _state(dps)
    for dp, (x, u, it) in zip(dps, start):
        dp.x0.copy_(x), dp.u_nom.copy_(u), dp.iter.copy_(it)
    for b, (dp, dm) in enumerate(zip(dps, dms)):
        _plain_control_step(dp, dm)
        assert torch.equal(dp.x0, after[b][0]) and torch.equal(dp.u_nom, after[b][1]), b
        assert torch.equal(dp.iter, after[b][2]), b


def test_batched_refuses_unsupported_tiles():
    # 33..128-row tiles only with the pieces forms (their shared-tile launch),
    # and 8 waves not with 17..32-row tiles
    host, dps, dms = _batch(variant=BF3)
    for dp in dps:
        dp.tile_samples, dp.variant = 128, 2
    with pytest.raises(pi.PiError, match="tile_samples=128 outside"):
        pi.BatchedRollout(dps, dms)
    for dp in dps:
        dp.tile_samples, dp.variant = 32, BF3
    dps[0].tile_waves = 8
    with pytest.raises(pi.PiError, match="tile_waves 8"):
        pi.BatchedRollout(dps, dms)
