"""Autotuner cache logic (CPU) and tuning runs (GPU): a tuned launch keeps
the oracle's results."""
import json

import numpy as np
import pytest

from paper_1503_00330_amd import tune


def test_cache_roundtrip_and_corruption(tmp_path):
    p = str(tmp_path / "t.json")
    assert tune.load_cache(p) == {}                      # absent
    tune.save_cache({"k": [16, 4, 2]}, p)
    assert tune.load_cache(p) == {"k": [16, 4, 2]}
    with open(p, "w") as f:
        f.write("{not json")
    assert tune.load_cache(p) == {}                      # corrupt -> untuned
    with open(p, "w") as f:
        json.dump({"k": [999, 4, 1], "j": "x", "ok": [8, 8, 1], "b": [32, 4], "bad": [32, 8]}, f)
    assert tune.load_cache(p) == {"ok": [8, 8, 1], "b": [32, 4]}   # invalid entries dropped


def test_shape_key_buckets_sample_counts():
    L = [0, 256, 512, 768, 1024, 1280, 1536]
    a = tune.shape_key("gfx950", 0, 16, 6, L, 4, 2048, 1, 100)
    b = tune.shape_key("gfx950", 0, 16, 6, L, 4, 2000, 1, 100)
    c = tune.shape_key("gfx950", 0, 16, 6, L, 4, 4096, 1, 100)
    d = tune.shape_key("gfx950", 0, 16, 6, L, 4, 2048, 1, 100, dyn=0)
    assert a == b and a != c and a != d


def test_candidate_space_covers_pairing_and_waves():
    # the launch knobs that matter: samples per tile, waves, and pairs of
    # workgroups per tile
    assert {c[2] for c in tune.CANDIDATES} == {1, 2}
    assert {c[1] for c in tune.CANDIDATES} == {4, 8}
    assert {c[0] for c in tune.CANDIDATES} == {8, 16, 32}


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    return torch


@pytest.mark.gpu
def test_tune_rollout_picks_a_candidate_with_oracle_parity(tmp_path):
    _gpu()
    import oracle
    import paper_1503_00330_amd as pi
    import synth
    prob, model, _ = synth.config(1, K=256, T=10)
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    path = str(tmp_path / "tune.json")
    best, times = tune.tune_rollout(dp, dm, reps=1, path=path)
    assert best in tune.candidates_for(dp) and len(times) == len(tune.candidates_for(dp))
    assert len(times) == len(tune.CANDIDATES)          # every knob applies to this problem
    dp2 = pi.DeviceProblem(prob)
    assert tune.apply(dp2, dm, path=path)
    assert (dp2.tile_samples, dp2.tile_waves, dp2.tile_split) == best
    g = pi.rollout_cost(dp2, dm).cpu().numpy().astype(np.float64)
    ref = oracle.rollout_cost(prob, model)
    r = np.abs(g.sum(1) - ref.sum(1)) / np.abs(ref.sum(1))
    assert r.max() <= 1e-4
    # ensure() uses the cache entry without tuning again
    dp3 = pi.DeviceProblem(prob)
    assert tune.ensure(dp3, dm, path=path) == best


@pytest.mark.gpu
def test_tune_hybrid_skips_eight_waves(tmp_path):
    _gpu()
    import paper_1503_00330_amd as pi
    import synth
    prob, model = synth.paper_shape(K=200, T=8)
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    best, times = tune.tune_rollout(dp, dm, reps=1, path=str(tmp_path / "t.json"))
    assert all(w == 4 for _, w, _ in times)


@pytest.mark.gpu
def test_tune_batched_keeps_plain_parity(tmp_path):
    torch = _gpu()
    import paper_1503_00330_amd as pi
    import synth
    probs = []
    for b, (K, T, L) in enumerate(((70, 5, 16), (33, 9, [20, 17, 33, 16, 1, 40]), (130, 4, 9))):
        prob, model = synth.tiny_problem(60 + b, dyn=synth.DYN_QUAD12, L=L, R=4, K=K, T=T, M=1,
                                         dtype=np.float32, n_obs=3)
        probs.append((prob, model))
    dps = [pi.DeviceProblem(p, tile_split=1) for p, _ in probs]
    dms = [pi.DeviceModel(m) for _, m in probs]
    path = str(tmp_path / "t.json")
    best, times = tune.tune_batched(dps, dms, reps=1, path=path)
    assert best in times and len(times) == len(tune.BATCH_CANDIDATES)
    assert tune.apply_batch(dps, dms, path=path)
    costs = [c.clone() for c in pi.BatchedRollout(dps, dms).run()]
    for b, (dp, dm) in enumerate(zip(dps, dms)):
        dp.tile_waves = dps[0].tile_waves
        assert torch.equal(pi.rollout_cost(dp, dm), costs[b]), b
