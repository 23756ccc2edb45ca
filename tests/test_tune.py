"""Autotuner cache logic (CPU) and tuning runs (GPU): a tuned launch keeps
the oracle's results."""
import json

import numpy as np
import pytest

from paper_1503_00330_amd import tune


def test_cache_roundtrip_and_corruption(tmp_path):
    p = str(tmp_path / "t.json")
    assert tune.load_cache(p) == {}                      # absent
    tune.save_cache({"k": [16, 4, 2, 2]}, p)
    assert tune.load_cache(p) == {"k": [16, 4, 2, 2]}
    with open(p, "w") as f:
        f.write("{not json")
    assert tune.load_cache(p) == {}                      # corrupt -> untuned
    with open(p, "w") as f:
        json.dump({"k": [999, 4, 1, 2], "j": "x", "ok": [8, 8, 1, 3], "b": [32, 4, 3], "bad": [32, 8, 2],
                   "old": [8, 8, 1], "v": [16, 4, 1, 1]}, f)
    # invalid entries (and entries without a contraction) dropped
    assert tune.load_cache(p) == {"ok": [8, 8, 1, 3], "b": [32, 4, 3]}


def test_shape_key_buckets_sample_counts():
    L = [0, 256, 512, 768, 1024, 1280, 1536]
    a = tune.shape_key("gfx950", 0, 16, 6, L, 4, 2048, 1, 100)
    b = tune.shape_key("gfx950", 0, 16, 6, L, 4, 2000, 1, 100)
    c = tune.shape_key("gfx950", 0, 16, 6, L, 4, 4096, 1, 100)
    d = tune.shape_key("gfx950", 0, 16, 6, L, 4, 2048, 1, 100, dyn=0)
    e = tune.shape_key("gfx950", 0, 16, 6, L, 4, 2048, 1, 100, variant=2)
    assert a == b and a != c and a != d and a != e


def test_candidate_space_covers_pairing_waves_and_contraction():
    # the launch knobs that matter: samples per tile, waves, pairs of
    # workgroups per tile, and float32 products or their bf16 three-piece form
    assert {c[2] for c in tune.CANDIDATES} == {1, 2}
    assert {c[1] for c in tune.CANDIDATES} == {4, 8}
    assert {c[0] for c in tune.CANDIDATES} == {8, 16, 32, 128}
    assert all(c[3] in (3, 4) for c in tune.CANDIDATES if c[0] > 32)   # shared-tile launch: the pieces forms
    # the fp16 form at every launch shape of the bf16 form
    assert {c[:3] for c in tune.CANDIDATES if c[3] == 4} == {c[:3] for c in tune.CANDIDATES if c[3] == 3}
    assert {c[3] for c in tune.CANDIDATES} == {2, 3, 4}
    assert {c[2] for c in tune.BATCH_CANDIDATES} == {2, 3, 4}


class _P:
    def __init__(self, dyn, dtype, variant=0):
        self.dyn, self.dtype, self.variant = dyn, dtype, variant


class _M:
    def __init__(self, d):
        self.d = d


def test_candidates_follow_the_requested_variant():
    import torch
    from paper_1503_00330_amd import PI_DYN_QUAD12, PI_DYN_POINTMASS2D
    q = tune.candidates_for(_P(PI_DYN_QUAD12, torch.float32), _M(16))
    assert {c[3] for c in q} == {2, 3, 4}
    assert (128, 8, 1, 4) in q and (128, 4, 1, 4) in q
    # bf16 form: no 8 waves with 32-sample tiles, no pairs above 16 samples
    assert (32, 8, 1, 3) not in q and (32, 4, 2, 3) not in q and (32, 4, 1, 3) in q
    assert (128, 4, 1, 3) in q and (128, 8, 1, 3) in q
    assert {c[3] for c in tune.candidates_for(_P(PI_DYN_QUAD12, torch.float32, 2), _M(16))} == {2}
    assert {c[3] for c in tune.candidates_for(_P(PI_DYN_QUAD12, torch.float32, 3), _M(16))} == {3}
    q4 = tune.candidates_for(_P(PI_DYN_QUAD12, torch.float32, 4), _M(16))
    assert {c[3] for c in q4} == {4} and (16, 8, 2, 4) in q4 and (128, 8, 1, 4) in q4 and (32, 8, 1, 4) not in q4
    # not eligible for the bf16 form: another d, float64, another plant
    assert {c[3] for c in tune.candidates_for(_P(PI_DYN_QUAD12, torch.float32), _M(8))} == {2}
    assert {c[3] for c in tune.candidates_for(_P(PI_DYN_QUAD12, torch.float64), _M(16))} == {2}
    assert {c[3] for c in tune.candidates_for(_P(PI_DYN_POINTMASS2D, torch.float32), _M(16))} == {2}
    # applying a tuned contraction keeps the request aside for the cache key
    p = _P(PI_DYN_QUAD12, torch.float32)
    tune._set_variant(p, 3)
    assert p.variant == 3 and tune._requested(p) == 0


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
    assert best in tune.candidates_for(dp, dm) and len(times) == len(tune.candidates_for(dp, dm))
    # every candidate applies to this problem, both contractions included
    assert len(times) == len(tune.CANDIDATES)
    assert dp.variant == 0                              # tuning leaves the problem as it was
    dp2 = pi.DeviceProblem(prob)
    assert tune.apply(dp2, dm, path=path)
    assert (dp2.tile_samples, dp2.tile_waves, dp2.tile_split, dp2.variant) == best
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
    assert all(w == 4 and v == 2 for _, w, _, v in times)


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
    assert best in times and len(times) == len(tune.batch_candidates_for(dps, dms))
    assert {c[2] for c in times} == {2, 3, 4}
    assert tune.apply_batch(dps, dms, path=path)
    costs = [c.clone() for c in pi.BatchedRollout(dps, dms).run()]
    for b, (dp, dm) in enumerate(zip(dps, dms)):
        dp.tile_waves = dps[0].tile_waves
        assert dp.variant == best[2]
        assert torch.equal(pi.rollout_cost(dp, dm), costs[b]), b
