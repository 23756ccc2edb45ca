"""Autotuner cache logic (CPU) and one tuning run (GPU)."""
import json

import numpy as np
import pytest

from paper_1503_00330_amd import tune


def test_cache_roundtrip_and_corruption(tmp_path):
    p = str(tmp_path / "t.json")
    assert tune.load_cache(p) == {}                      # absent
    tune.save_cache({"k": [16, 4]}, p)
    assert tune.load_cache(p) == {"k": [16, 4]}
    with open(p, "w") as f:
        f.write("{not json")
    assert tune.load_cache(p) == {}                      # corrupt -> untuned
    with open(p, "w") as f:
        json.dump({"k": [999, 4], "j": "x", "ok": [8, 8]}, f)
    assert tune.load_cache(p) == {"ok": [8, 8]}          # invalid entries dropped


def test_shape_key_buckets_sample_counts():
    a = tune.shape_key("gfx950", 0, 16, 6, [0, 256, 512, 768, 1024, 1280, 1536], 4, 2048, 1, 100)
    b = tune.shape_key("gfx950", 0, 16, 6, [0, 256, 512, 768, 1024, 1280, 1536], 4, 2000, 1, 100)
    c = tune.shape_key("gfx950", 0, 16, 6, [0, 256, 512, 768, 1024, 1280, 1536], 4, 4096, 1, 100)
    assert a == b and a != c


@pytest.mark.gpu
def test_tune_rollout_picks_a_candidate(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_1503_00330_amd as pi
    import synth
    prob, model, _ = synth.config(1, K=256, T=10)
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    path = str(tmp_path / "tune.json")
    best, times = tune.tune_rollout(dp, dm, reps=1, path=path)
    assert best in tune.CANDIDATES and len(times) == len(tune.CANDIDATES)
    dp2 = pi.DeviceProblem(prob)
    assert tune.apply(dp2, dm, path=path) and (dp2.tile_samples, dp2.tile_waves) == best
    a = pi.rollout_cost(dp, dm).cpu().numpy()
    b = pi.rollout_cost(dp2, dm).cpu().numpy()
    assert np.max(np.abs(a - b)) <= 1e-5 * np.abs(a).max()
