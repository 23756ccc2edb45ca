"""Autotuner for the rollout kernels' launch shape.

For a given problem shape the tuner times pi_rollout_cost for every candidate
launch (samples per tile, waves per workgroup, workgroups per tile) with HIP
events and caches the fastest in a JSON file keyed by the device architecture
and the shape; for a batch of problems it times the batched launch for every
uniform tile shape.  A missing, unreadable or corrupt cache simply means "not
tuned": the library's defaults apply.  The cache path is
$PI2RH_AUTOTUNE_CACHE or ~/.cache/pi2rh/tune.json.

Every candidate computes the same method; they differ only in how the
mixture's sums are grouped (so results agree to rounding, and are bitwise
reproducible for a fixed candidate).
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Iterable, Optional, Sequence, Tuple

# (samples per tile, waves per workgroup, workgroups per tile)
CANDIDATES: Tuple[Tuple[int, int, int], ...] = (
    (16, 4, 1), (16, 8, 1), (8, 4, 1), (8, 8, 1), (32, 4, 1), (16, 4, 2), (16, 8, 2))
# uniform tile shapes of a batched launch: (samples per tile, waves per workgroup)
BATCH_CANDIDATES: Tuple[Tuple[int, int], ...] = ((16, 4), (8, 4), (32, 4), (16, 8), (8, 8))


def cache_path() -> str:
    return os.environ.get("PI2RH_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "pi2rh", "tune.json"))


def shape_key(arch: str, dtype_code: int, d: int, n_out: int, L_off, R: int, K: int, M: int, T: int,
              dyn: int = 1) -> str:
    Ls = [int(L_off[i + 1]) - int(L_off[i]) for i in range(n_out)]
    kb = 1 << max(0, int(K * max(M, 1) - 1).bit_length())  # power-of-two bucket of samples
    return "%s|dyn%d|dt%d|d%d|o%d|L%s|R%d|S%d|T%d" % (arch, dyn, dtype_code, d, n_out,
                                                      "-".join(map(str, Ls)), R, kb, T)


def _valid(v) -> bool:
    if not isinstance(v, list) or not all(isinstance(x, int) for x in v):
        return False
    return tuple(v) in CANDIDATES or tuple(v) in BATCH_CANDIDATES


def load_cache(path: Optional[str] = None) -> Dict[str, list]:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        if not isinstance(data, dict):
            return {}
        return {k: [int(x) for x in v] for k, v in data.items() if isinstance(k, str) and _valid(v)}
    except (OSError, ValueError):
        return {}


def save_cache(data: Dict[str, list], path: Optional[str] = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _arch() -> str:
    import torch
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def key_for(prob, model) -> str:
    from . import _dt
    return shape_key(_arch(), _dt(prob.dtype), model.d, model.n_out, model.L_off, model.R, prob.K,
                     prob.M, prob.T, prob.dyn)


def batch_key(problems, models) -> str:
    h = hashlib.sha1("|".join(key_for(p, m) for p, m in zip(problems, models)).encode()).hexdigest()
    return "%s|batch%d|%s" % (_arch(), len(problems), h[:16])


def candidates_for(prob) -> Tuple[Tuple[int, int, int], ...]:
    """The candidates the library accepts for this problem: 8 waves only on the
    12-state quadrotor, pairs of workgroups only for tiles of <= 16 samples
    (float32)."""
    from . import PI_DYN_QUAD12
    import torch
    out = []
    for spw, waves, split in CANDIDATES:
        if waves == 8 and (prob.dyn != PI_DYN_QUAD12 or spw > 16):
            continue
        if split == 2 and (spw > 16 or prob.dtype != torch.float32):
            continue
        out.append((spw, waves, split))
    return tuple(out)


def apply(prob, model, path: Optional[str] = None) -> bool:
    """Sets prob's tile_samples/tile_waves/tile_split from the cache; False if untuned."""
    ent = load_cache(path).get(key_for(prob, model))
    if ent is None or len(ent) != 3:
        return False
    prob.tile_samples, prob.tile_waves, prob.tile_split = ent
    return True


def _time(fn, reps: int) -> float:
    import torch
    stream = torch.cuda.current_stream()
    fn()                                  # warm-up / first-launch costs
    evs = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        evs.append((a, b))
    torch.cuda.synchronize()
    return min(a.elapsed_time(b) for a, b in evs)


def tune_rollout(prob, model, candidates: Optional[Iterable[Tuple[int, int, int]]] = None, reps: int = 3,
                 path: Optional[str] = None, save: bool = True):
    """Times every candidate launch; stores and returns the fastest
    ((samples, waves, split), {candidate: ms})."""
    import torch
    from . import PI_VARIANT_MFMA, rollout_cost
    if prob.variant not in (0, PI_VARIANT_MFMA):
        raise ValueError("launch shapes apply to the matrix-core rollout kernels")
    cands = tuple(candidates) if candidates is not None else candidates_for(prob)
    saved = (prob.tile_samples, prob.tile_waves, prob.tile_split)
    cost = torch.empty((prob.K, prob.T), dtype=prob.dtype, device=prob.device)
    times = {}
    try:
        for spw, waves, split in cands:
            prob.tile_samples, prob.tile_waves, prob.tile_split = spw, waves, split
            times[(spw, waves, split)] = _time(lambda: rollout_cost(prob, model, out=cost), reps)
    finally:
        prob.tile_samples, prob.tile_waves, prob.tile_split = saved
    best = min(times, key=times.get)
    if save:
        data = load_cache(path)
        data[key_for(prob, model)] = list(best)
        save_cache(data, path)
    return best, times


def ensure(prob, model, path: Optional[str] = None, reps: int = 3):
    """Applies the cached launch for this shape, tuning (and caching) it first
    if there is none.  Returns the (samples, waves, split) in use."""
    if not apply(prob, model, path):
        best, _ = tune_rollout(prob, model, reps=reps, path=path)
        prob.tile_samples, prob.tile_waves, prob.tile_split = best
    return (prob.tile_samples, prob.tile_waves, prob.tile_split)


def apply_batch(problems: Sequence, models: Sequence, path: Optional[str] = None) -> bool:
    """Sets every problem's tile_samples and problem 0's tile_waves from the
    cache entry of this batch; False if untuned."""
    ent = load_cache(path).get(batch_key(problems, models))
    if ent is None or len(ent) != 2:
        return False
    for p in problems:
        p.tile_samples = ent[0]
    problems[0].tile_waves = ent[1]
    return True


def tune_batched(problems: Sequence, models: Sequence,
                 candidates: Iterable[Tuple[int, int]] = BATCH_CANDIDATES, reps: int = 2,
                 path: Optional[str] = None, save: bool = True):
    """Times the batched rollout launch for every uniform tile shape; stores
    and returns the fastest ((samples, waves), {candidate: ms})."""
    from . import BatchedRollout
    saved = [(p.tile_samples, p.tile_waves) for p in problems]
    times = {}
    try:
        for spw, waves in candidates:
            if waves == 8 and spw > 16:
                continue
            for p in problems:
                p.tile_samples = spw
            problems[0].tile_waves = waves
            br = BatchedRollout(problems, models)
            times[(spw, waves)] = _time(br.run, reps)
            del br
    finally:
        for p, (spw, waves) in zip(problems, saved):
            p.tile_samples, p.tile_waves = spw, waves
    best = min(times, key=times.get)
    if save:
        data = load_cache(path)
        data[batch_key(problems, models)] = list(best)
        save_cache(data, path)
    return best, times


def ensure_batch(problems: Sequence, models: Sequence, path: Optional[str] = None, reps: int = 2):
    if not apply_batch(problems, models, path):
        best, _ = tune_batched(problems, models, reps=reps, path=path)
        for p in problems:
            p.tile_samples = best[0]
        problems[0].tile_waves = best[1]
    return (problems[0].tile_samples, problems[0].tile_waves)
