"""Autotuner for the rollout kernels' tile shape.

For a given problem shape the tuner times pi_rollout_cost (or the batched
launch) for every candidate (samples per workgroup, waves per workgroup) with
HIP events and caches the fastest in a JSON file keyed by the device
architecture and the shape.  A missing, unreadable or corrupt cache simply
means "not tuned": the library's defaults apply.  The cache path is
$PI2RH_AUTOTUNE_CACHE or ~/.cache/pi2rh/tune.json.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, Optional, Tuple

CANDIDATES: Tuple[Tuple[int, int], ...] = ((8, 4), (16, 4), (32, 4), (8, 8), (16, 8))


def cache_path() -> str:
    return os.environ.get("PI2RH_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "pi2rh", "tune.json"))


def shape_key(arch: str, dtype_code: int, d: int, n_out: int, L_off, R: int, K: int, M: int, T: int) -> str:
    Ls = [int(L_off[i + 1]) - int(L_off[i]) for i in range(n_out)]
    kb = 1 << max(0, int(K * max(M, 1) - 1).bit_length())  # power-of-two bucket of samples
    return "%s|dt%d|d%d|o%d|L%s|R%d|S%d|T%d" % (arch, dtype_code, d, n_out, "-".join(map(str, Ls)),
                                               R, kb, T)


def load_cache(path: Optional[str] = None) -> Dict[str, list]:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        if not isinstance(data, dict):
            return {}
        out = {}
        for k, v in data.items():
            if (isinstance(k, str) and isinstance(v, list) and len(v) == 2
                    and all(isinstance(x, int) for x in v) and tuple(v) in CANDIDATES):
                out[k] = [int(v[0]), int(v[1])]
        return out
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
                     prob.M, prob.T)


def apply(prob, model, path: Optional[str] = None) -> bool:
    """Sets prob.tile_samples/tile_waves from the cache; False if untuned."""
    ent = load_cache(path).get(key_for(prob, model))
    if ent is None:
        return False
    prob.tile_samples, prob.tile_waves = ent
    return True


def tune_rollout(prob, model, candidates: Iterable[Tuple[int, int]] = CANDIDATES, reps: int = 3,
                 path: Optional[str] = None, save: bool = True):
    """Times every candidate tile shape; stores and returns the fastest
    ((samples, waves), {candidate: ms})."""
    import torch
    from . import PI_VARIANT_MFMA, rollout_cost
    if prob.variant not in (0, PI_VARIANT_MFMA):
        raise ValueError("tile shapes apply to the matrix-core rollout kernel")
    saved = (prob.tile_samples, prob.tile_waves)
    cost = torch.empty((prob.K, prob.T), dtype=prob.dtype, device=prob.device)
    stream = torch.cuda.current_stream()
    times = {}
    try:
        for spw, waves in candidates:
            prob.tile_samples, prob.tile_waves = spw, waves
            rollout_cost(prob, model, out=cost)          # warm-up / first-launch costs
            evs = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                rollout_cost(prob, model, out=cost)
                b.record(stream)
                evs.append((a, b))
            torch.cuda.synchronize()
            times[(spw, waves)] = min(a.elapsed_time(b) for a, b in evs)
    finally:
        prob.tile_samples, prob.tile_waves = saved
    best = min(times, key=times.get)
    if save:
        data = load_cache(path)
        data[key_for(prob, model)] = list(best)
        save_cache(data, path)
    return best, times
