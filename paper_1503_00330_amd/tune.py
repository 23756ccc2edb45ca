"""Autotuner for the rollout kernels' launch shape.

For a given problem shape the tuner times pi_rollout_cost for every candidate
launch (samples per tile, waves per workgroup, workgroups per tile, and the
contraction: float32 matrix-core products, their three-piece bf16 form or
their two-piece fp16 form)
with HIP events and caches the fastest in a JSON file keyed by the device
architecture, the shape and the requested variant; for a batch of problems it
times the batched launch for every uniform tile shape and contraction.  A
missing, unreadable or corrupt cache simply means "not tuned": the library's
defaults apply.  The cache path is $PI2RH_AUTOTUNE_CACHE or
~/.cache/pi2rh/tune.json.

The contraction is searched only when the problem asks for the library's
choice (PI_VARIANT_AUTO); a problem that names a variant keeps it.  Every
candidate computes the same method to float32 accuracy; they differ only in
how the mixture's sums are grouped and how the float32 products are formed
(results agree to rounding, and are bitwise reproducible for a fixed
candidate).
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Iterable, Optional, Sequence, Tuple

# contraction codes, as PI_VARIANT_MFMA, PI_VARIANT_MFMA_BF16X3 and PI_VARIANT_MFMA_F16X2
_MF, _BF, _HF = 2, 3, 4
_SHAPES = ((16, 4, 1), (16, 8, 1), (8, 4, 1), (8, 8, 1), (32, 4, 1), (16, 4, 2), (16, 8, 2))
_BATCH_SHAPES = ((16, 4), (8, 4), (32, 4), (16, 8), (8, 8))
# (samples per tile, waves per workgroup, workgroups per tile, contraction);
# 128-sample tiles are the pieces forms' shared-tile launch
CANDIDATES: Tuple[Tuple[int, int, int, int], ...] = (tuple(s + (v,) for v in (_MF, _BF, _HF) for s in _SHAPES)
                                                     + tuple((128, w, 1, v) for v in (_BF, _HF) for w in (4, 8)))
# uniform launches of a batch: (samples per tile, waves per workgroup, contraction)
BATCH_CANDIDATES: Tuple[Tuple[int, int, int], ...] = (tuple(s + (v,) for v in (_MF, _BF, _HF)
                                                            for s in _BATCH_SHAPES)
                                                      + tuple((128, w, v) for v in (_BF, _HF) for w in (4, 8)))


def cache_path() -> str:
    return os.environ.get("PI2RH_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "pi2rh", "tune.json"))


def shape_key(arch: str, dtype_code: int, d: int, n_out: int, L_off, R: int, K: int, M: int, T: int,
              dyn: int = 1, variant: int = 0) -> str:
    Ls = [int(L_off[i + 1]) - int(L_off[i]) for i in range(n_out)]
    kb = 1 << max(0, int(K * max(M, 1) - 1).bit_length())  # power-of-two bucket of samples
    return "%s|dyn%d|dt%d|d%d|o%d|L%s|R%d|S%d|T%d|v%d" % (arch, dyn, dtype_code, d, n_out,
                                                          "-".join(map(str, Ls)), R, kb, T, variant)


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


def _requested(prob) -> int:
    """The variant the caller asked for (a tuned problem keeps it aside, since
    applying a tuned entry sets prob.variant to the contraction it chose)."""
    return int(prob.__dict__.get("_requested_variant", prob.variant))


def _set_variant(prob, v: int) -> None:
    prob.__dict__.setdefault("_requested_variant", int(prob.variant))
    prob.variant = int(v)


def key_for(prob, model) -> str:
    from . import _dt
    return shape_key(_arch(), _dt(prob.dtype), model.d, model.n_out, model.L_off, model.R, prob.K,
                     prob.M, prob.T, prob.dyn, _requested(prob))


def batch_key(problems, models) -> str:
    h = hashlib.sha1("|".join(key_for(p, m) for p, m in zip(problems, models)).encode()).hexdigest()
    return "%s|batch%d|%s" % (_arch(), len(problems), h[:16])


def _variants_for(prob, models) -> Tuple[int, ...]:
    """Contractions to search: the named one, or with PI_VARIANT_AUTO float32
    products and, for float32 12-state quadrotor problems on d = 16 models,
    their three-piece bf16 and two-piece fp16 forms."""
    from . import PI_DYN_QUAD12
    import torch
    req = _requested(prob)
    if req in (_MF, _BF, _HF):
        return (req,)
    bf_ok = prob.dyn == PI_DYN_QUAD12 and prob.dtype == torch.float32 and all(m.d == 16 for m in models)
    return (_MF, _BF, _HF) if bf_ok else (_MF,)


def candidates_for(prob, model=None) -> Tuple[Tuple[int, int, int, int], ...]:
    """The candidates the library accepts for this problem: 8 waves only on the
    12-state quadrotor with tiles of <= 16 samples (or the pieces forms'
    128-sample shared tiles), pairs of workgroups only for tiles of <= 16
    samples of float32 problems, the pieces forms as _variants_for says (without a
    model: only the float32 products)."""
    from . import PI_DYN_QUAD12
    import torch
    variants = _variants_for(prob, [model]) if model is not None else (_MF,)
    out = []
    for spw, waves, split, v in CANDIDATES:
        if v not in variants:
            continue
        if waves == 8 and (prob.dyn != PI_DYN_QUAD12 or 16 < spw <= 32):
            continue
        if split == 2 and (spw > 16 or prob.dtype != torch.float32):
            continue
        out.append((spw, waves, split, v))
    return tuple(out)


def _launch(prob):
    return (prob.tile_samples, prob.tile_waves, prob.tile_split, prob.variant)


def _set_launch(prob, c) -> None:
    prob.tile_samples, prob.tile_waves, prob.tile_split = c[:3]
    _set_variant(prob, c[3])


def apply(prob, model, path: Optional[str] = None) -> bool:
    """Sets prob's tile_samples/tile_waves/tile_split/variant from the cache;
    False if untuned."""
    ent = load_cache(path).get(key_for(prob, model))
    if ent is None or len(ent) != 4:
        return False
    _set_launch(prob, ent)
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


def tune_rollout(prob, model, candidates: Optional[Iterable[Tuple[int, int, int, int]]] = None, reps: int = 3,
                 path: Optional[str] = None, save: bool = True):
    """Times every candidate launch; stores and returns the fastest
    ((samples, waves, split, variant), {candidate: ms})."""
    import torch
    from . import rollout_cost
    if _requested(prob) not in (0, _MF, _BF, _HF):
        raise ValueError("launch shapes apply to the matrix-core rollout kernels")
    cands = tuple(candidates) if candidates is not None else candidates_for(prob, model)
    saved = _launch(prob)
    cost = torch.empty((prob.K, prob.T), dtype=prob.dtype, device=prob.device)
    times = {}
    try:
        for c in cands:
            _set_launch(prob, c)
            times[tuple(c)] = _time(lambda: rollout_cost(prob, model, out=cost), reps)
    finally:
        prob.tile_samples, prob.tile_waves, prob.tile_split, prob.variant = saved
    best = min(times, key=times.get)
    if save:
        data = load_cache(path)
        data[key_for(prob, model)] = list(best)
        save_cache(data, path)
    return best, times


def ensure(prob, model, path: Optional[str] = None, reps: int = 3):
    """Applies the cached launch for this shape, tuning (and caching) it first
    if there is none.  Returns the (samples, waves, split, variant) in use."""
    if not apply(prob, model, path):
        best, _ = tune_rollout(prob, model, reps=reps, path=path)
        _set_launch(prob, best)
    return _launch(prob)


def _set_batch(problems, c) -> None:
    for p in problems:
        p.tile_samples = c[0]
        _set_variant(p, c[2])
    problems[0].tile_waves = c[1]


def apply_batch(problems: Sequence, models: Sequence, path: Optional[str] = None) -> bool:
    """Sets every problem's tile_samples and variant and problem 0's
    tile_waves from the cache entry of this batch; False if untuned."""
    ent = load_cache(path).get(batch_key(problems, models))
    if ent is None or len(ent) != 3:
        return False
    _set_batch(problems, ent)
    return True


def batch_candidates_for(problems: Sequence, models: Sequence) -> Tuple[Tuple[int, int, int], ...]:
    """Uniform launches the batched kernel accepts for these problems (8 waves
    only with tiles of <= 16 samples or the pieces forms' 128-sample shared
    tiles; the pieces forms when every problem allows them and asks for the
    library's choice)."""
    vs = set(_variants_for(problems[0], models))
    for p in problems[1:]:
        vs &= set(_variants_for(p, models))
    return tuple(c for c in BATCH_CANDIDATES if c[2] in vs and not (c[1] == 8 and 16 < c[0] <= 32))


def tune_batched(problems: Sequence, models: Sequence,
                 candidates: Optional[Iterable[Tuple[int, int, int]]] = None, reps: int = 2,
                 path: Optional[str] = None, save: bool = True):
    """Times the batched rollout launch for every uniform launch; stores and
    returns the fastest ((samples, waves, variant), {candidate: ms})."""
    from . import BatchedRollout
    cands = tuple(candidates) if candidates is not None else batch_candidates_for(problems, models)
    saved = [(p.tile_samples, p.tile_waves, p.variant) for p in problems]
    times = {}
    try:
        for c in cands:
            if c[1] == 8 and 16 < c[0] <= 32:
                continue
            _set_batch(problems, c)
            br = BatchedRollout(problems, models)
            times[tuple(c)] = _time(br.run, reps)
            del br
    finally:
        for p, (spw, waves, v) in zip(problems, saved):
            p.tile_samples, p.tile_waves, p.variant = spw, waves, v
    best = min(times, key=times.get)
    if save:
        data = load_cache(path)
        data[batch_key(problems, models)] = list(best)
        save_cache(data, path)
    return best, times


def ensure_batch(problems: Sequence, models: Sequence, path: Optional[str] = None, reps: int = 2):
    """Applies (tuning first if absent) the batch's launch; returns
    (samples, waves, variant)."""
    if not apply_batch(problems, models, path):
        best, _ = tune_batched(problems, models, reps=reps, path=path)
        _set_batch(problems, best)
    return (problems[0].tile_samples, problems[0].tile_waves, problems[0].variant)
