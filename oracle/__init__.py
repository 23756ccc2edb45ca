"""FP64 CPU oracle for PI^2-RH with LWPR dynamics -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The C source (pi2rh_oracle.c) shares nothing with the HIP
implementation; see its header for the paper passages each function follows.

Inputs are ``synth`` instances; every array is converted to float64 exactly
(float32 values are represented exactly in float64).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pi2rh_oracle.c")
_LIB = os.path.join(_HERE, "_build", "libpi2rh_oracle.so")

TAG_CTRL, TAG_DYN, TAG_PLANT = 0, 1, 2


def build(force: bool = True) -> str:
    """Compiles the oracle with gcc (-O2, OpenMP, strict IEEE: no fast-math)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-Wall", "-Wno-unused-function",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Model(C.Structure):
    _fields_ = [("d", C.c_int32), ("n_out", C.c_int32), ("R", C.c_int32),
                ("L_off", C.c_void_p), ("centre", C.c_void_p), ("metric", C.c_void_p),
                ("proj_u", C.c_void_p), ("proj_p", C.c_void_p), ("beta", C.c_void_p),
                ("sigma2", C.c_void_p)]


class _Problem(C.Structure):
    _fields_ = [("dyn", C.c_int32), ("K", C.c_int32), ("T", C.c_int32), ("M", C.c_int32),
                ("dt", C.c_double), ("lam", C.c_double), ("noise_std", C.c_double * 4),
                ("goal", C.c_double * 3), ("w_pos", C.c_double * 3), ("w_ang", C.c_double),
                ("w_vel", C.c_double), ("obs_kind", C.c_int32), ("n_obs", C.c_int32),
                ("obs", C.c_void_p), ("obs_penalty", C.c_double), ("obs_decay", C.c_double),
                ("weighting", C.c_int32), ("seed", C.c_uint64), ("problem_id", C.c_uint32),
                ("ctrl_cost", C.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = C.CDLL(_LIB)
        vp, i32, i64, u32, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
        lib.orc_philox.argtypes = [vp, vp, vp]
        lib.orc_normals.argtypes = [u64, u32, u32, u32, u32, u32, u32, i32, vp]
        lib.orc_lwpr_predict.argtypes = [vp, vp, i64, vp, vp, vp, i32]
        lib.orc_rollout_cost.argtypes = [vp, vp, vp, vp, u32, i64, i64, vp, vp, i32]
        lib.orc_update.argtypes = [vp, vp, u32, vp, vp]
        lib.orc_rh_shift.argtypes = [vp, vp, vp, vp, vp]
        lib.orc_adjoint.argtypes = [vp, vp, vp, vp, u32, vp, vp, vp, i32]
        lib.orc_adjoint.restype = C.c_double
        lib.orc_max_threads.restype = i32
        lib.orc_philox_many.argtypes = [i64, vp, vp, vp]
        lib.orc_noise_block.argtypes = [u64, u32, u32, u32, i64, i64, u32, i32, i32, vp]
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class _Keep:
    """Holds the float64 copies alive while a struct points at them."""

    def __init__(self):
        self.refs = []

    def __call__(self, a):
        if a is None:
            return None
        self.refs.append(a)
        return _ptr(a)


def _model_struct(model, keep):
    s = _Model()
    s.d, s.n_out, s.R = model.d, model.n_out, model.R
    s.L_off = keep(np.ascontiguousarray(model.L_off.astype(np.int64)))
    s.centre = keep(_f64(model.centre))
    s.metric = keep(_f64(model.metric))
    s.proj_u = keep(_f64(model.proj_u))
    s.proj_p = keep(None if model.proj_p is None else _f64(model.proj_p))
    s.beta = keep(_f64(model.beta))
    s.sigma2 = keep(_f64(model.sigma2))
    return s


def _problem_struct(prob, keep):
    s = _Problem()
    s.dyn, s.K, s.T, s.M = prob.dyn, prob.K, prob.T, prob.M
    s.dt, s.lam = float(prob.dt), float(prob.lam)
    for i, v in enumerate(np.asarray(prob.noise_std, dtype=np.float64)):
        s.noise_std[i] = v
    for i in range(3):
        s.goal[i] = float(prob.goal[i])
        s.w_pos[i] = float(prob.w_pos[i])
    s.w_ang, s.w_vel = float(prob.w_ang), float(prob.w_vel)
    s.obs_kind, s.n_obs = prob.obs_kind, prob.n_obs
    s.obs = keep(_f64(prob.obs).reshape(-1, 3)) if prob.n_obs else None
    s.obs_penalty, s.obs_decay = float(prob.obs_penalty), float(prob.obs_decay)
    s.weighting = prob.weighting
    s.seed, s.problem_id = int(prob.seed) & (2**64 - 1), int(prob.problem_id)
    s.ctrl_cost = int(getattr(prob, "ctrl_cost", 0))
    return s


def max_threads() -> int:
    return int(_load().orc_max_threads())


def philox(counter, key):
    """Philox4x32-10 block: 4 x uint32 counter, 2 x uint32 key -> 4 x uint32."""
    c = np.ascontiguousarray(np.asarray(counter, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, np.uint32)
    _load().orc_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def normals(seed, tag, problem_id, it, k, m, t, n):
    out = np.zeros(n, np.float64)
    _load().orc_normals(int(seed) & (2**64 - 1), tag, problem_id, it, k, m, t, n, _ptr(out))
    return out


def philox_many(ctr, key):
    """Philox blocks of counters ctr [N][4] under one key (2 x uint32)."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(-1, 4))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros_like(c)
    _load().orc_philox_many(c.shape[0], _ptr(c), _ptr(k), _ptr(out))
    return out


def noise_block(prob, tag, it=0, k0=0, nk=None, m=0, n=None):
    """Standard normals of draws (tag, k, m, t): [nk][T][n]."""
    nk = prob.K - k0 if nk is None else nk
    n = (prob.n_u if tag == TAG_CTRL else prob.n_out) if n is None else n
    out = np.zeros((nk, prob.T, n))
    _load().orc_noise_block(int(prob.seed) & (2**64 - 1), tag, prob.problem_id, it, k0, nk, m,
                            prob.T, n, _ptr(out))
    return out


def control_noise(prob, it=0, k0=0, nk=None):
    """eps_{k,t} = sigma_u * N(0, I): [K][T][n_u]."""
    return np.asarray(prob.noise_std, np.float64)[:prob.n_u] * noise_block(prob, TAG_CTRL, it, k0, nk)


def lwpr_predict(model, Z, weights: bool = False, nthreads: int = 0):
    keep = _Keep()
    ms = _model_struct(model, keep)
    Z = _f64(Z).reshape(-1, model.d)
    N = Z.shape[0]
    mean = np.zeros((N, model.n_out))
    var = np.zeros((N, model.n_out))
    W = np.zeros((N, model.Ltot)) if weights else None
    _load().orc_lwpr_predict(C.byref(ms), _ptr(Z), N, _ptr(mean), _ptr(var), _ptr(W), nthreads)
    return (mean, var, W) if weights else (mean, var)


def rollout_cost(prob, model, x0=None, u_nom=None, it: int = 0, k_range=None,
                 states: bool = False, nthreads: int = 0):
    """cbar_{k,t} for k in k_range (default all K); optionally every state."""
    keep = _Keep()
    ms, ps = _model_struct(model, keep), _problem_struct(prob, keep)
    x0 = _f64(prob.x0 if x0 is None else x0)
    u_nom = _f64(prob.u_nom if u_nom is None else u_nom)
    k0, k1 = (0, prob.K) if k_range is None else k_range
    cost = np.zeros((k1 - k0, prob.T))
    Ms = max(prob.M, 1)
    X = np.zeros((k1 - k0, Ms, prob.T + 1, prob.n_x)) if states else None
    _load().orc_rollout_cost(C.byref(ps), C.byref(ms), _ptr(x0), _ptr(u_nom), it, k0, k1,
                             _ptr(cost), _ptr(X), nthreads)
    return (cost, X) if states else cost


def update(prob, cost, u_nom=None, it: int = 0, weights: bool = False):
    """Returns the updated nominal controls (and the [T][K] weights)."""
    keep = _Keep()
    ps = _problem_struct(prob, keep)
    cost = _f64(cost).reshape(prob.K, prob.T)
    u = _f64(prob.u_nom if u_nom is None else u_nom).copy()
    W = np.zeros((prob.T, prob.K)) if weights else None
    _load().orc_update(C.byref(ps), _ptr(cost), it, _ptr(u), _ptr(W))
    return (u, W) if weights else u


def rh_shift(prob, model, x0, u_nom, it: int):
    """Plant step at iteration word `it` and plan shift; returns (x0, u_nom)."""
    keep = _Keep()
    ms, ps = _model_struct(model, keep), _problem_struct(prob, keep)
    x = _f64(x0).copy()
    u = _f64(u_nom).copy()
    itv = C.c_uint32(it)
    _load().orc_rh_shift(C.byref(ps), C.byref(ms), _ptr(x), _ptr(u), C.byref(itv))
    return x, u


def adjoint(prob, model, x0=None, u_nom=None, it: int = 0, nthreads: int = 0):
    """(J, dJ/du_nom [T][n_u], dJ/dc [Ltot][d], dJ/dD [Ltot][d][d])."""
    keep = _Keep()
    ms, ps = _model_struct(model, keep), _problem_struct(prob, keep)
    x0 = _f64(prob.x0 if x0 is None else x0)
    u_nom = _f64(prob.u_nom if u_nom is None else u_nom)
    gu = np.zeros((prob.T, prob.n_u))
    gc = np.zeros((model.Ltot, model.d))
    gD = np.zeros((model.Ltot, model.d, model.d))
    J = _load().orc_adjoint(C.byref(ps), C.byref(ms), _ptr(x0), _ptr(u_nom), it, _ptr(gu),
                            _ptr(gc), _ptr(gD), nthreads)
    return float(J), gu, gc, gD


def iteration(prob, model, it: int = 0, nthreads: int = 0):
    """One PI^2 iteration at iteration word `it`: rollout costs, then the
    update (after which the word advances to it + 1). Returns (cost, u_new)."""
    cost = rollout_cost(prob, model, it=it, nthreads=nthreads)
    return cost, update(prob, cost, it=it)


def rh_loop(prob, model, steps: int, iterations: int = 1, x0=None, u_nom=None, it: int = 0):
    """Receding-horizon loop: per control step `iterations` PI^2 iterations
    (each with its own iteration word), then the plant step and plan shift.
    Returns (x0, u_nom, it) after `steps` control steps."""
    x = _f64(prob.x0 if x0 is None else x0).copy()
    u = _f64(prob.u_nom if u_nom is None else u_nom).copy()
    for _ in range(steps):
        for _ in range(iterations):
            cost = rollout_cost(prob, model, x0=x, u_nom=u, it=it)
            u = update(prob, cost, u_nom=u, it=it)
            it += 1
        x, u = rh_shift(prob, model, x, u, it)
    return x, u, it


def rh_loop_goals(prob, model, steps: int, goals, radius: float = 0.25, iterations: int = 1,
                  g: int = 0, x0=None, u_nom=None, it: int = 0):
    """The receding-horizon loop of the flight experiments (Sec. 5): the state
    cost pulls toward goals[g]; once the plant's position has come within
    `radius` (Euclidean, over the position components) of that point, the
    goal moves to the next point of the cycle.  The controller is not told
    of a switch in advance, so the check follows each control step's plant
    update and takes effect from the next control step.
    Returns (x0, u_nom, it, g) after `steps` control steps."""
    import copy
    from synth import DYN_POINTMASS2D
    goals = np.asarray(goals, dtype=np.float64).reshape(-1, 3)
    npos = 2 if int(prob.dyn) == DYN_POINTMASS2D else 3
    pc = copy.deepcopy(prob)
    x = _f64(prob.x0 if x0 is None else x0).copy()
    u = _f64(prob.u_nom if u_nom is None else u_nom).copy()
    for _ in range(steps):
        pc.goal = goals[g].copy()
        x, u, it = rh_loop(pc, model, 1, iterations=iterations, x0=x, u_nom=u, it=it)
        if np.sqrt(np.sum((x[:npos] - goals[g, :npos]) ** 2)) < radius:
            g = (g + 1) % len(goals)
    return x, u, it, g
