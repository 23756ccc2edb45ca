"""Python binding of the MI355X PI^2-RH library (libpi2rh.so).

Argument marshalling only: every computation runs in the library's gfx950
kernels.  Tensors live on the current HIP device; work is enqueued on
torch's current stream.  If the compiled library is missing this module
raises -- there is no CPU fallback.

Names follow the C ABI (include/pi2rh.h): ``lwpr_predict``, ``rollout_cost``
(pi_rollout_cost), ``update`` (pi_update), ``rh_shift`` (pi_rh_shift),
``rollout_adjoint`` (pi_rollout_adjoint) and the batched rollouts.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpi2rh.so")

PI_F32, PI_F64 = 0, 1
PI_DYN_POINTMASS2D, PI_DYN_QUAD12, PI_DYN_QUAD_HYBRID = 0, 1, 2
PI_OBS_INDICATOR, PI_OBS_SMOOTH = 0, 1
PI_W_COST_TO_GO, PI_W_TRAJECTORY = 0, 1
PI_VARIANT_AUTO, PI_VARIANT_DIRECT, PI_VARIANT_MFMA, PI_VARIANT_MFMA_BF16X3, PI_VARIANT_MFMA_F16X2 = 0, 1, 2, 3, 4
PI_OP_PREDICT, PI_OP_ROLLOUT, PI_OP_UPDATE, PI_OP_ADJOINT, PI_OP_RH_SHIFT = 0, 1, 2, 3, 4
PI_MAX_OUT, PI_MAX_U = 8, 4
STATUS = {0: "PI_OK", 1: "PI_ERR_NULL", 2: "PI_ERR_SHAPE", 3: "PI_ERR_VALUE", 4: "PI_ERR_DTYPE",
          5: "PI_ERR_WORKSPACE", 6: "PI_ERR_DEVICE", 7: "PI_ERR_UNSUPPORTED"}
DYN_DIMS = {PI_DYN_POINTMASS2D: (4, 2, 2), PI_DYN_QUAD12: (12, 4, 6), PI_DYN_QUAD_HYBRID: (9, 4, 3)}
EXPORTED = ["pi_workspace_bytes", "pi_model_fold_bytes", "pi_model_fold", "pi_rollout_describe", "lwpr_predict", "pi_rollout_cost", "pi_rollout_cost_noalloc", "pi_update", "pi_rh_shift",
            "pi_rollout_adjoint", "pi_adjoint_workspace_bytes", "pi_batched_workspace_bytes",
            "pi_rollout_cost_batched", "pi_control_step_batched", "pi_pair_give_ups", "pi_philox4x32_10", "pi_noise",
            "pi_last_error", "pi_version"]
PI_TAG_CTRL, PI_TAG_DYN, PI_TAG_PLANT = 0, 1, 2


class PiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class pi_lwpr(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("d", C.c_int32), ("n_out", C.c_int32), ("R", C.c_int32),
                ("L_off", C.c_int32 * (PI_MAX_OUT + 1)), ("centre", C.c_void_p),
                ("metric", C.c_void_p), ("proj_u", C.c_void_p), ("proj_p", C.c_void_p),
                ("beta", C.c_void_p), ("sigma2", C.c_void_p), ("folded", C.c_void_p),
                ("folded_bytes", C.c_size_t)]


class pi_problem(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("dyn", C.c_int32), ("K", C.c_int32), ("T", C.c_int32),
                ("M", C.c_int32), ("dt", C.c_double), ("lambda_", C.c_double),
                ("noise_std", C.c_double * PI_MAX_U), ("goal", C.c_double * 3),
                ("w_pos", C.c_double * 3), ("w_ang", C.c_double), ("w_vel", C.c_double),
                ("obs_kind", C.c_int32), ("n_obs", C.c_int32), ("obs", C.c_void_p),
                ("obs_penalty", C.c_double), ("obs_decay", C.c_double),
                ("weighting", C.c_int32), ("problem_id", C.c_uint32), ("seed", C.c_uint64),
                ("variant", C.c_int32), ("tile_samples", C.c_int32), ("tile_waves", C.c_int32),
                ("tile_split", C.c_int32), ("ctrl_cost", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Loads libpi2rh.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libpi2rh.so not found at %s: build it with "
                           "`python -m paper_1503_00330_amd.build` (no CPU fallback exists)" % path)
    lib = C.CDLL(path)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    lib.pi_workspace_bytes.argtypes = [i32, vp, vp]
    lib.pi_workspace_bytes.restype = sz
    lib.pi_rollout_describe.argtypes = [vp, vp, vp]
    lib.pi_rollout_describe.restype = i32
    lib.pi_model_fold_bytes.argtypes = [vp]
    lib.pi_model_fold_bytes.restype = sz
    lib.pi_model_fold.argtypes = [vp, vp, sz, vp]
    lib.pi_model_fold.restype = i32
    lib.lwpr_predict.argtypes = [vp, vp, i64, vp, vp, i32, vp, sz, vp]
    lib.pi_rollout_cost.argtypes = [vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.pi_rollout_cost_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.pi_update.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
    lib.pi_rh_shift.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
    lib.pi_rollout_adjoint.argtypes = [vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.pi_adjoint_workspace_bytes.argtypes = [vp, vp, i32]
    lib.pi_adjoint_workspace_bytes.restype = sz
    lib.pi_batched_workspace_bytes.argtypes = [i32, vp, vp]
    lib.pi_batched_workspace_bytes.restype = sz
    lib.pi_rollout_cost_batched.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.pi_control_step_batched.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.pi_pair_give_ups.argtypes = [vp, vp]
    lib.pi_pair_give_ups.restype = i32
    lib.pi_philox4x32_10.argtypes = [vp, C.c_uint64, vp, i64, vp]
    lib.pi_noise.argtypes = [vp, i32, vp, i32, i32, i32, vp, vp]
    lib.pi_last_error.restype = C.c_char_p
    lib.pi_version.restype = C.c_char_p
    for name in ("lwpr_predict", "pi_rollout_cost", "pi_rollout_cost_noalloc", "pi_update", "pi_rh_shift",
                 "pi_rollout_adjoint", "pi_rollout_cost_batched", "pi_control_step_batched",
                 "pi_philox4x32_10", "pi_noise"):
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        raise PiError(status, load().pi_last_error().decode())


def last_error() -> str:
    return load().pi_last_error().decode()


# ----------------------------------------------------------------- helpers

def _torch():
    import torch
    return torch


def _dt(dtype) -> int:
    torch = _torch()
    if dtype in (torch.float32, np.float32):
        return PI_F32
    if dtype in (torch.float64, np.float64):
        return PI_F64
    raise ValueError("unsupported dtype %s" % dtype)


def _tdtype(code: int):
    torch = _torch()
    return torch.float32 if code == PI_F32 else torch.float64


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream() -> int:
    return _torch().cuda.current_stream().cuda_stream


class _Workspace:
    """Grows one device byte buffer per device; reuse keeps graph capture legal
    once the largest size has been reserved."""

    def __init__(self):
        self.buf = {}

    def get(self, nbytes: int, device):
        torch = _torch()
        dev = torch.device(device)
        key = (dev.type, dev.index)
        b = self.buf.get(key)
        if b is None or b.numel() < nbytes:
            b = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=dev)
            self.buf[key] = b
        return b


_ws = _Workspace()


def workspace(nbytes: int, device="cuda"):
    return _ws.get(nbytes, device)


class DeviceModel:
    """An LWPR model (any object with d, n_out, R, L_off, centre, metric,
    proj_u, proj_p, beta, sigma2 arrays) copied to device tensors."""

    def __init__(self, model, device="cuda", dtype=None):
        torch = _torch()
        dtype = dtype or (torch.float32 if np.asarray(model.centre).dtype == np.float32
                          else torch.float64)
        tt = lambda a: None if a is None else torch.as_tensor(np.ascontiguousarray(a), dtype=dtype,
                                                               device=device)
        self.d, self.n_out, self.R = int(model.d), int(model.n_out), int(model.R)
        self.L_off = [int(v) for v in model.L_off]
        self.centre, self.metric = tt(model.centre), tt(model.metric)
        self.proj_u, self.proj_p = tt(model.proj_u), tt(model.proj_p)
        self.beta, self.sigma2 = tt(model.beta), tt(model.sigma2)
        self.dtype = dtype
        self.device = torch.device(device)
        self.folded = None

    @property
    def Ltot(self):
        return self.L_off[-1]

    def fold(self):
        """Folds the model once (pi_model_fold) so that prediction, rollouts and
        the RH shift stop re-folding it on every call.  Call again after
        changing any of the model tensors; unfold() returns to per-call folds."""
        torch = _torch()
        s = self.struct(folded=False)
        lib = load()
        n = lib.pi_model_fold_bytes(C.byref(s))
        if n == C.c_size_t(-1).value:
            raise PiError(PI_ERR_VALUE, last_error())
        if self.folded is None or self.folded.numel() < n:
            self.folded = torch.empty(n, dtype=torch.uint8, device=self.device)
        _check(lib.pi_model_fold(C.byref(s), _ptr(self.folded), self.folded.numel(), _stream()))
        return self

    def unfold(self):
        self.folded = None
        return self

    def struct(self, folded: bool = True) -> pi_lwpr:
        s = pi_lwpr()
        s.dtype = _dt(self.dtype)
        s.d, s.n_out, s.R = self.d, self.n_out, self.R
        for i in range(PI_MAX_OUT + 1):
            s.L_off[i] = self.L_off[min(i, self.n_out)]
        s.centre, s.metric = _ptr(self.centre), _ptr(self.metric)
        s.proj_u, s.proj_p = _ptr(self.proj_u), _ptr(self.proj_p)
        s.beta, s.sigma2 = _ptr(self.beta), _ptr(self.sigma2)
        if folded and self.folded is not None:
            s.folded, s.folded_bytes = _ptr(self.folded), self.folded.numel()
        return s


class DeviceProblem:
    """A PI^2-RH problem: scalar settings (host struct) plus device-resident
    obstacles, start state x0, nominal controls u_nom and the iteration
    counter `iter` (the random stream's iteration word)."""

    def __init__(self, prob, device="cuda", dtype=None, variant: int = PI_VARIANT_AUTO,
                 tile_samples: int = 0, tile_waves: int = 0, tile_split: int = 0):
        torch = _torch()
        dtype = dtype or (torch.float32 if np.asarray(prob.x0).dtype == np.float32
                          else torch.float64)
        self.dtype, self.device = dtype, torch.device(device)
        self.prob = prob
        self.dyn, self.K, self.T, self.M = int(prob.dyn), int(prob.K), int(prob.T), int(prob.M)
        self.n_x, self.n_u, self.n_out = DYN_DIMS[self.dyn]
        self.obs = torch.as_tensor(np.ascontiguousarray(prob.obs, dtype=np.float64).reshape(-1, 3),
                                   dtype=dtype, device=device)
        self.x0 = torch.as_tensor(np.asarray(prob.x0), dtype=dtype, device=device).clone()
        self.u_nom = torch.as_tensor(np.asarray(prob.u_nom), dtype=dtype, device=device).clone()
        self.iter = torch.zeros(1, dtype=torch.int32, device=device)
        self.variant, self.tile_samples, self.tile_waves = variant, tile_samples, tile_waves
        self.tile_split = tile_split

    def struct(self) -> pi_problem:
        p, s = self.prob, pi_problem()
        s.dtype, s.dyn = _dt(self.dtype), self.dyn
        s.K, s.T, s.M = self.K, self.T, self.M
        s.dt, s.lambda_ = float(p.dt), float(p.lam)
        ns = np.asarray(p.noise_std, dtype=np.float64)
        for a in range(PI_MAX_U):
            s.noise_std[a] = float(ns[a]) if a < ns.size else 0.0
        for a in range(3):
            s.goal[a], s.w_pos[a] = float(p.goal[a]), float(p.w_pos[a])
        s.w_ang, s.w_vel = float(p.w_ang), float(p.w_vel)
        s.obs_kind, s.n_obs = int(p.obs_kind), int(self.obs.shape[0])
        s.obs = _ptr(self.obs) if s.n_obs else None
        s.obs_penalty, s.obs_decay = float(p.obs_penalty), float(p.obs_decay)
        s.weighting = int(p.weighting)
        s.problem_id = int(p.problem_id) & 0xFFFFFFFF
        s.seed = int(p.seed) & 0xFFFFFFFFFFFFFFFF
        s.variant, s.tile_samples = int(self.variant), int(self.tile_samples)
        s.tile_waves = int(self.tile_waves)
        s.tile_split = int(self.tile_split)
        s.ctrl_cost = int(getattr(p, "ctrl_cost", 0))
        return s


def workspace_bytes(op: int, prob: Optional[DeviceProblem], model: Optional[DeviceModel]) -> int:
    ps = prob.struct() if prob is not None else None
    ms = model.struct() if model is not None else None
    n = load().pi_workspace_bytes(op, C.byref(ps) if ps is not None else None,
                                  C.byref(ms) if ms is not None else None)
    if n == C.c_size_t(-1).value:
        raise PiError(2, last_error())
    return int(n)


# ------------------------------------------------------------ entry points

def lwpr_predict(model: DeviceModel, Z, variant: int = PI_VARIANT_AUTO, out=None):
    """Eq. (1) mixture mean and variance of every output at inputs Z [N][d]."""
    torch = _torch()
    lib = load()
    Z = Z.contiguous()
    N = int(Z.shape[0])
    mean, var = out if out is not None else (
        torch.empty((N, model.n_out), dtype=model.dtype, device=Z.device),
        torch.empty((N, model.n_out), dtype=model.dtype, device=Z.device))
    ms = model.struct()
    nb = workspace_bytes(PI_OP_PREDICT, None, model)
    ws = workspace(nb, Z.device)
    _check(lib.lwpr_predict(C.byref(ms), _ptr(Z), N, _ptr(mean), _ptr(var), variant, _ptr(ws),
                            ws.numel(), _stream()))
    return mean, var


def rollout_describe(prob: DeviceProblem, model: DeviceModel) -> dict:
    """The launch pi_rollout_cost makes for this problem on the current device."""
    out = (C.c_int32 * 4)()
    ps, ms = prob.struct(), model.struct()
    _check(load().pi_rollout_describe(C.byref(ps), C.byref(ms), out))
    mfma = out[0] in (PI_VARIANT_MFMA, PI_VARIANT_MFMA_BF16X3, PI_VARIANT_MFMA_F16X2)
    return {"variant": {PI_VARIANT_MFMA: "mfma", PI_VARIANT_MFMA_BF16X3: "mfma-bf16x3",
                        PI_VARIANT_MFMA_F16X2: "mfma-f16x2"}.get(out[0], "direct"),
            "tile_samples": out[1], "tile_waves": out[2], "tile_split": out[3],
            "kernel": ("rollout_pair_kernel" if out[3] == 2 else "rollout_mfma_kernel")
            if mfma else "rollout_direct_kernel"}


def rollout_cost(prob: DeviceProblem, model: DeviceModel, x0=None, u_nom=None, iter=None,
                 out=None):
    """cbar_{k,t} [K][T] of the sampled rollouts from x0 under u_nom."""
    torch = _torch()
    lib = load()
    x0 = prob.x0 if x0 is None else x0
    u_nom = prob.u_nom if u_nom is None else u_nom
    it = prob.iter if iter is None else iter
    cost = out if out is not None else torch.empty((prob.K, prob.T), dtype=prob.dtype,
                                                   device=x0.device)
    ps, ms = prob.struct(), model.struct()
    ws = workspace(workspace_bytes(PI_OP_ROLLOUT, prob, model), x0.device)
    _check(lib.pi_rollout_cost(C.byref(ps), C.byref(ms), _ptr(x0), _ptr(u_nom), _ptr(it),
                               _ptr(cost), _ptr(ws), ws.numel(), _stream()))
    return cost


def rollout_cost_noalloc(prob: DeviceProblem, model: DeviceModel, x0=None, u_nom=None, iter=None,
                         out=None):
    """rollout_cost through pi_rollout_cost_noalloc: no workspace, the library's
    static per-device scratch instead (pass `out` to allocate nothing here)."""
    torch = _torch()
    x0 = prob.x0 if x0 is None else x0
    u_nom = prob.u_nom if u_nom is None else u_nom
    it = prob.iter if iter is None else iter
    cost = out if out is not None else torch.empty((prob.K, prob.T), dtype=prob.dtype,
                                                   device=x0.device)
    ps, ms = prob.struct(), model.struct()
    _check(load().pi_rollout_cost_noalloc(C.byref(ps), C.byref(ms), _ptr(x0), _ptr(u_nom), _ptr(it),
                                          _ptr(cost), _stream()))
    return cost


def update(prob: DeviceProblem, cost, u_nom=None, iter=None, weights: bool = False):
    """Eq. (2): updates u_nom in place and advances iter; returns (u_nom, weights [T][K] or None)."""
    torch = _torch()
    lib = load()
    u_nom = prob.u_nom if u_nom is None else u_nom
    it = prob.iter if iter is None else iter
    W = torch.empty((prob.T, prob.K), dtype=torch.float64, device=u_nom.device) if weights else None
    ps = prob.struct()
    ws = workspace(workspace_bytes(PI_OP_UPDATE, prob, None), u_nom.device)
    _check(lib.pi_update(C.byref(ps), _ptr(cost.contiguous()), _ptr(it), _ptr(u_nom), _ptr(W),
                         _ptr(ws), ws.numel(), _stream()))
    return u_nom, W


def rh_shift(prob: DeviceProblem, model: DeviceModel, x0=None, u_nom=None, iter=None):
    """Executes u_nom[0] on the sampled plant and shifts the plan (in place)."""
    lib = load()
    x0 = prob.x0 if x0 is None else x0
    u_nom = prob.u_nom if u_nom is None else u_nom
    it = prob.iter if iter is None else iter
    ps, ms = prob.struct(), model.struct()
    ws = workspace(workspace_bytes(PI_OP_RH_SHIFT, prob, model), x0.device)
    _check(lib.pi_rh_shift(C.byref(ps), C.byref(ms), _ptr(x0), _ptr(u_nom), _ptr(it), _ptr(ws),
                           ws.numel(), _stream()))
    return x0, u_nom, it


def iteration(prob: DeviceProblem, model: DeviceModel, cost=None):
    """One PI^2 iteration on the device: rollouts, then the update of u_nom."""
    cost = rollout_cost(prob, model, out=cost)
    update(prob, cost)
    return cost


class BatchedRollout:
    """Many independent problems in one persistent launch: run() gives every
    problem's rollout costs (pi_rollout_cost_batched); control_step() runs
    their rollouts, updates and receding-horizon advances
    (pi_control_step_batched).  The struct arrays and the pointer arrays are
    built here once; the problems' tensors (x0, u_nom, iter, costs) are
    updated in place, so a call can be captured into a HIP graph (capture())
    and replayed."""

    def __init__(self, problems, models, costs=None):
        torch = _torch()
        lib = load()
        self.problems, self.models = list(problems), list(models)
        B = self.B = len(self.problems)
        self.ps = (pi_problem * B)(*[p.struct() for p in self.problems])
        self.ms = (pi_lwpr * B)(*[m.struct() for m in self.models])
        dev = self.problems[0].device
        self.costs = costs if costs is not None else [
            torch.empty((p.K, p.T), dtype=torch.float32, device=dev) for p in self.problems]
        nws = lib.pi_batched_workspace_bytes(B, self.ps, self.ms)
        if nws == C.c_size_t(-1).value:
            raise PiError(2, last_error())
        self.ws = torch.empty(max(int(nws), 256), dtype=torch.uint8, device=dev)
        arr = lambda xs: (C.c_void_p * B)(*[int(x) for x in xs])
        self.x0 = arr(p.x0.data_ptr() for p in self.problems)
        self.u_nom = arr(p.u_nom.data_ptr() for p in self.problems)
        self.iter = arr(p.iter.data_ptr() for p in self.problems)
        self.cost_ptrs = arr(c.data_ptr() for c in self.costs)
        self.graph = None

    def run(self):
        _check(load().pi_rollout_cost_batched(self.B, self.ps, self.ms, self.x0, self.u_nom, self.iter,
                                              self.cost_ptrs, self.ws.data_ptr(), self.ws.numel(), _stream()))
        return self.costs

    def control_step(self):
        _check(load().pi_control_step_batched(self.B, self.ps, self.ms, self.x0, self.u_nom, self.iter,
                                              self.cost_ptrs, self.ws.data_ptr(), self.ws.numel(), _stream()))

    def capture(self):
        """Records one batched control step into a HIP graph (state not advanced)."""
        torch = _torch()
        saved = [(p.x0.clone(), p.u_nom.clone(), p.iter.clone()) for p in self.problems]
        self.control_step()           # per-device checks before capture
        torch.cuda.synchronize()
        for p, (x, u, it) in zip(self.problems, saved):
            p.x0.copy_(x)
            p.u_nom.copy_(u)
            p.iter.copy_(it)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                self.control_step()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = g
        return g

    def step(self, graph: bool = True):
        """One batched control step (graph replay unless graph=False)."""
        if not graph:
            self.control_step()
            return
        if self.graph is None:
            self.capture()
        self.graph.replay()


def rollout_adjoint(prob: DeviceProblem, model: DeviceModel, x0=None, u_nom=None, iter=None,
                    ckpt_every: int = 0, gJ=None):
    """J and the gradients of gJ * J w.r.t. (u_nom, centres, metrics) of the
    expected rollout cost with the noise held fixed (pi_rollout_adjoint);
    gJ: optional device double scalar seed (None = 1)."""
    torch = _torch()
    lib = load()
    x0 = prob.x0 if x0 is None else x0
    u_nom = (prob.u_nom if u_nom is None else u_nom).contiguous()
    it = prob.iter if iter is None else iter
    dev = x0.device
    J = torch.empty(1, dtype=torch.float64, device=dev)
    gu = torch.empty_like(u_nom)
    gc = torch.empty_like(model.centre)
    gD = torch.empty_like(model.metric)
    ps, ms = prob.struct(), model.struct()
    need = lib.pi_adjoint_workspace_bytes(C.byref(ps), C.byref(ms), int(ckpt_every))
    if need == C.c_size_t(-1).value:
        raise PiError(2, last_error())
    ws = workspace(int(need), dev)
    if gJ is not None:
        gJ = gJ.to(device=dev, dtype=torch.float64).reshape(1).contiguous()
    _check(lib.pi_rollout_adjoint(C.byref(ps), C.byref(ms), _ptr(x0), _ptr(u_nom), _ptr(it), int(ckpt_every),
                                  _ptr(gJ), _ptr(J), _ptr(gu), _ptr(gc), _ptr(gD), _ptr(ws), ws.numel(),
                                  _stream()))
    return J, gu, gc, gD


def pair_give_ups() -> int:
    """Paired-rollout workgroups that abandoned their tile on the current
    device so far (pi_pair_give_ups); synchronises the current stream."""
    torch = _torch()
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    _check(load().pi_pair_give_ups(_ptr(out), _stream()))
    return int(out.item())


def philox4x32_10(ctr, key: int):
    """Raw Philox4x32-10 blocks for uint32 counters ctr [N][4] (a device int32 tensor)."""
    torch = _torch()
    ctr = ctr.contiguous()
    out = torch.empty_like(ctr)
    _check(load().pi_philox4x32_10(_ptr(ctr), int(key) & 0xFFFFFFFFFFFFFFFF, _ptr(out),
                                   int(ctr.shape[0]), _stream()))
    return out


def noise(prob: DeviceProblem, tag: int, k0: int = 0, nk: Optional[int] = None, m: int = 0,
          iter=None):
    """The draws of stream `tag` exactly as the kernels form them (see pi_noise)."""
    torch = _torch()
    nk = prob.K - k0 if nk is None else nk
    it = prob.iter if iter is None else iter
    if tag == PI_TAG_PLANT:
        out = torch.empty(prob.n_out, dtype=prob.dtype, device=prob.device)
    else:
        n = prob.n_u if tag == PI_TAG_CTRL else prob.n_out
        out = torch.empty((nk, prob.T, n), dtype=prob.dtype, device=prob.device)
    ps = prob.struct()
    _check(load().pi_noise(C.byref(ps), tag, _ptr(it), k0, nk, m, _ptr(out), _stream()))
    return out


def version() -> str:
    return load().pi_version().decode()
