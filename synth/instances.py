"""Synthetic PI^2-RH instances: LWPR models, problems and the benchmark configs.

Everything is drawn in FP64 with numpy's PCG64 and rounded once to the run
dtype (``astype``), so that a float32 GPU run and the FP64 oracle read
bit-identical parameter values.  Distributions follow the workload recipe:

* centres c_j ~ U[-1, 1]^d;
* metrics D_j = A A^T + 0.5 I with A_ab ~ N(0, 0.09) (variance 0.09);
* PLS projection directions u_{j,r}: random unit vectors; loadings p = u;
* regression coefficients beta_{j,0..R} ~ N(0, 1);
* local noise sigma_j ~ U[0.01, 0.1] (stored as sigma_j^2);
* start position and goal ~ U[-1, 1]^{2 or 3}, all velocities, angles and
  rates zero; obstacle centres ~ U[-1, 1]^2 with radius 0.2, redrawn when the
  start or the goal lies inside.

LWPR input is z = [state ; control] for the point mass and the 12-state
quadrotor; the hybrid quadrotor follows Sec. 4.1 (three models of the euler
angles and the thrust give the cartesian accelerations, the angles follow
their commanded rates).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

DYN_POINTMASS2D = 0   # state [px, py, vx, vy], control [ax, ay]
DYN_QUAD12 = 1        # state [p(3), v(3), euler(3), rates(3)], control [thrust, 3 torques]
DYN_QUAD_HYBRID = 2   # state [p(3), v(3), euler(3)], control [commanded rates(3), thrust]
# dyn -> (n_x, n_u, n_out)
DYN_DIMS = {DYN_POINTMASS2D: (4, 2, 2), DYN_QUAD12: (12, 4, 6), DYN_QUAD_HYBRID: (9, 4, 3)}
# dyn -> LWPR input size d
DYN_D = {DYN_POINTMASS2D: 6, DYN_QUAD12: 16, DYN_QUAD_HYBRID: 4}

OBS_INDICATOR = 0
OBS_SMOOTH = 1
W_COST_TO_GO = 0
W_TRAJECTORY = 1


@dataclass
class LWPRModel:
    """n_out independent LWPR mixtures over one input z in R^d.

    Models of output o are rows L_off[o] .. L_off[o+1]-1 of every array.
    """
    d: int
    n_out: int
    R: int
    L_off: np.ndarray          # int64 [n_out+1]
    centre: np.ndarray         # [Ltot, d]
    metric: np.ndarray         # [Ltot, d, d]
    proj_u: np.ndarray         # [Ltot, R, d]
    proj_p: Optional[np.ndarray]  # [Ltot, R, d] or None (p = u)
    beta: np.ndarray           # [Ltot, R+1]
    sigma2: np.ndarray         # [Ltot]

    @property
    def Ltot(self) -> int:
        return int(self.L_off[-1])

    @property
    def dtype(self):
        return self.centre.dtype

    def astype(self, dtype) -> "LWPRModel":
        cv = lambda a: None if a is None else np.ascontiguousarray(a.astype(dtype))
        return dataclasses.replace(
            self, centre=cv(self.centre), metric=cv(self.metric), proj_u=cv(self.proj_u),
            proj_p=cv(self.proj_p), beta=cv(self.beta), sigma2=cv(self.sigma2),
            L_off=np.ascontiguousarray(self.L_off.astype(np.int64)))

    def copy(self) -> "LWPRModel":
        cp = lambda a: None if a is None else a.copy()
        return dataclasses.replace(
            self, centre=cp(self.centre), metric=cp(self.metric), proj_u=cp(self.proj_u),
            proj_p=cp(self.proj_p), beta=cp(self.beta), sigma2=cp(self.sigma2),
            L_off=self.L_off.copy())


@dataclass
class Problem:
    """One PI^2-RH instance: dynamics kind, sampling sizes, cost and RNG key."""
    dyn: int
    K: int
    T: int
    M: int                      # 0: mean-only rollouts; >= 1: M sampled sub-rollouts
    dt: float
    lam: float
    noise_std: np.ndarray       # [n_u] control noise std
    goal: np.ndarray            # [3]
    w_pos: np.ndarray           # [3]
    w_ang: float
    w_vel: float
    obs_kind: int
    obs: np.ndarray             # [n_obs, 3] (cx, cy, r)
    obs_penalty: float
    obs_decay: float
    weighting: int
    seed: int
    problem_id: int
    x0: np.ndarray              # [n_x]
    u_nom: np.ndarray           # [T, n_u]
    dtype: type = np.float64
    ctrl_cost: int = 0          # 1: the control terms of the cost-to-go (hybrid model only)

    @property
    def n_x(self):
        return DYN_DIMS[self.dyn][0]

    @property
    def n_u(self):
        return DYN_DIMS[self.dyn][1]

    @property
    def n_out(self):
        return DYN_DIMS[self.dyn][2]

    @property
    def d(self):
        return self.n_x + self.n_u

    @property
    def n_obs(self):
        return int(self.obs.shape[0])

    def astype(self, dtype) -> "Problem":
        return dataclasses.replace(
            self, x0=np.ascontiguousarray(self.x0.astype(dtype)),
            u_nom=np.ascontiguousarray(self.u_nom.astype(dtype)), dtype=dtype)

    def copy(self) -> "Problem":
        return dataclasses.replace(self, x0=self.x0.copy(), u_nom=self.u_nom.copy(),
                                   noise_std=self.noise_std.copy(), goal=self.goal.copy(),
                                   w_pos=self.w_pos.copy(), obs=self.obs.copy())


def _unit_rows(rng, shape):
    v = rng.standard_normal(shape)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def make_lwpr(rng: np.random.Generator, d: int, L: Sequence[int] | int, R: int,
              n_out: Optional[int] = None, loadings_equal_u: bool = True,
              metric_ridge: float = 0.5, metric_a_var: float = 0.09) -> LWPRModel:
    """Draws an LWPR model with the recipe in the module docstring (FP64)."""
    if isinstance(L, (int, np.integer)):
        assert n_out is not None
        Ls = [int(L)] * n_out
    else:
        Ls = [int(x) for x in L]
        n_out = len(Ls)
    L_off = np.concatenate([[0], np.cumsum(Ls)]).astype(np.int64)
    Lt = int(L_off[-1])
    centre = rng.uniform(-1.0, 1.0, (Lt, d))
    A = rng.normal(0.0, np.sqrt(metric_a_var), (Lt, d, d))
    metric = A @ np.transpose(A, (0, 2, 1)) + metric_ridge * np.eye(d)[None]
    metric = 0.5 * (metric + np.transpose(metric, (0, 2, 1)))
    proj_u = _unit_rows(rng, (Lt, R, d))
    proj_p = None if loadings_equal_u else _unit_rows(rng, (Lt, R, d))
    beta = rng.standard_normal((Lt, R + 1))
    sigma2 = rng.uniform(0.01, 0.1, Lt) ** 2
    return LWPRModel(d=d, n_out=n_out, R=R, L_off=L_off, centre=centre, metric=metric,
                     proj_u=proj_u, proj_p=proj_p, beta=beta, sigma2=sigma2)


def _obstacles(rng, n_obs, radius, avoid: List[np.ndarray]):
    obs = np.zeros((n_obs, 3))
    for i in range(n_obs):
        while True:
            c = rng.uniform(-1.0, 1.0, 2)
            if all(np.sum((p[:2] - c) ** 2) >= radius * radius for p in avoid):
                break
        obs[i, :2] = c
        obs[i, 2] = radius
    return obs


def make_problem(rng: np.random.Generator, dyn: int, K: int, T: int, M: int = 1,
                 dt: float = 0.02, lam: float = 1.0, noise_std: float = 0.5,
                 n_obs: int = 3, radius: float = 0.2, obs_kind: int = OBS_INDICATOR,
                 obs_penalty: Optional[float] = None, obs_decay: float = 10.0,
                 weighting: int = W_COST_TO_GO, seed: int = 0xC0FFEE00,
                 problem_id: int = 0) -> Problem:
    n_x, n_u, n_out = DYN_DIMS[dyn]
    npos = 2 if dyn == DYN_POINTMASS2D else 3
    x0 = np.zeros(n_x)
    x0[:npos] = rng.uniform(-1.0, 1.0, npos)
    goal = np.zeros(3)
    goal[:npos] = rng.uniform(-1.0, 1.0, npos)
    obs = _obstacles(rng, n_obs, radius, [x0[:npos], goal[:npos]])
    if dyn == DYN_POINTMASS2D:
        w_pos, w_ang, w_vel = np.array([1.0, 1.0, 0.0]), 0.0, 0.0
    else:  # state cost weights of the quadrotor task (Sec. 5)
        w_pos, w_ang, w_vel = np.array([1.0, 1.0, 10.0]), 0.2, 0.1
    if obs_penalty is None:
        obs_penalty = 1000.0 if obs_kind == OBS_INDICATOR else 100.0
    return Problem(dyn=dyn, K=K, T=T, M=M, dt=dt, lam=lam,
                   noise_std=np.full(n_u, float(noise_std)), goal=goal, w_pos=w_pos,
                   w_ang=w_ang, w_vel=w_vel, obs_kind=obs_kind, obs=obs,
                   obs_penalty=float(obs_penalty), obs_decay=float(obs_decay),
                   weighting=weighting, seed=int(seed), problem_id=int(problem_id),
                   x0=x0, u_nom=np.zeros((T, n_u)))


def config(cfg: int, dtype=None, K: Optional[int] = None, T: Optional[int] = None,
           obs_kind: int = OBS_INDICATOR):
    """The five benchmark workloads (configs 0-2 and 4; 3 is `batched_config`).

    Returns (problem, model, extra) with extra = dict(rh_steps=..., ckpt=...).
    ``K``/``T`` override the sample count / horizon (e.g. a bounded CPU sample).
    """
    rng = np.random.Generator(np.random.PCG64(1000 + cfg))
    seed = 0xC0FFEE00 + cfg
    extra = {}
    if cfg == 0:
        dt = np.float64
        model = make_lwpr(rng, 6, 16, 2, n_out=2)
        prob = make_problem(rng, DYN_POINTMASS2D, 256, 20, M=1, n_obs=3, seed=seed,
                            obs_kind=obs_kind)
        extra.update(rh_steps=1)
    elif cfg in (1, 2, 4):
        dt = np.float32
        L = {1: 256, 2: 1024, 4: 256}[cfg]
        Kc = {1: 2048, 2: 65536, 4: 8192}[cfg]
        Tc = {1: 100, 2: 200, 4: 400}[cfg]
        model = make_lwpr(rng, 16, L, 4, n_out=6)
        prob = make_problem(rng, DYN_QUAD12, Kc, Tc, M=1, n_obs=20, seed=seed,
                            obs_kind=obs_kind)
        extra.update(rh_steps={1: 10, 2: 50, 4: 1}[cfg], ckpt=20 if cfg == 4 else 0)
    else:
        raise ValueError("config %d has no single-problem form" % cfg)
    if dtype is None:
        dtype = dt
    if K is not None:
        prob.K = int(K)
    if T is not None:
        prob.T = int(T)
        prob.u_nom = np.zeros((prob.T, prob.n_u))
    return prob.astype(dtype), model.astype(dtype), extra


def batched_config(dtype=np.float32, B: int = 64, K_range=(512, 16384), L_range=(64, 1024),
                   T_range=(50, 200), obs_range=(10, 40), seed_base: int = 0xC0FFEE03):
    """B independent quadrotor problems with uneven K, L, T and obstacle counts."""
    rng = np.random.Generator(np.random.PCG64(1003))
    out = []
    for b in range(B):
        K = int(rng.integers(K_range[0], K_range[1] + 1))
        L = int(rng.integers(L_range[0], L_range[1] + 1))
        T = int(rng.integers(T_range[0], T_range[1] + 1))
        n_obs = int(rng.integers(obs_range[0], obs_range[1] + 1))
        model = make_lwpr(rng, 16, L, 4, n_out=6)
        prob = make_problem(rng, DYN_QUAD12, K, T, M=1, n_obs=n_obs, seed=seed_base,
                            problem_id=b)
        out.append((prob.astype(dtype), model.astype(dtype)))
    return out


def paper_shape(M: int = 1, K: int = 1000, T: int = 50, dtype=np.float32, seed: int = 7,
                R: int = 2):
    """The paper's own model and GPU timing shapes (Sec. 4, 4.1): the hybrid
    quadrotor whose three LWPR models (15, 15 and 24 local models) map the euler
    angles and the thrust (d = 4) to the cartesian accelerations, 1000 rollouts
    of 50 steps and M sub-rollouts (M = 0: mean prediction only)."""
    rng = np.random.Generator(np.random.PCG64(2000 + seed))
    model = make_lwpr(rng, DYN_D[DYN_QUAD_HYBRID], [15, 15, 24], R)
    prob = make_problem(rng, DYN_QUAD_HYBRID, K, T, M=M, n_obs=3, obs_kind=OBS_SMOOTH,
                        seed=0xC0FFEE10 + seed)
    return prob.astype(dtype), model.astype(dtype)


def tiny_problem(seed: int = 0, dyn: int = DYN_POINTMASS2D, L=3, R: int = 2, K: int = 5,
                 T: int = 4, M: int = 1, dtype=np.float64, **kw):
    """Small instance for pins and quick parity checks."""
    rng = np.random.Generator(np.random.PCG64(5000 + seed))
    n_x, n_u, n_out = DYN_DIMS[dyn]
    model = make_lwpr(rng, DYN_D[dyn], L, R, n_out=n_out)
    prob = make_problem(rng, dyn, K, T, M=M, seed=0xC0FFEE00 + 97 * seed, **kw)
    prob.u_nom = rng.normal(0.0, 0.3, (T, n_u))
    return prob.astype(dtype), model.astype(dtype)
