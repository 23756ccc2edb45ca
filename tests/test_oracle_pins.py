"""Pins of the FP64 oracle against facts other than itself.

Each test checks the oracle against an independent source: another Philox
implementation (ROCm's rocRAND engine), a library regression (scikit-learn's
PLS), a Gaussian density (SciPy), closed forms of special cases (a single
affine model gives linear dynamics; K = 1 gives delta u = eps), statistics, and
finite differences of the oracle's own forward pass for its adjoint.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle
import synth
from synth import DYN_POINTMASS2D, DYN_QUAD12, DYN_QUAD_HYBRID, OBS_SMOOTH, W_TRAJECTORY

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ Philox

@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_philox_ref")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1",
                           os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", exe])
    return exe


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(11)
    n = 4000
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64)
    ctr[:, 1] %= 2**29  # keeps rocRAND's 4*offset inside 64 bits
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64)
    ctr[:8] = 0
    key[:4] = 0
    ctr[8:16] = 2**32 - 1
    ctr[8:16, 1] = 2**29 - 1
    lines = "\n".join(" ".join(str(int(v)) for v in list(c) + list(k)) for c, k in zip(ctr, key))
    out = subprocess.run([rocrand_ref], input=lines + "\n", capture_output=True, text=True,
                         check=True).stdout.split()
    ref = np.array(out, dtype=np.uint64).reshape(n, 4)
    mine = np.stack([oracle.philox(c.astype(np.uint32), k.astype(np.uint32))
                     for c, k in zip(ctr, key)]).astype(np.uint64)
    assert np.array_equal(mine, ref)


def test_normals_statistics():
    # 2^17 normals from counters that sweep t and k: mean 0, variance 1, KS vs N(0,1)
    vals = []
    for k in range(256):
        for t in range(128):
            vals.append(oracle.normals(0xC0FFEE00, oracle.TAG_CTRL, 0, 0, k, 0, t, 4))
    x = np.concatenate(vals)
    n = x.size
    assert abs(x.mean()) < 5.0 / np.sqrt(n)
    assert abs(x.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert stats.kstest(x, "norm").pvalue > 1e-3
    # the four normals of one block are independent: correlation ~ 0
    b = x.reshape(-1, 4)
    c = np.corrcoef(b.T)
    assert np.all(np.abs(c - np.eye(4)) < 5.0 / np.sqrt(b.shape[0]))


def test_streams_are_distinct():
    a = oracle.normals(1, oracle.TAG_CTRL, 0, 0, 3, 0, 5, 8)
    assert not np.allclose(a, oracle.normals(1, oracle.TAG_DYN, 0, 0, 3, 0, 5, 8))
    assert not np.allclose(a, oracle.normals(1, oracle.TAG_CTRL, 1, 0, 3, 0, 5, 8))
    assert not np.allclose(a, oracle.normals(1, oracle.TAG_CTRL, 0, 1, 3, 0, 5, 8))
    assert not np.allclose(a, oracle.normals(1, oracle.TAG_CTRL, 0, 0, 3, 1, 5, 8))
    assert not np.allclose(a, oracle.normals(2, oracle.TAG_CTRL, 0, 0, 3, 0, 5, 8))
    # normals 4..7 come from the next counter block, not a repeat of 0..3
    assert not np.allclose(a[:4], a[4:])


# ------------------------------------------------------------------ LWPR, Eq. (1)

def _model(seed=0, d=5, L=(7, 4), R=2, **kw):
    rng = np.random.default_rng(100 + seed)
    return synth.make_lwpr(rng, d, list(L), R, **kw)


def _single(model, j):
    """The LWPR model made of local model j alone (its mean is y_j(z))."""
    m = model.copy()
    sl = slice(j, j + 1)
    m.n_out = 1
    m.L_off = np.array([0, 1], np.int64)
    m.centre, m.metric, m.proj_u = m.centre[sl], m.metric[sl], m.proj_u[sl]
    m.proj_p = None if m.proj_p is None else m.proj_p[sl]
    m.beta, m.sigma2 = m.beta[sl], m.sigma2[sl]
    return m


def test_weights_sum_to_one_and_match_gaussian_density():
    model = _model(1, d=4, L=(6,), R=2)
    Z = np.random.default_rng(3).uniform(-1, 1, (20, 4))
    _, _, W = oracle.lwpr_predict(model, Z, weights=True)
    assert np.allclose(W.sum(1), 1.0, atol=1e-15, rtol=0)
    # w_j is proportional to a Gaussian density with covariance D_j^{-1},
    # rescaled by sqrt(det(2 pi D_j^{-1}))
    for n, z in enumerate(Z):
        raw = []
        for j in range(model.Ltot):
            cov = np.linalg.inv(model.metric[j])
            pdf = stats.multivariate_normal(mean=model.centre[j], cov=cov).pdf(z)
            raw.append(pdf * np.sqrt(np.linalg.det(2 * np.pi * cov)))
        raw = np.array(raw)
        assert np.allclose(W[n], raw / raw.sum(), rtol=1e-10, atol=1e-300)


def test_single_model_is_affine_with_its_own_variance():
    model = _model(2, d=5, L=(1,), R=3)
    rng = np.random.default_rng(4)
    z1, z2 = rng.uniform(-1, 1, (2, 5))
    for a in (0.0, 0.3, 1.7):
        mu, v = oracle.lwpr_predict(model, (a * z1 + (1 - a) * z2)[None])
        mu1, _ = oracle.lwpr_predict(model, z1[None])
        mu2, _ = oracle.lwpr_predict(model, z2[None])
        assert np.allclose(mu, a * mu1 + (1 - a) * mu2, rtol=1e-12, atol=1e-12)
        assert np.allclose(v, model.sigma2[0], rtol=1e-14)
    # at the centre the prediction is the offset beta_0
    mu, _ = oracle.lwpr_predict(model, model.centre[:1])
    assert np.isclose(mu[0, 0], model.beta[0, 0], rtol=1e-14)


@pytest.mark.parametrize("R", [1, 3, 5])
def test_local_model_matches_sklearn_pls(R):
    from sklearn.cross_decomposition import PLSRegression
    rng = np.random.default_rng(5 + R)
    d = 5
    X = rng.normal(size=(80, d))
    y = X @ rng.normal(size=d) + 0.3 * np.sin(X[:, 0]) + 0.05 * rng.normal(size=80)
    pls = PLSRegression(n_components=R, scale=False).fit(X, y)
    model = _model(0, d=d, L=(1,), R=R)
    model.centre = pls._x_mean[None].copy()
    model.proj_u = pls.x_weights_.T[None].copy()
    model.proj_p = pls.x_loadings_.T[None].copy()
    model.beta = np.concatenate([[float(np.ravel(pls._y_mean)[0])],
                                 pls.y_loadings_.ravel()])[None]
    Zq = rng.normal(size=(25, d))
    mu, _ = oracle.lwpr_predict(model, Zq)
    assert np.allclose(mu[:, 0], np.ravel(pls.predict(Zq)), rtol=1e-10, atol=1e-12)


def test_full_rank_orthonormal_projections_reduce_to_linear_model():
    # R = d with orthonormal directions and p = u: deflation changes nothing
    d = 4
    model = _model(3, d=d, L=(1,), R=d)
    Q, _ = np.linalg.qr(np.random.default_rng(9).normal(size=(d, d)))
    model.proj_u = Q.T[None].copy()
    model.proj_p = None
    z = np.random.default_rng(10).uniform(-1, 1, (6, d))
    mu, _ = oracle.lwpr_predict(model, z)
    expect = model.beta[0, 0] + ((z - model.centre[0]) @ Q) @ model.beta[0, 1:]
    assert np.allclose(mu[:, 0], expect, rtol=1e-12, atol=1e-13)


def test_equal_weights_and_mixture_moments():
    # D = 0: every model gets weight 1/L, so the mean is the plain average of
    # the single-model means and the variance is the mixture variance.
    model = _model(4, d=3, L=(5,), R=2)
    model.metric[:] = 0.0
    z = np.random.default_rng(12).uniform(-1, 1, (3, 3))
    mu, v, W = oracle.lwpr_predict(model, z, weights=True)
    assert np.allclose(W, 0.2, atol=1e-15)
    ys = np.stack([oracle.lwpr_predict(_single(model, j), z)[0][:, 0] for j in range(5)], 1)
    assert np.allclose(mu[:, 0], ys.mean(1), rtol=1e-13)
    mix_var = (ys ** 2 + model.sigma2[None]).mean(1) - ys.mean(1) ** 2
    assert np.allclose(v[:, 0], mix_var, rtol=1e-11)


def test_variance_is_the_mixture_variance_monte_carlo():
    model = _model(5, d=3, L=(6,), R=2)
    model.sigma2[:] = np.linspace(0.05, 0.4, 6) ** 2
    z = np.array([[0.2, -0.1, 0.4]])
    mu, v, W = oracle.lwpr_predict(model, z, weights=True)
    ys = np.array([oracle.lwpr_predict(_single(model, j), z)[0][0, 0] for j in range(6)])
    rng = np.random.default_rng(13)
    n = 2_000_000
    comp = rng.choice(6, size=n, p=W[0])
    draws = ys[comp] + np.sqrt(model.sigma2[comp]) * rng.standard_normal(n)
    assert abs(draws.mean() - mu[0, 0]) < 5 * np.sqrt(v[0, 0] / n)
    assert abs(draws.var() - v[0, 0]) < 6 * v[0, 0] * np.sqrt(2.0 / n) * 2


def test_permuting_models_changes_nothing():
    model = _model(6, d=4, L=(9,), R=2)
    perm = np.random.default_rng(1).permutation(9)
    m2 = model.copy()
    for name in ("centre", "metric", "proj_u", "beta", "sigma2"):
        setattr(m2, name, getattr(model, name)[perm].copy())
    z = np.random.default_rng(2).uniform(-1, 1, (7, 4))
    a = oracle.lwpr_predict(model, z)
    b = oracle.lwpr_predict(m2, z)
    assert np.allclose(a[0], b[0], rtol=1e-13) and np.allclose(a[1], b[1], rtol=1e-13)


def test_far_inputs_stay_finite():
    # the max-shift keeps the normalisation finite where every exp underflows
    model = _model(7, d=4, L=(5,), R=2)
    mu, v = oracle.lwpr_predict(model, np.full((1, 4), 40.0))
    assert np.all(np.isfinite(mu)) and np.all(np.isfinite(v))


# ------------------------------------------------------------------ rollout

def _affine_system(prob, model):
    """With one local model per output the mixture is y = beta0 + b^T (z - c):
    returns (b [n_out][d], off [n_out]) with the PLS deflation written as the
    product of rank-one updates  r_{r+1} = (I - p_r u_r^T) r_r."""
    d, R = model.d, model.R
    bs, offs = [], []
    for j in range(model.Ltot):
        U = model.proj_u[j]
        P = U if model.proj_p is None else model.proj_p[j]
        Mx = np.eye(d)
        b = np.zeros(d)
        for r in range(R):
            b += model.beta[j, r + 1] * (U[r] @ Mx)
            Mx = (np.eye(d) - np.outer(P[r], U[r])) @ Mx
        bs.append(b)
        offs.append(model.beta[j, 0] - b @ model.centre[j])
    return np.array(bs), np.array(offs)


def _hand_rollout(prob, model, eps, xi=None, var=None):
    """Steps x_{t+1} = x_t + dt (E x_t + S a_t), a = b z + off (+ sqrt(var) xi)."""
    n_x, n_u = prob.n_x, prob.n_u
    bs, offs = _affine_system(prob, model)
    npos = 2 if prob.dyn == DYN_POINTMASS2D else 3
    E = np.zeros((n_x, n_x))
    S = np.zeros((n_x, model.n_out))
    for a in range(npos):
        E[a, npos + a] = 1.0
        S[npos + a, a] = 1.0
    if prob.dyn == DYN_QUAD12:
        for a in range(3):
            E[6 + a, 9 + a] = 1.0
            S[9 + a, 3 + a] = 1.0
    xs = [np.asarray(prob.x0, np.float64)]
    for t in range(prob.T):
        z = np.concatenate([xs[-1], prob.u_nom[t] + eps[t]])
        acc = bs @ z + offs
        if xi is not None:
            acc = acc + np.sqrt(var) * xi[t]
        xs.append(xs[-1] + prob.dt * (E @ xs[-1] + S @ acc))
    return np.array(xs)


def _goal_cost(prob, x):
    npos = 2 if prob.dyn == DYN_POINTMASS2D else 3
    c = sum(prob.w_pos[a] * (x[a] - prob.goal[a]) ** 2 for a in range(npos))
    c += prob.w_vel * np.sum(x[npos:2 * npos] ** 2)
    if prob.dyn == DYN_QUAD12:
        c += prob.w_ang * np.sum(x[6:9] ** 2)
    return c


@pytest.mark.parametrize("dyn", [DYN_POINTMASS2D, DYN_QUAD12])
def test_single_model_zero_noise_is_hand_stepped_linear_dynamics(dyn):
    prob, model = synth.tiny_problem(1, dyn=dyn, L=1, R=3, K=3, T=7, M=0, n_obs=0)
    prob.noise_std[:] = 0.0
    cost, X = oracle.rollout_cost(prob, model, states=True)
    xs = _hand_rollout(prob, model, np.zeros((prob.T, prob.n_u)))
    for k in range(prob.K):
        assert np.allclose(X[k, 0], xs, rtol=1e-12, atol=1e-13)
        expect = [prob.dt * _goal_cost(prob, xs[t + 1]) for t in range(prob.T)]
        assert np.allclose(cost[k], expect, rtol=1e-12, atol=1e-15)


def test_hybrid_angles_follow_commanded_rates_closed_form():
    # Sec. 4.1: the angles obey dr/dt = 25 (r_commanded - r), independent of the
    # learned models; explicit Euler with a constant command c gives the
    # geometric approach r_n = c + (r_0 - c)(1 - 25 dt)^n
    prob, model = synth.tiny_problem(21, dyn=DYN_QUAD_HYBRID, L=[2, 3, 1], R=2, K=2, T=9, M=0, n_obs=0)
    prob.noise_std[:] = 0.0
    cmd = np.array([0.3, -0.2, 0.05])
    prob.u_nom[:, :3] = cmd
    prob.x0[6:9] = [-0.1, 0.4, 0.0]
    _, X = oracle.rollout_cost(prob, model, states=True)
    n = np.arange(prob.T + 1)[:, None]
    expect = cmd + (prob.x0[6:9] - cmd) * (1.0 - 25.0 * prob.dt) ** n
    assert np.allclose(X[0, 0, :, 6:9], expect, rtol=1e-12, atol=1e-14)


def test_hybrid_single_model_is_hand_stepped():
    # one local model per output: the accelerations are affine in the model
    # input (phi, theta, psi, F) = (x_6, x_7, x_8, u_3); positions and
    # velocities integrate them, the angles follow the commanded rates
    prob, model = synth.tiny_problem(22, dyn=DYN_QUAD_HYBRID, L=1, R=3, K=2, T=8, M=0, n_obs=0)
    prob.noise_std[:] = 0.0
    prob.x0[6:9] = [0.2, -0.3, 0.1]
    cost, X = oracle.rollout_cost(prob, model, states=True)
    bs, offs = _affine_system(prob, model)
    x = np.asarray(prob.x0, np.float64).copy()
    xs, cs = [x.copy()], []
    for t in range(prob.T):
        u = prob.u_nom[t]
        acc = bs @ np.array([x[6], x[7], x[8], u[3]]) + offs
        xn = x.copy()
        xn[0:3] = x[0:3] + prob.dt * x[3:6]
        xn[3:6] = x[3:6] + prob.dt * acc
        xn[6:9] = x[6:9] + prob.dt * 25.0 * (u[0:3] - x[6:9])
        x = xn
        xs.append(x.copy())
        c = sum(prob.w_pos[a] * (x[a] - prob.goal[a]) ** 2 for a in range(3))
        c += prob.w_vel * np.sum(x[3:6] ** 2) + prob.w_ang * np.sum(x[6:9] ** 2)
        cs.append(prob.dt * c)
    assert np.allclose(X[0, 0], np.array(xs), rtol=1e-12, atol=1e-13)
    assert np.allclose(cost[0], cs, rtol=1e-12, atol=1e-15)


def test_single_model_with_noise_follows_its_perturbations():
    prob, model = synth.tiny_problem(2, L=1, R=2, K=4, T=6, M=1, n_obs=0)
    model.sigma2[:] = [0.04, 0.09]
    cost, X = oracle.rollout_cost(prob, model, states=True)
    eps = oracle.control_noise(prob)
    for k in range(prob.K):
        xi = np.stack([oracle.normals(prob.seed, oracle.TAG_DYN, prob.problem_id, 0, k, 0, t, 2)
                       for t in range(prob.T)])
        xs = _hand_rollout(prob, model, eps[k], xi=xi, var=model.sigma2)
        assert np.allclose(X[k, 0], xs, rtol=1e-12, atol=1e-13)


def test_zero_model_variance_makes_sub_rollouts_identical():
    base, model = synth.tiny_problem(3, L=1, R=2, K=4, T=5, M=1)
    model.sigma2[:] = 0.0
    costs = []
    for M in (0, 1, 3):
        p = base.copy()
        p.M = M
        costs.append(oracle.rollout_cost(p, model))
    assert np.array_equal(costs[0], costs[1]) and np.allclose(costs[1], costs[2], rtol=1e-14)


def test_sub_rollout_costs_are_averaged():
    prob, model = synth.tiny_problem(4, L=3, R=2, K=2, T=5, M=3, n_obs=0)
    cost, X = oracle.rollout_cost(prob, model, states=True)
    for k in range(prob.K):
        per_m = [[prob.dt * _goal_cost(prob, X[k, m, t + 1]) for t in range(prob.T)]
                 for m in range(3)]
        assert np.allclose(cost[k], np.mean(per_m, 0), rtol=1e-13)
        assert not np.allclose(X[k, 0], X[k, 1])  # sub-rollouts differ


def test_rollout_k_does_not_depend_on_K():
    prob, model = synth.tiny_problem(5, L=3, R=2, K=9, T=6, M=2)
    full = oracle.rollout_cost(prob, model)
    part = oracle.rollout_cost(prob, model, k_range=(4, 7))
    small = prob.copy()
    small.K = 5
    assert np.array_equal(full[4:7], part)
    assert np.array_equal(full[:5], oracle.rollout_cost(small, model))


def test_obstacle_penalty_counts_steps_inside():
    # constant acceleration along +x through a disc of radius 0.2 at (0, 0)
    prob, model = synth.tiny_problem(6, L=1, R=1, K=1, T=60, M=0, n_obs=1)
    prob.noise_std[:] = 0.0
    prob.x0[:] = [-0.5, 0.0, 0.0, 0.0]
    prob.obs[:] = [[0.0, 0.0, 0.2]]
    prob.goal[:] = 0.0
    model.beta[:] = 0.0
    model.beta[0, 0] = 2.0      # a_x = 2
    model.beta[1, 0] = 0.0      # a_y = 0
    cost, X = oracle.rollout_cost(prob, model, states=True)
    xs = X[0, 0, 1:, 0]
    inside = (xs ** 2 < 0.04)
    assert 0 < inside.sum() < prob.T
    expect = prob.dt * (xs ** 2 + prob.obs_penalty * inside)
    assert np.allclose(cost[0], expect, rtol=1e-13)


@pytest.mark.parametrize("dyn", [DYN_POINTMASS2D, DYN_QUAD12])
def test_smooth_obstacle_cost_on_a_constant_acceleration_path(dyn):
    # Sec. 5: the smooth obstacle term is 100 sum_i exp(-10 (dx_i^2 + dy_i^2))
    # over the horizontal distances to every obstacle centre.  One affine model
    # with only its offset set makes the acceleration constant, so explicit
    # Euler from rest gives the closed form v_n = n dt a,
    # p_n = p_0 + a dt^2 n (n - 1) / 2, and every step cost is dt q(x_{n+1})
    # written out from the task's weights.
    prob, model = synth.tiny_problem(6, dyn=dyn, L=1, R=1, K=1, T=50, M=0, n_obs=2,
                                     obs_kind=OBS_SMOOTH)
    assert prob.obs_penalty == 100.0 and prob.obs_decay == 10.0
    npos = 2 if dyn == DYN_POINTMASS2D else 3
    prob.noise_std[:] = 0.0
    prob.x0[:] = 0.0
    prob.x0[:npos] = [-0.5, -0.1, 0.2][:npos]
    prob.obs[:] = [[0.0, 0.0, 0.2], [0.25, 0.1, 0.2]]
    prob.goal[:] = [0.3, -0.2, 0.4]
    prob.w_vel = 0.3
    model.beta[:] = 0.0
    a = np.zeros(model.n_out)
    a[:2] = [2.0, 0.5]
    model.beta[:, 0] = a                    # y_o = beta_o0: constant accelerations
    cost, X = oracle.rollout_cost(prob, model, states=True)
    n = np.arange(1, prob.T + 1)[:, None]
    p = prob.x0[:npos] + a[:npos] * prob.dt ** 2 * n * (n - 1) / 2
    v = a[:npos] * prob.dt * n
    assert np.allclose(X[0, 0, 1:, :npos], p, rtol=1e-12, atol=1e-14)
    q = ((p - prob.goal[:npos]) ** 2 * prob.w_pos[:npos]).sum(1) + prob.w_vel * (v ** 2).sum(1)
    bumps = sum(100.0 * np.exp(-10.0 * ((p[:, 0] - cx) ** 2 + (p[:, 1] - cy) ** 2))
                for cx, cy, _ in prob.obs)
    # the path passes close enough for the bumps to dominate some steps
    assert bumps.max() > 50.0 and bumps.max() > 5.0 * bumps.min()
    assert np.allclose(cost[0], prob.dt * (q + bumps), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("dyn", [DYN_POINTMASS2D, DYN_QUAD12])
def test_rh_shift_plant_draw_is_a_sample_of_the_model(rocrand_ref, dyn):
    # Sec. 3.1, last paragraph: the first control of the plan is executed on
    # the plant -- here one draw from the learned model, N(y(z), sigma^2) per
    # output with a single affine local model -- and the plan shifts by one
    # step.  The draw's standard normals are formed here from rocRAND's Philox
    # words at the plant stream's counter (t = 0, k = 0, block, tag 2 with the
    # problem and iteration words) and the Box-Muller pairs written out.
    prob, model = synth.tiny_problem(31, dyn=dyn, L=1, R=3, K=2, T=5, n_obs=0)
    prob.problem_id = 5
    model.sigma2[:] = np.linspace(0.04, 0.09, model.n_out)
    it = 0x12345 + 3
    x0 = prob.x0.copy()
    x0[prob.n_x // 2:] = np.linspace(-0.3, 0.4, prob.n_x - prob.n_x // 2)
    x, u = oracle.rh_shift(prob, model, x0, prob.u_nom, it)
    assert np.array_equal(u[:-1], prob.u_nom[1:]) and np.array_equal(u[-1], prob.u_nom[-1])
    word3 = (2 << 30) | ((prob.problem_id & 0x3FF) << 20) | (it & 0xFFFFF)
    key = (prob.seed & 0xFFFFFFFF, prob.seed >> 32)
    nblk = (model.n_out + 3) // 4
    lines = "\n".join("0 0 %d %d %d %d" % (b, word3, key[0], key[1]) for b in range(nblk))
    raw = np.array(subprocess.run([rocrand_ref], input=lines + "\n", capture_output=True,
                                  text=True, check=True).stdout.split(), np.uint64).reshape(nblk, 4)
    un = ((raw >> 9).astype(np.float64) + 0.5) * 2.0 ** -23
    rad0, rad1 = np.sqrt(-2 * np.log(un[:, 0])), np.sqrt(-2 * np.log(un[:, 2]))
    xi = np.stack([rad0 * np.cos(2 * np.pi * un[:, 1]), rad0 * np.sin(2 * np.pi * un[:, 1]),
                   rad1 * np.cos(2 * np.pi * un[:, 3]), rad1 * np.sin(2 * np.pi * un[:, 3])],
                  1).reshape(-1)[:model.n_out]
    bs, offs = _affine_system(prob, model)
    acc = bs @ np.concatenate([x0, prob.u_nom[0]]) + offs + np.sqrt(model.sigma2) * xi
    npos = 2 if dyn == DYN_POINTMASS2D else 3
    expect = x0.copy()
    expect[:npos] += prob.dt * x0[npos:2 * npos]
    expect[npos:2 * npos] += prob.dt * acc[:npos]
    if dyn == DYN_QUAD12:
        expect[6:9] += prob.dt * x0[9:12]
        expect[9:12] += prob.dt * acc[3:6]
    assert np.allclose(x, expect, rtol=1e-12, atol=1e-14)
    # the draw is not the mean: the noise term moves the velocities measurably
    mean_only = expect.copy()
    mean_only[npos:2 * npos] -= prob.dt * (np.sqrt(model.sigma2) * xi)[:npos]
    assert np.max(np.abs(x - mean_only)) > 1e-4


# ------------------------------------------------------------------ update, Eq. (2)

def _upd_case(seed=0, K=6, T=5, **kw):
    prob, model = synth.tiny_problem(seed, K=K, T=T, **kw)
    cost = np.random.default_rng(seed).uniform(0.0, 2.0, (K, T))
    return prob, cost


def test_update_with_one_sample_returns_its_perturbation():
    prob, cost = _upd_case(K=1)
    u = oracle.update(prob, cost)
    eps = oracle.control_noise(prob)[0]
    assert np.allclose(u - prob.u_nom, eps, rtol=1e-14, atol=1e-15)


def test_update_with_equal_costs_is_the_mean_perturbation():
    prob, cost = _upd_case(K=7)
    cost[:] = 0.3
    u = oracle.update(prob, cost)
    assert np.allclose(u - prob.u_nom, oracle.control_noise(prob).mean(0), rtol=1e-12, atol=1e-15)


def test_update_limits_of_lambda():
    prob, cost = _upd_case(K=8)
    eps = oracle.control_noise(prob)
    S = np.cumsum(cost[:, ::-1], 1)[:, ::-1]     # cost-to-go
    p = prob.copy()
    p.lam = 1e-9
    u = oracle.update(p, cost)
    best = S.argmin(0)
    assert np.allclose(u - prob.u_nom, eps[best, np.arange(prob.T)], rtol=1e-12, atol=1e-14)
    p.lam = 1e12
    u = oracle.update(p, cost)
    assert np.allclose(u - prob.u_nom, eps.mean(0), rtol=1e-9, atol=1e-12)


def test_update_weights_are_softmax_of_cost_to_go():
    prob, cost = _upd_case(K=6, T=4)
    prob.lam = 0.7
    _, W = oracle.update(prob, cost, weights=True)
    S = np.array([[cost[k, i:].sum() for i in range(prob.T)] for k in range(prob.K)])
    from scipy.special import softmax
    assert np.allclose(W, softmax(-S / prob.lam, axis=0).T, rtol=1e-12)
    assert np.allclose(W.sum(1), 1.0, atol=1e-15)
    # invariance to adding a constant to the costs of one step for every k
    c2 = cost.copy()
    c2[:, 2] += 123.0
    assert np.allclose(oracle.update(prob, c2), oracle.update(prob, cost), rtol=1e-12)


def test_trajectory_weighting_uses_the_first_row():
    prob, cost = _upd_case(K=6, T=5)
    _, Wc = oracle.update(prob, cost, weights=True)
    p = prob.copy()
    p.weighting = W_TRAJECTORY
    _, Wt = oracle.update(p, cost, weights=True)
    assert np.allclose(Wt, np.repeat(Wc[:1], prob.T, 0), rtol=1e-14)


def test_rh_shift_moves_the_plan():
    prob, model = synth.tiny_problem(8, K=2, T=5)
    x, u = oracle.rh_shift(prob, model, prob.x0, prob.u_nom, 3)
    assert np.array_equal(u[:-1], prob.u_nom[1:]) and np.array_equal(u[-1], prob.u_nom[-1])
    # velocities change by dt * a, positions by dt * v (v0 = 0)
    assert np.allclose(x[:2], prob.x0[:2]) and not np.allclose(x[2:], prob.x0[2:])


def _goal_case():
    prob, model = synth.tiny_problem(9, K=6, T=5)
    goals = np.array([[0.5, -0.5, 0.0], [-0.7, 0.2, 0.0], [0.1, 0.9, 0.0]])
    return prob, model, goals


def test_goal_switching_with_zero_radius_is_the_plain_loop():
    # nothing is ever within distance 0: the loop is the fixed-goal loop
    prob, model, goals = _goal_case()
    x, u, it, g = oracle.rh_loop_goals(prob, model, 3, goals, radius=0.0)
    prob.goal = goals[0].copy()
    xr, ur, itr = oracle.rh_loop(prob, model, 3)
    assert g == 0 and it == itr and np.array_equal(x, xr) and np.array_equal(u, ur)


def test_goal_switching_with_unbounded_radius_cycles_every_step():
    # every plant update is within reach: step n optimises toward goal n mod 3,
    # which is the plain loop with that goal, one control step at a time
    prob, model, goals = _goal_case()
    x, u, it, g = oracle.rh_loop_goals(prob, model, 4, goals, radius=np.inf)
    assert g == 4 % 3
    xr, ur, itr = prob.x0, prob.u_nom, 0
    for n in range(4):
        prob.goal = goals[n % 3].copy()
        xr, ur, itr = oracle.rh_loop(prob, model, 1, x0=xr, u_nom=ur, it=itr)
    assert np.array_equal(x, xr) and np.array_equal(u, ur) and it == itr


def test_goal_switching_waits_for_the_plant_update():
    # the start lies on goal 0: the switch follows the first control step (the
    # plant moves by about dt^2 a / 2 from rest, far less than the radius),
    # not the initial state, so the first step still optimises toward goal 0
    prob, model, goals = _goal_case()
    goals[0, :2] = prob.x0[:2]
    x1, u1, _, g1 = oracle.rh_loop_goals(prob, model, 1, goals)
    assert g1 == 1
    prob.goal = goals[0].copy()
    xr, ur, _ = oracle.rh_loop(prob, model, 1)
    assert np.array_equal(x1, xr) and np.array_equal(u1, ur)
    assert np.linalg.norm(x1[:2] - goals[0, :2]) < 0.25


# ------------------------------------------------------------------ adjoint

def _fd(fun, x, idx, h):
    xp, xm = x.copy(), x.copy()
    xp.flat[idx] += h
    xm.flat[idx] -= h
    return (fun(xp) - fun(xm)) / (2 * h)


def _J(prob, model):
    return float(oracle.rollout_cost(prob, model).sum(1).mean())


@pytest.mark.parametrize("dyn,M", [(DYN_POINTMASS2D, 1), (DYN_POINTMASS2D, 2), (DYN_QUAD12, 1),
                                   (DYN_POINTMASS2D, 0)])
def test_adjoint_matches_central_differences(dyn, M):
    prob, model = synth.tiny_problem(9, dyn=dyn, L=3, R=2, K=3, T=6, M=M, n_obs=2,
                                     obs_kind=OBS_SMOOTH)
    prob.obs[:, :2] = prob.x0[:2] + 0.15  # close enough for the bump to matter
    J, gu, gc, gD = oracle.adjoint(prob, model)
    assert np.isclose(J, _J(prob, model), rtol=1e-13)
    h = 1e-5
    rng = np.random.default_rng(0)

    def f_u(u):
        p = prob.copy()
        p.u_nom = u
        return _J(p, model)

    def f_c(c):
        m = model.copy()
        m.centre = c
        return _J(prob, m)

    def f_D(D):
        m = model.copy()
        m.metric = D
        return _J(prob, m)

    for fun, x, g in ((f_u, prob.u_nom, gu), (f_c, model.centre, gc), (f_D, model.metric, gD)):
        for idx in rng.choice(x.size, size=min(12, x.size), replace=False):
            fd = _fd(fun, x, idx, h)
            assert abs(fd - g.flat[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, g.flat[idx])


def test_adjoint_linear_quadratic_closed_form():
    # one affine model per output, mean-only, no obstacles: the state is an
    # affine function of the nominal controls and J is quadratic in them.
    prob, model = synth.tiny_problem(10, dyn=DYN_QUAD12, L=1, R=3, K=2, T=5, M=0, n_obs=0)
    _, gu, _, _ = oracle.adjoint(prob, model)
    n_x, n_u, T = prob.n_x, prob.n_u, prob.T
    bs, offs = _affine_system(prob, model)
    E = np.zeros((n_x, n_x))
    S = np.zeros((n_x, 6))
    for a in range(3):
        E[a, 3 + a] = E[6 + a, 9 + a] = 1.0
        S[3 + a, a] = S[9 + a, 3 + a] = 1.0
    Ax = np.eye(n_x) + prob.dt * (E + S @ bs[:, :n_x])
    Bu = prob.dt * S @ bs[:, n_x:]
    W = np.diag(np.concatenate([prob.w_pos, np.full(3, prob.w_vel), np.full(3, prob.w_ang),
                                np.zeros(3)]))
    g = np.concatenate([prob.goal, np.zeros(9)])
    eps = oracle.control_noise(prob)
    grad = np.zeros((T, n_u))
    for k in range(prob.K):
        xs = _hand_rollout(prob, model, eps[k])
        # G_t = d x_t / d u_s  (s < t)
        for t in range(1, T + 1):
            r = 2 * prob.dt * W @ (xs[t] - g)
            for s in range(t):
                Gts = np.linalg.matrix_power(Ax, t - 1 - s) @ Bu
                grad[s] += Gts.T @ r
    grad /= prob.K
    assert np.allclose(gu, grad, rtol=1e-11, atol=1e-13)


# ------------------------------------------------------------------ control terms of S-tilde

def _ctrl_case(seed=51, K=6, T=7, M=1):
    prob, model = synth.tiny_problem(seed, dyn=DYN_QUAD_HYBRID, L=[3, 4, 2], R=2, K=K, T=T, M=M,
                                     n_obs=2)
    prob.noise_std[:] = [0.5, 0.3, 0.4, 0.6]
    prob.lam = 0.7
    return prob, model


def test_control_terms_are_the_noise_likelihood_ratio():
    # Sec. 3.1: with B B^T = lambda G R^-1 G^T the control terms of S-tilde,
    # divided by lambda, are  u^T S^-1 u + u^T S^-1 eps  (S = diag(sigma^2) of
    # the commanded rates' perturbation eps):  the log-density ratio
    # log N(eps; 0, S) - log N(u + eps; 0, S) plus (1/2) u^T S^-1 u, written
    # here with SciPy's Gaussian.  The dynamics do not change, so the state
    # costs cancel in the difference of the two cost arrays.
    for M in (1, 3):
        prob, model = _ctrl_case(M=M)
        off = oracle.rollout_cost(prob, model)
        p = prob.copy()
        p.ctrl_cost = 1
        on = oracle.rollout_cost(p, model)
        eps = oracle.control_noise(prob)[:, :, :3]
        Sig = np.diag(prob.noise_std[:3] ** 2)
        g = stats.multivariate_normal(mean=np.zeros(3), cov=Sig)
        u = prob.u_nom[:, :3]
        for k in range(prob.K):
            ratio = g.logpdf(eps[k]) - g.logpdf(u + eps[k]) + 0.5 * np.einsum(
                "ta,ab,tb->t", u, np.linalg.inv(Sig), u)
            assert np.allclose((on[k] - off[k]) / prob.lam, ratio, rtol=1e-10, atol=1e-12)


def test_control_terms_vanish_for_a_zero_plan_and_keep_the_one_sample_update():
    prob, model = _ctrl_case()
    prob.u_nom[:] = 0.0
    p = prob.copy()
    p.ctrl_cost = 1
    assert np.array_equal(oracle.rollout_cost(p, model), oracle.rollout_cost(prob, model))
    # K = 1: the update returns its own perturbation whatever the costs
    p1, m1 = _ctrl_case(K=1)
    p1.ctrl_cost = 1
    cost = oracle.rollout_cost(p1, m1)
    u = oracle.update(p1, cost)
    assert np.allclose(u - p1.u_nom, oracle.control_noise(p1)[0], rtol=1e-14, atol=1e-15)
