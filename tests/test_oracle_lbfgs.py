"""Pins for the oracle optimiser: the two-loop recursion against the explicit dense BFGS
inverse update (textbook identity), the converged point against SciPy's L-BFGS-B, the
whole loop driving inverse-crime data to zero cost, and resume/failure paths."""
import numpy as np
import pytest
import scipy.optimize as so

from oracle import lbfgs, model
from paper_2202_08627_amd import synth
from helpers import geometry, tiny_cfg


def test_two_loop_equals_dense_bfgs():
    """P11a: H g from the two-loop recursion = explicit BFGS recursion from gamma I."""
    rng = np.random.default_rng(0)
    n = 20
    M = rng.standard_normal((n, n))
    Q = M @ M.T + n * np.eye(n)
    S, Y = [], []
    for _ in range(6):
        s = rng.standard_normal(n)
        S.append(s)
        Y.append(Q @ s)
    g = rng.standard_normal(n)
    H = lbfgs.dense_bfgs_inverse(S, Y, n)
    assert np.allclose(lbfgs.two_loop(g, S, Y), H @ g, rtol=1e-12, atol=1e-12 * np.abs(H @ g).max())


def test_quadratic_minimum():
    """On a strictly convex quadratic the method reaches the unique minimiser."""
    rng = np.random.default_rng(1)
    n = 30
    M = rng.standard_normal((n, n))
    Q = M @ M.T + np.eye(n)
    b = rng.standard_normal(n)
    fun = lambda z: (0.5 * z @ Q @ z - b @ z, Q @ z - b)
    z, st, tr = lbfgs.minimize(fun, np.zeros(n), 500, tol_rel_step=1e-14)
    # Armijo comparisons on F stop resolving progress near |dz| ~ sqrt(eps cond)
    assert np.allclose(z, np.linalg.solve(Q, b), rtol=1e-6, atol=1e-8)
    assert all(np.diff(tr.cost) <= 0)


def _tiny_problem(seed=0, n=16, lam=None, noise=True):
    cfg = tiny_cfg(n=n, n_theta=24 if n == 16 else 45)
    c = synth.make_case(cfg, seed=seed, noise=noise)
    geo = geometry(c, model)
    return c, geo, cfg


def test_fixed_point_matches_scipy():
    """P11b: the converged point equals SciPy's L-BFGS-B minimiser (gtol 1e-10)."""
    c, geo, cfg = _tiny_problem()
    prob = model.ScaledProblem(c.s_exp, geo, cfg.lam, cfg.mu_scale, cfg.delta_scale)
    z0 = np.zeros((2, cfg.n, cfg.n))
    z, st, _ = lbfgs.minimize(prob, z0, 3000, tol_rel_step=1e-12)
    fun = lambda v: (lambda fg: (fg[0], fg[1].ravel()))(prob(v.reshape(z0.shape)))
    r = so.minimize(fun, z0.ravel(), jac=True, method="L-BFGS-B",
                    options=dict(gtol=1e-10, ftol=1e-15, maxiter=20000, maxcor=10))
    assert np.linalg.norm(r.x - z.ravel()) / np.linalg.norm(z) < 1e-6
    assert st.f == pytest.approx(r.fun, rel=1e-10)


def test_inverse_crime_cost_to_zero():
    """P10: data made by the model itself with lam = 0 has minimum S = 0 at the phantom;
    the loop drives S down monotonically by > 6 orders of magnitude."""
    cfg = tiny_cfg(n=32, n_theta=45)
    c = synth.make_case(cfg)
    geo = geometry(c, model)
    *_, s_clean = model.forward(c.mu_true, c.delta_true, geo)
    prob = model.ScaledProblem(s_clean, geo, 0.0, cfg.mu_scale, cfg.delta_scale)
    z0 = np.zeros((2, 32, 32))
    S0 = prob(z0)[0]
    z, st, tr = lbfgs.minimize(prob, z0, 300)
    assert all(np.diff(tr.cost) <= 0)
    assert tr.cost[-1] / S0 < 1e-6
    x = prob.to_x(z)
    assert np.linalg.norm(x[0] - c.mu_true) / np.linalg.norm(c.mu_true) < 0.05


def test_resume_equals_uninterrupted():
    c, geo, cfg = _tiny_problem(seed=4)
    prob = model.ScaledProblem(c.s_exp, geo, cfg.lam, cfg.mu_scale, cfg.delta_scale)
    z0 = np.zeros((2, cfg.n, cfg.n))
    z_full, st_full, _ = lbfgs.minimize(prob, z0, 30)
    _, st_half, _ = lbfgs.minimize(prob, z0, 12)
    z_res, st_res, _ = lbfgs.minimize(prob, None, 30, state=st_half.copy())
    assert np.array_equal(z_full, z_res)
    assert st_full.evals == st_res.evals


def test_forced_line_search_failure():
    c, geo, cfg = _tiny_problem()
    prob = model.ScaledProblem(c.s_exp, geo, cfg.lam, cfg.mu_scale, cfg.delta_scale)
    z, st, tr = lbfgs.minimize(prob, np.zeros((2, cfg.n, cfg.n)), 5, max_ls=0)
    assert tr.status == lbfgs.STATUS_LINESEARCH and st.k == 0


def test_nonfinite_input_detected():
    c, geo, cfg = _tiny_problem()
    s = c.s_exp.copy()
    s[0, 0, 0] = np.nan
    prob = model.ScaledProblem(s, geo, cfg.lam, cfg.mu_scale, cfg.delta_scale)
    z, st, tr = lbfgs.minimize(prob, np.zeros((2, cfg.n, cfg.n)), 5)
    assert tr.status == lbfgs.STATUS_NONFINITE


def test_small_config_iterations_reduce_cost():
    """The 64^2 / 90-angle / M = 5 workload: 50 iterations reduce the cost monotonically
    and bring mu close to the phantom."""
    from paper_2202_08627_amd import configs
    cfg = configs.SMALL_64
    c = synth.make_case(cfg)
    geo = geometry(c, model)
    prob = model.ScaledProblem(c.s_exp, geo, cfg.lam, cfg.mu_scale, cfg.delta_scale)
    x, st, tr = lbfgs.reconstruct(prob, np.zeros((2, 64, 64)), cfg.iters)
    assert st.k == cfg.iters and all(np.diff(tr.cost) <= 0)
    assert np.linalg.norm(x[0] - c.mu_true) / np.linalg.norm(c.mu_true) < 0.2


# ---------------------------------------------------------------------------------------
# Step-control rules, pinned by traces worked out by hand (not by running `minimize`).
# Each scripted function records every point the optimiser asks for, so the test sees the
# exact sequence of trial steps, the accept/reject decisions (through where the next trial
# lands), the memory resets and the stored pairs.

class _Recorder:
    def __init__(self, fun):
        self.fun = fun
        self.points = []

    def __call__(self, z):
        self.points.append(np.array(z, dtype=np.float64, copy=True))
        return self.fun(z)


def _quad(z):
    """F = (4 z1^2 + z2^2) / 2, gradient (4 z1, z2)."""
    return 0.5 * (4.0 * z[0] ** 2 + z[1] ** 2), np.array([4.0 * z[0], z[1]])


def _walled_quad(z):
    """The quadratic plus 1 wherever z1 < 0 and z2 < 0.195 (the gradient ignores the wall)."""
    f, g = _quad(z)
    return f + (1.0 if (z[0] < 0.0 and z[1] < 0.195) else 0.0), g


def test_first_step_halving_and_acceptance_by_hand():
    """F = (4 z1^2 + z2^2)/2 from z0 = (0.075, 0.4), by hand:
    g0 = (0.3, 0.4), |g0| = 0.5, so the first trial is alpha = 1/|g0| = 2 along d0 = -g0;
    F0 = 0.09125 and g0.d0 = -0.25.
      alpha = 2   -> (-0.525, -0.4), F = 0.63125  > F0 - 1e-4 * 2 * 0.25    reject
      alpha = 1   -> (-0.225,  0.0), F = 0.10125  > F0 - 1e-4 * 1 * 0.25    reject
      alpha = 1/2 -> (-0.075,  0.2), F = 0.03125 <= F0 - 1e-4 * 0.5 * 0.25  accept
    The pair s = (-0.15, -0.2), y = g1 - g0 = (-0.6, -0.2) has s.y = 0.13 > 0: stored.
    Iteration 2 starts at alpha = 1 along d1 = -H g1 with g1 = (-0.3, 0.2) and, from the one
    pair (H0 = (s.y / y.y) I = 0.325 I), d1 = (51, -127) / 1040:
      q = g1 - (s.g1 / s.y) y = g1 - y/26; r = 0.325 q = (-0.09, 0.0675);
      beta = y.r / s.y = 81/260; r += s (1/26 - 81/260) -> r = (-12.75, 31.75)/260 = -d1."""
    rec = _Recorder(_quad)
    z, st, tr = lbfgs.minimize(rec, np.array([0.075, 0.4]), 2)
    P = rec.points
    expect_it1 = [(0.075, 0.4), (-0.525, -0.4), (-0.225, 0.0), (-0.075, 0.2)]
    for p, e in zip(P[:4], expect_it1):
        assert np.allclose(p, e, rtol=0, atol=1e-15), (p, e)
    d1 = np.array([51.0, -127.0]) / 1040.0
    assert np.allclose(P[4], np.array([-0.075, 0.2]) + d1, rtol=0, atol=1e-15)
    assert tr.trials[0] == 3 and tr.alpha[0] == 0.5
    assert tr.alpha[1] == 1.0
    assert tr.cost[0] == pytest.approx(0.03125, abs=1e-16)


def test_sufficient_decrease_term_rejects_equal_cost():
    """F = 2 z^2 from z0 = 0.125 (binary-exact values): g0 = 0.5, first trial alpha = 2, d0 = -0.5.
    Trials land at -0.875, -0.375 and -0.125; the last has F = F0 = 0.03125 exactly, which the
    c1 = 1e-4 term rejects (0.03125 > 0.03125 - 1e-4 * 0.5 * 0.25). The fourth trial, alpha = 1/4,
    lands on 0. A missing c1 term would stop at three trials."""
    rec = _Recorder(lambda z: (2.0 * float(z[0]) ** 2, np.array([4.0 * z[0]])))
    z, st, tr = lbfgs.minimize(rec, np.array([0.125]), 1)
    assert [float(p[0]) for p in rec.points] == [0.125, -0.875, -0.375, -0.125, 0.0]
    assert tr.trials == [4] and tr.alpha == [0.25] and float(z[0]) == 0.0


def test_failed_search_clears_memory_and_redoes_along_gradient():
    """The quadratic of the first hand trace with a wall (+1 where z1 < 0 and z2 < 0.195) and
    at most 4 trials. Iteration 1 is unchanged (its third trial (-0.075, 0.2) is outside the
    wall). Iteration 2's quasi-Newton trials z1 + alpha d1, alpha = 1, 1/2, 1/4, 1/8, are
    (-0.02596, 0.07788), (-0.05048, 0.13894), (-0.06274, 0.16947), (-0.06887, 0.18474): all
    inside the wall, all rejected. The memory is then cleared and the iteration redone along
    -g1 = (0.3, -0.2) from alpha = 1/|g1| = 1/sqrt(0.13):
      alpha     -> ( 0.75705, -0.35470)  F = 1.2092  reject
      alpha/2   -> ( 0.34103, -0.07735)  F = 0.2356  reject
      alpha/4   -> ( 0.13301,  0.06133)  F = 0.0373  reject (F1 = 0.03125)
      alpha/8   -> ( 0.02901,  0.13066)  F = 0.0102  accept
    So 1 + 3 + 4 + 4 = 12 evaluations, trials [3, 4], and the memory holds the one new pair."""
    rec = _Recorder(_walled_quad)
    z, st, tr = lbfgs.minimize(rec, np.array([0.075, 0.4]), 2, max_ls=4)
    P = rec.points
    z1 = np.array([-0.075, 0.2])
    d1 = np.array([51.0, -127.0]) / 1040.0
    for q, a in enumerate((1.0, 0.5, 0.25, 0.125)):
        assert np.allclose(P[4 + q], z1 + a * d1, rtol=0, atol=1e-15)
    a0 = 1.0 / np.sqrt(0.13)
    for q, a in enumerate((a0, a0 / 2, a0 / 4, a0 / 8)):
        assert np.allclose(P[8 + q], z1 + a * np.array([0.3, -0.2]), rtol=0, atol=1e-14)
    assert len(P) == 12 and st.evals == 12 and st.k == 2
    assert tr.trials == [3, 4]
    assert tr.alpha[1] == pytest.approx(a0 / 8, rel=1e-15)
    assert len(st.S) == 1
    assert np.allclose(st.S[0], P[11] - z1, rtol=0, atol=1e-15)
    assert np.allclose(st.Y[0], np.array([4.0 * P[11][0] + 0.3, P[11][1] - 0.2]), rtol=0, atol=1e-15)
    assert np.array_equal(z, P[11])


def test_failed_search_with_empty_memory_stops():
    """Same walled quadratic, at most 2 trials: iteration 1 (empty memory) rejects alpha = 2 and
    alpha = 1, and with nothing to clear the run stops with the line-search status, at z0,
    after 3 evaluations."""
    rec = _Recorder(_walled_quad)
    z, st, tr = lbfgs.minimize(rec, np.array([0.075, 0.4]), 5, max_ls=2)
    assert tr.status == lbfgs.STATUS_LINESEARCH and st.k == 0 and st.evals == 3
    assert np.array_equal(z, np.array([0.075, 0.4]))


@pytest.mark.parametrize("eps,stored", [(1e-9, True), (1e-11, False), (0.0, False)])
def test_pair_acceptance_threshold(eps, stored):
    """F(z) = z1 with the scripted gradient (1, 0) at z0 = 0 and (1 - eps, 1) elsewhere. The
    first step is alpha = 1 along (-1, 0), accepted at once (F drops by 1). Then s = (-1, 0),
    y = (-eps, 1): s.y = eps against 1e-10 |s||y| = 1e-10 sqrt(1 + eps^2). The pair is kept
    for eps = 1e-9 only. The next iteration starts at alpha = 1 with a pair, else at
    1/|g1| = 1/sqrt((1 - eps)^2 + 1)."""
    def fun(z):
        g = np.array([1.0, 0.0]) if not np.any(z) else np.array([1.0 - eps, 1.0])
        return float(z[0]), g
    z, st, tr = lbfgs.minimize(fun, np.zeros(2), 2)
    assert tr.alpha[0] == 1.0
    if stored:
        assert len(st.S) >= 1 and tr.alpha[1] == 1.0
    else:
        assert tr.alpha[1] == pytest.approx(1.0 / np.hypot(1.0 - eps, 1.0), rel=1e-15)


def test_memory_keeps_newest_pairs():
    """With m = 2 on a convex quadratic, after 5 iterations the memory holds exactly the pairs
    of iterations 4 and 5, oldest first (s_k = z_k - z_(k-1), y_k = Q s_k)."""
    Q = np.diag([1.0, 3.0, 7.0])
    zs = []
    fun = lambda z: (0.5 * z @ Q @ z, Q @ z)
    z, st, tr = lbfgs.minimize(fun, np.array([1.0, -2.0, 0.5]), 5, m=2,
                               callback=lambda s: zs.append(s.z.copy()))
    assert len(zs) == 5 and len(st.S) == 2
    for q, k in enumerate((3, 4)):
        assert np.allclose(st.S[q], zs[k] - zs[k - 1], rtol=0, atol=1e-15)
        assert np.allclose(st.Y[q], Q @ (zs[k] - zs[k - 1]), rtol=0, atol=1e-14)
