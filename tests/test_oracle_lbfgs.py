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
