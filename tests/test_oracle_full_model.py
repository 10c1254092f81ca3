"""Pins for the oracle's full forward model (eq. 4 with drift m_o, ring term m_r, h-mode and
tabulated flats; oracle/full_model.py): reduction to the pinned two-map model, finite
differences of the cost in every kind of unknown, the gauge ambiguity the paper points out,
closed forms with no sample, and the cubic-convolution table against polynomials it must
reproduce and the Gaussian it samples."""
import dataclasses

import numpy as np
import pytest

from oracle import full_model as fm
from oracle import model
from paper_2202_08627_amd import synth
from helpers import geometry, tiny_cfg


def _setup(n=12, n_theta=10, n_mask=3, seed=0, **kw):
    cfg = tiny_cfg(n=n, n_theta=n_theta, n_mask=n_mask, jitter=0.05)
    c = synth.make_case(cfg, seed=seed)
    st = fm.Setup(n, c.theta, cfg.n_det, c.mask_pos, c.flat_amp, c.flat_ctr, c.flat_sigma,
                  cfg.kappa, **kw)
    return c, cfg, st


def _params(st, c, rng, off_amp=0.05):
    nn = st.n * st.n
    if st.hmode:
        maps = [0.9 * c.mu_true.ravel() + 0.1 * c.cfg.mu_scale * rng.uniform(0, 1, nn)]
    else:
        maps = [0.9 * c.mu_true.ravel() + 0.1 * c.cfg.mu_scale * rng.uniform(0, 1, nn),
                0.9 * c.delta_true.ravel() + 1e-4 * rng.uniform(0, 1, nn)]
    parts = maps
    if st.fit_mo:
        parts.append(off_amp * rng.standard_normal(st.theta.size))
    if st.fit_mr:
        parts.append(off_amp * rng.standard_normal(st.n_det))
    return np.concatenate(parts)


def _fd_check(st, p, s_exp, lam_mu, lam_de, idx, h, rtol):
    S, g = fm.cost_and_grad(st, p, s_exp, lam_mu, lam_de)
    gmax = np.abs(g).max()
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (fm.cost(st, p + e, s_exp, lam_mu, lam_de) - fm.cost(st, p - e, s_exp, lam_mu, lam_de)) / (2 * h)
        assert abs(fd - g[i]) <= rtol * max(abs(g[i]), 1e-3 * gmax), (i, fd, g[i])


def test_reduces_to_two_map_model():
    """No offsets, Gaussian flats, two maps: the same cost and gradient as the pinned model."""
    c, cfg, st = _setup()
    geo = geometry(c, model)
    p = _params(st, c, np.random.default_rng(1))
    S, g = fm.cost_and_grad(st, p, c.s_exp, cfg.lam_mu, cfg.lam_delta)
    nn = st.n * st.n
    S0, gm, gd = model.cost_and_grad(p[:nn].reshape(st.n, st.n), p[nn:].reshape(st.n, st.n),
                                     c.s_exp, geo, cfg.lam_mu, cfg.lam_delta)
    assert S == pytest.approx(S0, rel=1e-14)
    assert np.allclose(g[:nn], gm.ravel(), rtol=1e-12, atol=1e-12 * np.abs(gm).max())
    assert np.allclose(g[nn:], gd.ravel(), rtol=1e-12, atol=1e-12 * np.abs(gd).max())


def test_hmode_is_the_two_map_model_on_the_line_delta_gamma_mu():
    """h-mode = two-map model at (mu, delta) = (h, gamma h): equal cost, and by the chain rule
    grad h = grad mu + gamma grad delta (with the regulariser on h only)."""
    c, cfg, st = _setup(hmode=True, gamma=5.0)
    st2 = dataclasses.replace(st, hmode=False)
    rng = np.random.default_rng(2)
    h = _params(st, c, rng)
    lam = 3.0
    S, g = fm.cost_and_grad(st, h, c.s_exp, lam)
    S2, g2 = fm.cost_and_grad(st2, np.concatenate([h, 5.0 * h]), c.s_exp, lam, 0.0)
    nn = st.n * st.n
    assert S == pytest.approx(S2, rel=1e-14)
    assert np.allclose(g, g2[:nn] + 5.0 * g2[nn:], rtol=1e-12, atol=1e-12 * np.abs(g).max())


@pytest.mark.parametrize("kw", [dict(hmode=True, gamma=5.0), dict(fit_mo=True), dict(fit_mr=True),
                                dict(hmode=True, fit_mo=True, fit_mr=True)],
                         ids=["hmode", "drift", "ring", "hmode-drift-ring"])
def test_gradient_matches_central_differences(kw):
    c, cfg, st = _setup(**kw)
    rng = np.random.default_rng(3)
    p = _params(st, c, rng)
    nn = st.n * st.n
    idx = list(rng.choice(nn, 12, replace=False))
    if not st.hmode:
        idx += list(nn + rng.choice(nn, 6, replace=False))
    idx += list(range(st.n_maps * nn, st.n_params))          # every offset
    lam = (cfg.lam_mu, cfg.lam_delta)
    for i in idx:
        h = 1e-6 * (cfg.mu_scale if i < nn else (1e-3 if i < st.n_maps * nn else 1.0))
        _fd_check(st, p, c.s_exp, *lam, [i], h, 1e-5)


def test_gauge_ambiguity_of_drift_and_ring_terms():
    """m_o + a and m_r - a leave every model value unchanged (theory section): the cost is
    invariant along that line and its derivative along it, sum(dS/dm_o) - sum(dS/dm_r), is 0."""
    c, cfg, st = _setup(fit_mo=True, fit_mr=True)
    p = _params(st, c, np.random.default_rng(4))
    nn2 = 2 * st.n * st.n
    nt, nd = st.theta.size, st.n_det
    q = p.copy()
    q[nn2:nn2 + nt] += 0.037
    q[nn2 + nt:] -= 0.037
    S, g = fm.cost_and_grad(st, p, c.s_exp, cfg.lam_mu, cfg.lam_delta)
    Sq = fm.cost(st, q, c.s_exp, cfg.lam_mu, cfg.lam_delta)
    assert Sq == pytest.approx(S, rel=1e-13)
    gm, gr = g[nn2:nn2 + nt], g[nn2 + nt:]
    assert abs(gm.sum() - gr.sum()) <= 1e-10 * np.abs(g).max()
    # without the ring term the drift alone is identifiable: moving it changes the cost
    st1 = dataclasses.replace(st, fit_mr=False)
    p1 = p[:nn2 + nt]
    q1 = p1.copy()
    q1[nn2:] += 0.037
    assert abs(fm.cost(st1, q1, c.s_exp, cfg.lam_mu, cfg.lam_delta)
               - fm.cost(st1, p1, c.s_exp, cfg.lam_mu, cfg.lam_delta)) > 1e-3 * S


def test_no_sample_with_offsets_is_the_shifted_flat():
    """mu = delta = 0: s_mod[a][j][k] = A_k exp(-(m_j - m_o[a] - m_r[k] - c_k)^2 / (2 s_k^2))."""
    c, cfg, st = _setup(fit_mo=True, fit_mr=True)
    rng = np.random.default_rng(5)
    nn2 = 2 * st.n * st.n
    mo = 0.1 * rng.standard_normal(st.theta.size)
    mr = 0.1 * rng.standard_normal(st.n_det)
    p = np.concatenate([np.zeros(nn2), mo, mr])
    *_, s = fm.forward(st, p)
    u = c.mask_pos[None, :, None] - mo[:, None, None] - mr[None, None, :] - c.flat_ctr
    ref = c.flat_amp * np.exp(-u * u / (2 * c.flat_sigma ** 2))
    assert np.allclose(s, ref, rtol=1e-14, atol=0)


# ------------------------------------------------------------------ tabulated flats
def _table_setup(F, Q=33, **kw):
    c, cfg, st = _setup(**kw)
    return dataclasses.replace(st, flat_table=F, table_u0=-0.5, table_du=1.0 / (Q - 1)), c, cfg


def test_table_interpolation_reproduces_quadratics_and_nodes():
    Q = 33
    nd = 12
    uq = -0.5 + np.arange(Q) / (Q - 1)
    rng = np.random.default_rng(6)
    a, b, cq = rng.uniform(0.5, 1, nd), rng.uniform(-1, 1, nd), rng.uniform(-1, 1, nd)
    F = a[:, None] + b[:, None] * uq[None, :] + cq[:, None] * uq[None, :] ** 2
    st, _, _ = _table_setup(F)
    # interior cells: the four samples exist, cubic convolution is exact for degree <= 2
    u = rng.uniform(uq[1], uq[Q - 2], (50, nd))
    f, fp = fm.flat_ic(st, u)
    assert np.allclose(f, a + b * u + cq * u * u, rtol=0, atol=1e-14)
    assert np.allclose(fp, b + 2 * cq * u, rtol=0, atol=1e-12)
    # nodes return the table
    f, _ = fm.flat_ic(st, np.broadcast_to(uq[5:9, None], (4, nd)).copy())
    assert np.allclose(f, F[:, 5:9].T, rtol=0, atol=1e-15)
    # outside the scanned period: end values, zero slope
    f, fp = fm.flat_ic(st, np.full((2, nd), 0.7))
    assert np.allclose(f, F[:, -1], rtol=0, atol=1e-15) and np.all(fp == 0.0)


def test_table_of_a_gaussian_converges_at_third_order():
    """Sampling the Gaussian flat at Q and 2Q - 1 points: the interpolated value's error drops
    by about 8 (third order), the slope's by at least 4."""
    _, _, st0 = _setup()
    u = np.linspace(-0.35, 0.35, 401)[:, None] * np.ones(st0.n_det)
    f_true, fp_true = fm.flat_ic(st0, u)
    errs = []
    for Q in (17, 33, 65):
        uq = -0.5 + np.arange(Q) / (Q - 1)
        F = st0.flat_amp[:, None] * np.exp(-(uq[None, :] - st0.flat_ctr[:, None]) ** 2
                                           / (2 * st0.flat_sigma[:, None] ** 2))
        st = dataclasses.replace(st0, flat_table=F, table_u0=-0.5, table_du=1.0 / (Q - 1))
        f, fp = fm.flat_ic(st, u)
        errs.append((np.abs(f - f_true).max(), np.abs(fp - fp_true).max()))
    for (e1, d1), (e2, d2) in zip(errs[:-1], errs[1:]):
        assert e1 / e2 > 6.0 and d1 / d2 > 3.5, errs
    assert errs[1][0] < 1e-4


def test_tabulated_flat_gradient_matches_central_differences():
    rng = np.random.default_rng(7)
    Q = 33
    uq = -0.5 + np.arange(Q) / (Q - 1)
    _, _, st0 = _setup()
    F = np.exp(-(uq[None, :] ** 2) / (2 * 0.6 ** 2)) * (1 + 0.01 * rng.standard_normal((st0.n_det, Q)))
    st, c, cfg = _table_setup(F, hmode=True, gamma=5.0, fit_mo=True, fit_mr=True)
    p = _params(st, c, rng, off_amp=0.02)
    nn = st.n * st.n
    idx = list(rng.choice(nn, 10, replace=False)) + list(range(nn, st.n_params))
    for i in idx:
        h = 1e-6 * (cfg.mu_scale if i < nn else 1.0)
        _fd_check(st, p, c.s_exp, cfg.lam_mu, 0.0, [i], h, 1e-5)
