"""Pins for the oracle IC model, cost and analytic gradient (eq. 2, eq. 4 with m_o = m_r = 0,
eq. 5). Checked against the no-sample identity s = f, a closed-form shifted Gaussian,
central finite differences and torch.autograd over a dense system matrix (FP64, CPU)."""
import numpy as np
import pytest
import torch

from oracle import model, radon
from paper_2202_08627_amd import synth
from helpers import geometry, tiny_cfg


def _case(seed=0, **kw):
    c = synth.make_case(tiny_cfg(**kw), seed=seed)
    return c, geometry(c, model)


def test_no_sample_gives_flat_field():
    """P6: mu = delta = 0 => T = 1, Delta = 0, s_mod = f(m) exactly."""
    c, geo = _case()
    n = c.cfg.n
    _, _, T, Dl, s = model.forward(np.zeros((n, n)), np.zeros((n, n)), geo)
    assert np.all(T == 1.0) and np.all(Dl == 0.0)
    f = c.flat_amp * np.exp(-(c.mask_pos[:, None] - c.flat_ctr) ** 2 / (2 * c.flat_sigma ** 2))
    assert np.array_equal(s, np.broadcast_to(f, s.shape))


def test_constant_attenuation_linear_phase_closed_form():
    """P7: constant P_mu and linear P_delta give constant T and Delta in the interior and
    s(m) = T A exp(-(m - Delta - c)^2 / 2 sigma^2) (the IC shifted by Delta)."""
    c, geo = _case(jitter=0.05)
    nt, nd = c.cfg.n_theta, c.cfg.n_det
    P_mu = np.full((nt, nd), 0.37)
    slope = 0.004
    P_de = slope * np.arange(nd)[None, :] + np.linspace(0, 1, nt)[:, None]
    T, Dl, s = model.ic_model(P_mu, P_de, geo)
    assert np.allclose(T, np.exp(-0.37), rtol=1e-15)
    assert np.allclose(Dl[:, 1:-1], geo.kappa * slope, rtol=1e-12)
    d = geo.kappa * slope
    ref = np.exp(-0.37) * c.flat_amp * np.exp(-(c.mask_pos[:, None] - d - c.flat_ctr) ** 2
                                              / (2 * c.flat_sigma ** 2))
    assert np.max(np.abs(s[:, :, 1:-1] - ref[None, :, 1:-1])) < 1e-14


def test_gradient_central_differences():
    """P8: analytic gradient vs central differences (h = 1e-6) in the scaled unknowns."""
    c, geo = _case()
    cfg = c.cfg
    prob = model.ScaledProblem(c.s_exp, geo, cfg.lam, cfg.mu_scale, cfg.delta_scale)
    rng = np.random.default_rng(5)
    z = prob.to_z(c.x_true) + 0.1 * rng.standard_normal(c.x_true.shape)
    _, g = prob(z)
    h = 1e-6
    fd = np.zeros_like(z)
    for q in range(z.size):
        e = np.zeros(z.size)
        e[q] = h
        e = e.reshape(z.shape)
        fd.flat[q] = (prob(z + e)[0] - prob(z - e)[0]) / (2 * h)
    assert np.max(np.abs(fd - g)) < 1e-8 * np.max(np.abs(g))


def test_gradient_autograd_dense_brute_force():
    """P9: cost via the dense system matrix and library autograd (torch, FP64, CPU)."""
    c, geo = _case(seed=2)
    cfg = c.cfg
    n, nt, nd = cfg.n, cfg.n_theta, cfg.n_det
    A = torch.tensor(radon.system_matrix(n, c.theta, nd))
    rng = np.random.default_rng(7)
    x0 = c.x_true + 0.2 * np.stack([cfg.mu_scale * rng.standard_normal((n, n)),
                                    cfg.delta_scale * rng.standard_normal((n, n))])
    mu = torch.tensor(x0[0], requires_grad=True)
    de = torch.tensor(x0[1], requires_grad=True)
    Pm = (A @ mu.reshape(-1)).reshape(nt, nd)
    Pd = (A @ de.reshape(-1)).reshape(nt, nd)
    Pd_pad = torch.nn.functional.pad(Pd, (1, 1))
    Dl = cfg.kappa * 0.5 * (Pd_pad[:, 2:] - Pd_pad[:, :-2])
    m = torch.tensor(c.mask_pos)[None, :, None]
    A_, c_, s_ = (torch.tensor(v) for v in (c.flat_amp, c.flat_ctr, c.flat_sigma))
    u = m - Dl[:, None, :]
    s_mod = torch.exp(-Pm)[:, None, :] * A_ * torch.exp(-(u - c_) ** 2 / (2 * s_ ** 2))
    r = s_mod - torch.tensor(c.s_exp.astype(np.float64))
    S = (r * r).sum() + cfg.lam_mu * (mu * mu).sum() + cfg.lam_delta * (de * de).sum()
    S.backward()
    S_o, gm, gd = model.cost_and_grad(x0[0], x0[1], c.s_exp, geo, cfg.lam_mu, cfg.lam_delta)
    assert S_o == pytest.approx(S.item(), rel=1e-12)
    assert np.max(np.abs(gm - mu.grad.numpy())) <= 1e-12 * np.max(np.abs(gm))
    assert np.max(np.abs(gd - de.grad.numpy())) <= 1e-12 * np.max(np.abs(gd))


def test_cost_matches_cost_and_grad_and_scaling():
    c, geo = _case(seed=3)
    cfg = c.cfg
    x = c.x_true * 0.9
    S1 = model.cost(x[0], x[1], c.s_exp, geo, cfg.lam_mu, cfg.lam_delta)
    S2, gm, gd = model.cost_and_grad(x[0], x[1], c.s_exp, geo, cfg.lam_mu, cfg.lam_delta)
    assert S1 == pytest.approx(S2, rel=1e-14)
    prob = model.ScaledProblem(c.s_exp, geo, cfg.lam, cfg.mu_scale, cfg.delta_scale)
    F, gz = prob(prob.to_z(x))
    assert F == pytest.approx(S2, rel=1e-12)
    assert np.allclose(gz[0], cfg.mu_scale * gm, rtol=1e-12, atol=1e-14)
    assert np.allclose(gz[1], cfg.delta_scale * gd, rtol=1e-12, atol=1e-14)


def test_noiseless_phantom_matches_analytic_simulation():
    """Noiseless data simulated from exact line integrals agree with the discrete model at
    the true phantom up to edge-voxel discretisation error, which shrinks with N, and fix
    the sign of the refraction term: flipping or dropping delta, or dropping mu, makes the
    mismatch clearly larger."""
    out = {}
    for n, nt in ((64, 90), (128, 180)):
        cfg = tiny_cfg(n=n, n_theta=nt)
        c = synth.make_case(cfg, noise=False)
        geo = geometry(c, model)

        def rms(mu, de):
            *_, s_mod = model.forward(mu, de, geo)
            r = s_mod - c.s_exp
            return np.sqrt(np.mean(r * r))
        out[n] = (rms(c.mu_true, c.delta_true), rms(c.mu_true, -c.delta_true),
                  rms(c.mu_true, 0 * c.delta_true), rms(0 * c.mu_true, c.delta_true))
    r, flip, no_de, no_mu = out[128]
    assert r < 0.008 and out[128][0] < 0.6 * out[64][0]
    assert flip > 2 * r and no_de > 1.4 * r and no_mu > 10 * r
