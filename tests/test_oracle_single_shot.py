"""Pins for the oracle single-shot reconstruction (retrieval + filtered backprojection)."""
import os

import numpy as np

from oracle import radon, single_shot
from paper_2202_08627_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_ramlak_matches_textbook_values():
    rows = np.loadtxt(os.path.join(GOLDEN, "ramlak_kernel.txt"))
    h = single_shot.ramlak(8)           # n = -7..7
    for n, v in rows:
        assert abs(h[int(n) + 7] - v) < 1e-16
        assert abs(h[-int(n) + 7] - v) < 1e-16


def test_log_fit_recovers_noiseless_pixel():
    """P12a: a noiseless shifted, attenuated Gaussian IC gives back (T, Delta) exactly."""
    m = synth.mask_positions(8)
    amp = np.array([1.0, 0.8, 1.3])
    ctr = np.array([0.0, 0.05, -0.03])
    sig = np.array([0.6, 0.57, 0.63])
    T = np.array([[0.7, 0.2, 0.95]])
    dl = np.array([[0.12, -0.2, 0.0]])
    s = T[:, None, :] * amp * np.exp(-(m[:, None] - dl[:, None, :] - ctr) ** 2 / (2 * sig ** 2))
    logT, d = single_shot.retrieve(s, m, amp, ctr, sig)
    assert np.allclose(logT, np.log(T), atol=1e-12)
    assert np.allclose(d, dl, atol=1e-12)


def test_fbp_of_disk_recovers_value():
    """P12b: FBP of the exact projections of a uniform disk recovers its value
    (within 1 % on average inside 0.8 R)."""
    n, R, v = 128, 40.0, 0.7
    th = radon.angles(180)
    t = np.arange(n) - (n - 1) / 2
    e = np.array([[0.0, 0.0, R, R, 0.0, v, 0.0]])
    p = synth.ellipse_line_integrals(e, 5, th, t)
    img = single_shot.fbp(p, th, n)
    x = np.arange(n) - (n - 1) / 2
    inside = x[None, :] ** 2 + x[:, None] ** 2 < (0.8 * R) ** 2
    assert abs(img[inside].mean() - v) < 0.01 * v
    r2 = x[None, :] ** 2 + x[:, None] ** 2
    ring = (r2 > (1.2 * R) ** 2) & (r2 < (1.5 * R) ** 2)
    assert np.abs(img[ring]).mean() < 0.02 * v


def test_integrate_refraction_inverts_central_difference():
    """Trapezoid integral of a sampled derivative recovers a profile vanishing at both ends."""
    nd = 200
    t = np.arange(nd) - (nd - 1) / 2
    R = 60.0
    p = np.where(np.abs(t) < R, (R * R - t * t) ** 2 / R ** 3, 0.0)
    dp = np.where(np.abs(t) < R, -4 * t * (R * R - t * t) / R ** 3, 0.0)
    P = single_shot.integrate_refraction((10.0 * dp)[None], 10.0)[0]
    assert np.max(np.abs(P - p)) < 2e-3 * p.max()


def test_single_shot_small_case_is_close():
    from paper_2202_08627_amd import configs
    cfg = configs.SMALL_64
    c = synth.make_case(cfg)
    x = single_shot.reconstruct(c.s_exp, c.theta, cfg.n, c.mask_pos, c.flat_amp, c.flat_ctr,
                                c.flat_sigma, cfg.kappa)
    err_mu = np.linalg.norm(x[0] - c.mu_true) / np.linalg.norm(c.mu_true)
    err_de = np.linalg.norm(x[1] - c.delta_true) / np.linalg.norm(c.delta_true)
    assert err_mu < 0.5 and err_de < 0.7


# ------------------------------------------------------------------ eq. 3 (one mask position)
def _circ_diff(p):
    return 0.5 * (np.roll(p, -1, axis=-1) - np.roll(p, 1, axis=-1))


def test_eq3_inverts_the_linearised_model_exactly():
    """Data made by the linearised model s/f = T + beta D T (D the circular central difference,
    beta = kappa gamma f'/f): the retrieval returns -log T to rounding. A wrong sign of the
    derivative term, q in place of sin q, or beta missing its factor would not."""
    from oracle import single_shot as ss
    from paper_2202_08627_amd import synth
    nt, nd = 7, 64
    theta = synth.angles(nt)
    t = np.arange(nd) - (nd - 1) / 2
    P = 0.3 * synth.ellipse_line_integrals(np.array([[3.0, -2.0, 20.0, 14.0, 0.4, 0.02, 0.0]]),
                                           5, theta, t)
    T = np.exp(-P)
    f_px = np.full(nd, 0.8)
    fbar, fpbar, kg = 0.8, -0.9, 0.7
    beta = kg * fpbar / fbar
    s = f_px * (T + beta * _circ_diff(T))
    R = ss.retrieve_eq3(s, f_px, fbar, fpbar, kg)
    assert np.allclose(R, P, rtol=0, atol=1e-12)


def test_eq3_error_on_nonlinear_data_is_first_order_in_strength():
    """Data from the full h-mode model (oracle, one mask position on the slope of a Gaussian
    flat): the retrieval's relative error comes from the linearisation alone and halves when
    the object's strength halves."""
    from oracle import full_model as fm
    from oracle import single_shot as ss
    from paper_2202_08627_amd import synth
    n, nt = 32, 24
    theta = np.arange(nt) * (2 * np.pi / nt)
    m = np.array([0.24])
    nd = n
    amp, ctr, sig = np.ones(nd), np.zeros(nd), np.full(nd, 0.6)
    st = fm.Setup(n, theta, nd, m, amp, ctr, sig, kappa=0.14, hmode=True, gamma=5.0)
    yy, xx = np.mgrid[0:n, 0:n] - (n - 1) / 2
    disk = ((xx - 2) ** 2 + (yy + 1) ** 2 <= 9.0 ** 2).astype(float)
    f0 = np.exp(-(m[0]) ** 2 / (2 * 0.36))
    fp0 = -m[0] / 0.36 * f0
    errs = []
    for eps in (0.02, 0.01, 0.005):
        h = eps * disk
        P_mu, _, _, _, _, s = fm.forward(st, h.ravel())
        R = ss.retrieve_eq3(s[:, 0, :], np.full(nd, f0), f0, fp0, 0.14 * 5.0)
        errs.append(np.linalg.norm(R - P_mu) / np.linalg.norm(P_mu))
    assert errs[0] < 0.1
    assert errs[0] / errs[1] > 1.7 and errs[1] / errs[2] > 1.7, errs
