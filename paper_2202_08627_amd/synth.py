"""Seeded synthetic inputs for edge-illumination tomography.

This module is the only code shared by the GPU path's tests/benchmarks and the
CPU oracle. It simulates a measurement from continuous, analytic objects (ellipse
phantoms and their exact line integrals); it holds none of the discrete method
(no pixel-grid projector, no finite-difference derivative, no cost or gradient).

Physics of the simulated measurement (the paper's eq. 2 with the drift and ring
terms of eq. 4 set to zero):
    s(t, theta, m) = exp(-p_mu(t, theta)) * f_t(m - Delta(t, theta))
where p_mu is the exact line integral of mu, Delta = kappa * d/dt p_delta averaged
over the detector pixel (difference of the exact p_delta at the pixel edges, which
avoids generating the data with the reconstruction's own discretisation), and the
flat-field curve f_t is a per-pixel Gaussian A_t exp(-(u - c_t)^2 / (2 sigma_t^2)).
Counts are Poisson at `counts` photons for the flat peak; s_exp = counts / peak.

Ellipse line integrals follow the standard closed form for a uniform ellipse
(Kak & Slaney, cited in the theory section): p(t, theta) =
2 rho a b sqrt(alpha^2 - t'^2) / alpha^2 with
alpha^2 = a^2 cos^2(theta - phi) + b^2 sin^2(theta - phi) and
t' = t - x0 cos(theta) - y0 sin(theta).

Geometry convention: voxel (i, j) has centre (x_i, y_j) = (i - (N-1)/2, j - (N-1)/2),
stored as [j][i]; detector pixel k sits at t_k = k - (N_t-1)/2; angle a is
theta_a = a*pi/N_theta; a ray is the line x cos(theta) + y sin(theta) = t.
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np

from .configs import SliceConfig


@dataclass
class Phantom:
    # ellipse table: columns x0, y0, a, b, phi, v_mu, v_delta (pixel units)
    ellipses: np.ndarray
    n: int


@dataclass
class Case:
    cfg: SliceConfig
    theta: np.ndarray          # [n_theta] float64 radians
    mask_pos: np.ndarray       # [n_mask] float64 mask periods
    flat_amp: np.ndarray       # [n_det] float64
    flat_ctr: np.ndarray       # [n_det] float64
    flat_sigma: np.ndarray     # [n_det] float64
    s_exp: np.ndarray          # [n_theta][n_mask][n_det] float32 (canonical input)
    mu_true: np.ndarray        # [n][n] float64 (4x4 supersampled rasterisation)
    delta_true: np.ndarray     # [n][n] float64
    phantom: Phantom

    @property
    def x_true(self) -> np.ndarray:
        return np.stack([self.mu_true, self.delta_true])


def angles(n_theta: int) -> np.ndarray:
    return np.arange(n_theta, dtype=np.float64) * (np.pi / n_theta)


def mask_positions(n_mask: int) -> np.ndarray:
    """M positions spread evenly over one period, centred on the IC peak."""
    return (np.arange(n_mask, dtype=np.float64) + 0.5) / n_mask - 0.5


def random_ellipses(n: int, n_ell: int, rng: np.random.Generator, axis_max: float = 0.4) -> np.ndarray:
    """Random ellipses inside radius 0.9*n/2 (semi-axes U[0.08, axis_max] * n/2, at most
    0.8 * n/2); raw values U(0,1) per map."""
    half = n / 2.0
    a = rng.uniform(0.08, axis_max, n_ell) * half
    b = rng.uniform(0.08, axis_max, n_ell) * half
    phi = rng.uniform(0.0, np.pi, n_ell)
    rmax = 0.9 * half - np.maximum(a, b)
    rc = rmax * np.sqrt(rng.uniform(0.0, 1.0, n_ell))
    ang = rng.uniform(0.0, 2 * np.pi, n_ell)
    x0 = rc * np.cos(ang)
    y0 = rc * np.sin(ang)
    v_mu = rng.uniform(0.0, 1.0, n_ell)
    v_de = rng.uniform(0.0, 1.0, n_ell)
    return np.stack([x0, y0, a, b, phi, v_mu, v_de], axis=1)


def shepp_style_ellipses(n: int, n_inner: int, rng: np.random.Generator) -> np.ndarray:
    """Head-like phantom: a bright outer shell (ellipse pair) and seeded interior
    ellipses with independent mu and delta contrasts. Not the classical table."""
    half = n / 2.0
    rows = []
    A, B = 0.69 * 0.9 * half / 0.92, 0.9 * half            # outer shell, aspect 0.69:0.92
    rows.append([0.0, 0.0, A, B, 0.0, 1.0, 1.0])
    rows.append([0.0, -0.02 * half, 0.92 * A, 0.94 * B, 0.0, -0.75, -0.7])
    placed = 0
    while placed < n_inner:
        a = rng.uniform(0.05, 0.25) * half
        b = rng.uniform(0.05, 0.25) * half
        phi = rng.uniform(0.0, np.pi)
        # centre inside the inner ellipse, keeping the whole ellipse inside it
        r = max(a, b)
        u, v = rng.uniform(-1, 1, 2)
        x0 = u * max(0.92 * A - r, 0.0)
        y0 = -0.02 * half + v * max(0.94 * B - r, 0.0)
        if (x0 / (0.92 * A - r + 1e-9)) ** 2 + ((y0 + 0.02 * half) / (0.94 * B - r + 1e-9)) ** 2 > 1.0:
            continue
        rows.append([x0, y0, a, b, phi, rng.uniform(0.05, 0.4), rng.uniform(0.05, 0.4)])
        placed += 1
    return np.array(rows, dtype=np.float64)


def rasterize(ell: np.ndarray, n: int, col: int, ss: int = 4) -> np.ndarray:
    """Area-fraction voxelisation with ss x ss supersampling of column `col`."""
    c = (n - 1) / 2.0
    off = (np.arange(ss) + 0.5) / ss - 0.5
    xs = (np.arange(n)[:, None] + off[None, :]).reshape(-1) - c   # n*ss sub-sample coords
    out = np.zeros((n * ss, n * ss), dtype=np.float64)
    X = xs[None, :]
    Y = xs[:, None]
    for e in ell:
        x0, y0, a, b, phi = e[:5]
        v = e[col]
        if v == 0.0:
            continue
        cp, sp = np.cos(phi), np.sin(phi)
        dx = X - x0
        dy = Y - y0
        xp = dx * cp + dy * sp
        yp = -dx * sp + dy * cp
        out += v * ((xp / a) ** 2 + (yp / b) ** 2 <= 1.0)
    return out.reshape(n, ss, n, ss).mean(axis=(1, 3))


def ellipse_line_integrals(ell: np.ndarray, col: int, theta: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Exact line integrals [n_theta][len(t)] of the ellipse table's column `col`."""
    th = theta[:, None]
    out = np.zeros((theta.size, t.size), dtype=np.float64)
    for e in ell:
        x0, y0, a, b, phi = e[:5]
        v = e[col]
        if v == 0.0:
            continue
        al2 = a * a * np.cos(th - phi) ** 2 + b * b * np.sin(th - phi) ** 2
        tp = t[None, :] - x0 * np.cos(th) - y0 * np.sin(th)
        rad = np.maximum(al2 - tp * tp, 0.0)
        out += 2.0 * v * a * b * np.sqrt(rad) / al2
    return out


def make_phantom(cfg: SliceConfig, rng: np.random.Generator) -> Phantom:
    if cfg.phantom == "random":
        ell = random_ellipses(cfg.n, cfg.n_ellipses, rng, cfg.axis_max)
    elif cfg.phantom == "shepp":
        ell = shepp_style_ellipses(cfg.n, max(cfg.n_ellipses - 2, 1), rng)
    else:
        raise ValueError(cfg.phantom)
    return Phantom(ellipses=ell, n=cfg.n)


def scale_phantom(ph: Phantom, mu_max: float, delta_max: float):
    """Scale each map so its rasterised maximum equals the configured range top.
    Scaling the ellipse values keeps the analytic projections exact."""
    ell = ph.ellipses.copy()
    mu = rasterize(ell, ph.n, 5)
    de = rasterize(ell, ph.n, 6)
    smu = mu_max / mu.max() if mu.max() > 0 else 0.0
    sde = delta_max / de.max() if de.max() > 0 else 0.0
    ell[:, 5] *= smu
    ell[:, 6] *= sde
    return Phantom(ellipses=ell, n=ph.n), mu * smu, de * sde


def make_flats(cfg: SliceConfig, rng: np.random.Generator):
    amp = np.ones(cfg.n_det)
    ctr = np.zeros(cfg.n_det)
    if cfg.sigma_jitter > 0:
        sig = cfg.sigma * (1.0 + cfg.sigma_jitter * rng.uniform(-1.0, 1.0, cfg.n_det))
    else:
        sig = np.full(cfg.n_det, cfg.sigma)
    return amp, ctr, sig


def simulate(ph: Phantom, cfg: SliceConfig, theta, mask_pos, amp, ctr, sig,
             rng: np.random.Generator | None, counts: float | None = None) -> np.ndarray:
    """Noisy (or noiseless when rng is None) IC data [n_theta][n_mask][n_det]."""
    t = np.arange(cfg.n_det, dtype=np.float64) - (cfg.n_det - 1) / 2.0
    p_mu = ellipse_line_integrals(ph.ellipses, 5, theta, t)
    p_hi = ellipse_line_integrals(ph.ellipses, 6, theta, t + 0.5)
    p_lo = ellipse_line_integrals(ph.ellipses, 6, theta, t - 0.5)
    dlt = cfg.kappa * (p_hi - p_lo)                      # pixel-averaged refraction
    trans = np.exp(-p_mu)
    u = mask_pos[None, :, None] - dlt[:, None, :] - ctr[None, None, :]
    s = trans[:, None, :] * amp[None, None, :] * np.exp(-u * u / (2.0 * sig[None, None, :] ** 2))
    if rng is None:
        return s
    c = cfg.counts if counts is None else counts
    return rng.poisson(c * s) / c


def make_case(cfg: SliceConfig, seed: int | None = None, noise: bool = True) -> Case:
    """Build one seeded slice problem. The phantom, flats and noise are drawn from
    independent streams of one numpy Generator seeded by `seed` (default cfg.seed)."""
    seed = cfg.seed if seed is None else seed
    ss = np.random.SeedSequence([seed, cfg.n, cfg.n_theta, cfg.n_mask])
    r_ph, r_fl, r_no = [np.random.default_rng(s) for s in ss.spawn(3)]
    ph = make_phantom(cfg, r_ph)
    ph, mu, de = scale_phantom(ph, cfg.mu_scale, cfg.delta_scale)
    theta = angles(cfg.n_theta)
    m = mask_positions(cfg.n_mask)
    amp, ctr, sig = make_flats(cfg, r_fl)
    s = simulate(ph, cfg, theta, m, amp, ctr, sig, r_no if noise else None)
    return Case(cfg=cfg, theta=theta, mask_pos=m, flat_amp=amp, flat_ctr=ctr,
                flat_sigma=sig, s_exp=s.astype(np.float32), mu_true=mu,
                delta_true=de, phantom=ph)


def random_volume(n: int, rng: np.random.Generator, scale=(1.0, 1.0)) -> np.ndarray:
    """Dense random [2][n][n] test vector (for adjoint identities and parity)."""
    x = rng.standard_normal((2, n, n))
    x[0] *= scale[0]
    x[1] *= scale[1]
    return x


def disk_mask(n: int, radius_frac: float = 0.9) -> np.ndarray:
    c = (n - 1) / 2.0
    yy, xx = np.mgrid[0:n, 0:n] - c
    return (xx * xx + yy * yy) <= (radius_frac * n / 2.0) ** 2
