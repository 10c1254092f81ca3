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
    # measured flat IC (cfg.flat_scans >= 1): [n_det][n_table] at u_q = table_u0 + q*table_du
    flat_table: np.ndarray | None = None
    table_u0: float = -0.5
    table_du: float = 0.0
    drift_true: np.ndarray | None = None    # [n_theta] mask drift used to simulate, periods

    @property
    def x_true(self) -> np.ndarray:
        return np.stack([self.mu_true, self.delta_true])


def angles(n_theta: int, span: float = 1.0) -> np.ndarray:
    """theta_a = a * span * pi / n_theta (span 1: 180 degrees, 2: 360 degrees)."""
    return np.arange(n_theta, dtype=np.float64) * (span * np.pi / n_theta)


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


def measure_flat_table(cfg: SliceConfig, amp, ctr, sig, rng: np.random.Generator):
    """The flat IC measured without the sample over one mask period: n_table positions
    u_q = -1/2 + q/(n_table - 1), Poisson counts at flat_scans * counts photons for the peak.
    Returns (table [n_det][n_table], u0, du)."""
    Q = cfg.n_table
    u0, du = -0.5, 1.0 / (Q - 1)
    uq = u0 + du * np.arange(Q)
    f = amp[:, None] * np.exp(-(uq[None, :] - ctr[:, None]) ** 2 / (2.0 * sig[:, None] ** 2))
    c = cfg.counts * cfg.flat_scans
    return rng.poisson(c * f) / c, u0, du


def mask_drift(cfg: SliceConfig, rng: np.random.Generator) -> np.ndarray:
    """Seeded slow per-angle drift of the sample mask (two random Fourier modes over the scan),
    at most drift_amp periods."""
    a = np.arange(cfg.n_theta) / cfg.n_theta
    p1, p2 = rng.uniform(0, 2 * np.pi, 2)
    return cfg.drift_amp * (0.6 * np.sin(2 * np.pi * a + p1) + 0.4 * np.sin(6 * np.pi * a + p2))


def make_flats(cfg: SliceConfig, rng: np.random.Generator):
    amp = np.ones(cfg.n_det)
    ctr = np.zeros(cfg.n_det)
    if cfg.sigma_jitter > 0:
        sig = cfg.sigma * (1.0 + cfg.sigma_jitter * rng.uniform(-1.0, 1.0, cfg.n_det))
    else:
        sig = np.full(cfg.n_det, cfg.sigma)
    return amp, ctr, sig


def simulate(ph: Phantom, cfg: SliceConfig, theta, mask_pos, amp, ctr, sig,
             rng: np.random.Generator | None, counts: float | None = None,
             drift: np.ndarray | None = None) -> np.ndarray:
    """Noisy (or noiseless when rng is None) IC data [n_theta][n_mask][n_det]; `drift`
    [n_theta] offsets the sample mask per angle."""
    t = np.arange(cfg.n_det, dtype=np.float64) - (cfg.n_det - 1) / 2.0
    p_mu = ellipse_line_integrals(ph.ellipses, 5, theta, t)
    p_hi = ellipse_line_integrals(ph.ellipses, 6, theta, t + 0.5)
    p_lo = ellipse_line_integrals(ph.ellipses, 6, theta, t - 0.5)
    dlt = cfg.kappa * (p_hi - p_lo)                      # pixel-averaged refraction
    trans = np.exp(-p_mu)
    mo = np.zeros(theta.size) if drift is None else drift
    u = mask_pos[None, :, None] - mo[:, None, None] - dlt[:, None, :] - ctr[None, None, :]
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
    # the first three streams are those of the plain model; the others serve the variants
    r_ph, r_fl, r_no, r_tab, r_dr = [np.random.default_rng(s) for s in ss.spawn(5)]
    ph = make_phantom(cfg, r_ph)
    if cfg.gamma_h > 0:
        # homogeneous object: one material map h with mu = h and delta = gamma_h * h
        ph, mu, _ = scale_phantom(ph, cfg.mu_scale, cfg.delta_scale)
        ell = ph.ellipses.copy()
        ell[:, 6] = cfg.gamma_h * ell[:, 5]
        ph = Phantom(ellipses=ell, n=ph.n)
        de = cfg.gamma_h * mu
    else:
        ph, mu, de = scale_phantom(ph, cfg.mu_scale, cfg.delta_scale)
    theta = angles(cfg.n_theta, cfg.angle_span)
    m = np.asarray(cfg.mask_list, dtype=np.float64) if cfg.mask_list else mask_positions(cfg.n_mask)
    if m.size != cfg.n_mask:
        raise ValueError("mask_list must hold n_mask positions")
    amp, ctr, sig = make_flats(cfg, r_fl)
    drift = mask_drift(cfg, r_dr) if cfg.drift_amp > 0 else None
    s = simulate(ph, cfg, theta, m, amp, ctr, sig, r_no if noise else None, drift=drift)
    table, u0, du = (measure_flat_table(cfg, amp, ctr, sig, r_tab) if cfg.flat_scans >= 1
                     else (None, -0.5, 0.0))
    return Case(cfg=cfg, theta=theta, mask_pos=m, flat_amp=amp, flat_ctr=ctr,
                flat_sigma=sig, s_exp=s.astype(np.float32), mu_true=mu,
                delta_true=de, phantom=ph, flat_table=table, table_u0=u0, table_du=du,
                drift_true=drift)


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


# ---------------------------------------------------------------------------------------------
# 3-D stacks (combined-results section: a 220 x 220 x 75 volume of plastic granules of three
# materials, reconstructed slice by slice).

GRANULE_VALUES = (1.0, 0.62, 0.38)     # relative attenuation of the three granule materials


@dataclass
class Granule:
    x0: float
    y0: float
    z0: float
    a: float
    b: float
    c: float
    phi: float
    material: int


def granule_volume(n: int, n_slices: int, n_granules: int, rng: np.random.Generator):
    """Non-overlapping ellipsoidal granules (semi-axes a, b in the slice plane rotated by phi,
    c along the stack axis) inside the cylinder of radius 0.85 n/2, materials in turn."""
    half = n / 2.0
    out: list[Granule] = []
    tries = 0
    while len(out) < n_granules and tries < 200 * n_granules:
        tries += 1
        a = rng.uniform(0.12, 0.22) * half
        b = rng.uniform(0.12, 0.22) * half
        c = rng.uniform(0.25, 0.45) * n_slices
        rmax = 0.85 * half - max(a, b)
        rc = rmax * np.sqrt(rng.uniform())
        ang = rng.uniform(0, 2 * np.pi)
        g = Granule(rc * np.cos(ang), rc * np.sin(ang), rng.uniform(0, n_slices - 1), a, b, c,
                    rng.uniform(0, np.pi), len(out) % len(GRANULE_VALUES))
        # reject overlaps (bounding spheroids in the plane, full extent along the stack)
        ok = True
        for h in out:
            dxy = np.hypot(g.x0 - h.x0, g.y0 - h.y0)
            if dxy < max(g.a, g.b) + max(h.a, h.b) + 2.0 and abs(g.z0 - h.z0) < g.c + h.c:
                ok = False
                break
        if ok:
            out.append(g)
    return out


def stack_slice_ellipses(granules, z: float, mu_max: float) -> np.ndarray:
    """Ellipse table (x0, y0, a, b, phi, v_mu, v_delta) of the granules' cross-sections with
    the plane of slice z (v_delta filled by the caller)."""
    rows = []
    for g in granules:
        t = 1.0 - ((z - g.z0) / g.c) ** 2
        if t <= 0.0:
            continue
        s = np.sqrt(t)
        rows.append([g.x0, g.y0, g.a * s, g.b * s, g.phi, GRANULE_VALUES[g.material] * mu_max, 0.0])
    return np.array(rows, dtype=np.float64).reshape(-1, 7)


def make_stack(cfg: SliceConfig, n_slices: int, n_granules: int = 9, seed: int = 0,
               noise_seed: int | None = None) -> tuple[list, list]:
    """Seeded 3-D granule volume and one Case per slice (homogeneous object when cfg.gamma_h > 0,
    else delta proportional to mu with delta_scale for the brightest material). Every slice
    has its own flat-table and count noise (noise_seed selects an independent realisation of
    the same volume) and shares the mask drift. Returns (cases, granules)."""
    rng = np.random.default_rng([seed, cfg.n, n_slices, 7])
    granules = granule_volume(cfg.n, n_slices, n_granules, rng)
    ns = seed if noise_seed is None else noise_seed
    theta = angles(cfg.n_theta, cfg.angle_span)
    m = np.asarray(cfg.mask_list, dtype=np.float64) if cfg.mask_list else mask_positions(cfg.n_mask)
    ss = np.random.SeedSequence([seed, cfg.n, cfg.n_theta, 11])
    r_fl, r_dr = [np.random.default_rng(s) for s in ss.spawn(2)]
    amp, ctr, sig = make_flats(cfg, r_fl)
    drift = mask_drift(cfg, r_dr) if cfg.drift_amp > 0 else None
    ratio = cfg.gamma_h if cfg.gamma_h > 0 else cfg.delta_scale / cfg.mu_scale
    cases = []
    for z in range(n_slices):
        ell = stack_slice_ellipses(granules, float(z), cfg.mu_scale)
        ell[:, 6] = ratio * ell[:, 5]
        ph = Phantom(ellipses=ell, n=cfg.n)
        mu = rasterize(ell, cfg.n, 5) if ell.shape[0] else np.zeros((cfg.n, cfg.n))
        r_no, r_tab = [np.random.default_rng(s) for s in
                       np.random.SeedSequence([ns, z, cfg.n, 13]).spawn(2)]
        s = simulate(ph, cfg, theta, m, amp, ctr, sig, r_no, drift=drift)
        table, u0, du = (measure_flat_table(cfg, amp, ctr, sig, r_tab) if cfg.flat_scans >= 1
                         else (None, -0.5, 0.0))
        cases.append(Case(cfg=cfg, theta=theta, mask_pos=m, flat_amp=amp, flat_ctr=ctr,
                          flat_sigma=sig, s_exp=s.astype(np.float32), mu_true=mu,
                          delta_true=ratio * mu, phantom=ph, flat_table=table, table_u0=u0,
                          table_du=du, drift_true=drift))
    return cases, granules
