"""Oracle: the paper's full forward model (theory section, eq. 4) and its cost (eq. 5), in
the generality the library supports.

TEST INFRASTRUCTURE ONLY (FP64 NumPy, shares no code with the HIP path).

Unknowns, in one flat parameter vector (raw units), in this order:
  maps   two-map mode: [mu][n][n], [delta][n][n] (eq. 2);
         h-mode: [h][n][n] with mu = h and delta = gamma h (the homogeneous-object assumption
         of the theory section that leads to eq. 4: exp(-R[h]) and the shift z gamma d/dt R[h]);
  m_o    [n_theta] per-angle offset of the sample mask (drift), if fitted (eq. 4);
  m_r    [n_det] per-pixel ring term, if fitted (eq. 4).
Model, with T = exp(-R mu), Delta = kappa D R delta (kappa plays the role of z, D the central
difference of the experiment section's finite differences):
  s_mod[a][j][k] = T[a][k] f_k(m_j - m_o[a] - m_r[k] - Delta[a][k])
Flat-field IC f_k: the analytic per-pixel Gaussian A_k exp(-(u - c_k)^2 / (2 s_k^2)), or a
table of measured values F[k][q] at u_q = u0 + q du (the experiment section scans one period
of the mask in 33 steps), interpolated by cubic convolution (Keys 1981, a = -1/2; C1, exact
for quadratics) and held at the end values outside [u_0, u_(Q-1)] (derivative 0 there).
Cost (eq. 5): S = sum (s_mod - s_exp)^2 + lam_mu ||mu||^2 + lam_delta ||delta||^2 in two-map
mode, S = sum (...)^2 + lam_h ||h||^2 in h-mode; the offsets are not regularised.
Gradient (chain rule), r = s_mod - s_exp, u = m_j - m_o - m_r - Delta:
  G_T[a][k]     = 2 sum_j r f_k(u)              G_Pmu = -T G_T
  G_Delta[a][k] = -2 T sum_j r f_k'(u)          G_Pdelta = kappa D^T G_Delta
  dS/dm_o[a] = sum_k G_Delta[a][k]             dS/dm_r[k] = sum_a G_Delta[a][k]
  (u depends on m_o, m_r and Delta with the same coefficient -1)
  two-map: grad mu = R^T G_Pmu + 2 lam_mu mu, grad delta = R^T G_Pdelta + 2 lam_delta delta
  h-mode:  grad h = R^T (G_Pmu + gamma G_Pdelta) + 2 lam_h h
The paper notes the gauge ambiguity m_o + a, m_r - a when both offsets are fitted; the cost
here has it too (both are unregularised).
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np

from . import radon


@dataclass
class Setup:
    n: int
    theta: np.ndarray              # [n_theta] radians
    n_det: int
    mask_pos: np.ndarray           # [n_mask] mask periods
    flat_amp: np.ndarray           # [n_det] Gaussian flats (used when flat_table is None)
    flat_ctr: np.ndarray
    flat_sigma: np.ndarray
    kappa: float
    hmode: bool = False
    gamma: float = 5.0
    fit_mo: bool = False
    fit_mr: bool = False
    flat_table: np.ndarray | None = None    # [n_det][Q] measured flat IC
    table_u0: float = -0.5
    table_du: float = 1.0 / 32.0

    @property
    def n_maps(self) -> int:
        return 1 if self.hmode else 2

    @property
    def n_params(self) -> int:
        return self.n_maps * self.n * self.n + (self.theta.size if self.fit_mo else 0) \
            + (self.n_det if self.fit_mr else 0)


def unpack(st: Setup, p: np.ndarray):
    """(mu, delta, m_o, m_r) in raw units from the flat parameter vector."""
    p = np.asarray(p, dtype=np.float64).ravel()
    nn = st.n * st.n
    if st.hmode:
        h = p[:nn].reshape(st.n, st.n)
        mu, de, off = h, st.gamma * h, nn
    else:
        mu, de, off = p[:nn].reshape(st.n, st.n), p[nn:2 * nn].reshape(st.n, st.n), 2 * nn
    mo = np.zeros(st.theta.size)
    mr = np.zeros(st.n_det)
    if st.fit_mo:
        mo = p[off:off + st.theta.size]
        off += st.theta.size
    if st.fit_mr:
        mr = p[off:off + st.n_det]
    return mu, de, mo, mr


def keys_weights(t):
    """Cubic-convolution weights (a = -1/2) of the samples q-1, q, q+1, q+2 at fraction t, and
    their derivatives in t."""
    t2, t3 = t * t, t * t * t
    w = [0.5 * (-t3 + 2.0 * t2 - t), 0.5 * (3.0 * t3 - 5.0 * t2 + 2.0),
         0.5 * (-3.0 * t3 + 4.0 * t2 + t), 0.5 * (t3 - t2)]
    dw = [0.5 * (-3.0 * t2 + 4.0 * t - 1.0), 0.5 * (9.0 * t2 - 10.0 * t),
          0.5 * (-9.0 * t2 + 8.0 * t + 1.0), 0.5 * (3.0 * t2 - 2.0 * t)]
    return w, dw


def flat_ic(st: Setup, u: np.ndarray):
    """(f_k(u), f_k'(u)) for u broadcast over a trailing detector axis."""
    if st.flat_table is None:
        d = u - st.flat_ctr
        f = st.flat_amp * np.exp(-d * d / (2.0 * st.flat_sigma ** 2))
        return f, -d / st.flat_sigma ** 2 * f
    F = np.asarray(st.flat_table, dtype=np.float64)           # [n_det][Q]
    Q = F.shape[1]
    lo, hi = st.table_u0, st.table_u0 + (Q - 1) * st.table_du
    inside = (u >= lo) & (u <= hi)
    uc = np.clip(u, lo, hi)
    xq = (uc - lo) / st.table_du
    q = np.clip(np.floor(xq).astype(np.int64), 0, Q - 2)
    t = xq - q
    w, dw = keys_weights(t)
    k = np.broadcast_to(np.arange(st.n_det), u.shape)
    f = np.zeros(u.shape)
    fp = np.zeros(u.shape)
    for s in range(4):
        v = F[k, np.clip(q - 1 + s, 0, Q - 1)]
        f += w[s] * v
        fp += dw[s] * v
    return f, np.where(inside, fp / st.table_du, 0.0)


def forward(st: Setup, p: np.ndarray):
    """(P_mu, P_delta, T, Delta, u, s_mod[n_theta][n_mask][n_det])."""
    mu, de, mo, mr = unpack(st, p)
    P_mu = radon.project(mu, st.theta, st.n_det)
    P_de = radon.project(de, st.theta, st.n_det)
    T = np.exp(-P_mu)
    Dl = st.kappa * radon.deriv(P_de)
    u = st.mask_pos[None, :, None] - mo[:, None, None] - mr[None, None, :] - Dl[:, None, :]
    f, _ = flat_ic(st, u)
    return P_mu, P_de, T, Dl, u, T[:, None, :] * f


def cost(st: Setup, p, s_exp, lam_mu: float, lam_delta: float = 0.0) -> float:
    """S of eq. 5; in h-mode lam_mu is the weight on ||h||^2 and lam_delta is unused."""
    mu, de, _, _ = unpack(st, p)
    *_, s_mod = forward(st, p)
    r = s_mod - np.asarray(s_exp, dtype=np.float64)
    reg = lam_mu * np.sum(mu * mu) if st.hmode else lam_mu * np.sum(mu * mu) + lam_delta * np.sum(de * de)
    return float(np.sum(r * r) + reg)


def cost_and_grad(st: Setup, p, s_exp, lam_mu: float, lam_delta: float = 0.0):
    """(S, dS/dp) with dS/dp in the parameter vector's layout."""
    p = np.asarray(p, dtype=np.float64).ravel()
    mu, de, mo, mr = unpack(st, p)
    _, _, T, Dl, u, s_mod = forward(st, p)
    r = s_mod - np.asarray(s_exp, dtype=np.float64)
    f, fp = flat_ic(st, u)
    G_T = 2.0 * np.sum(r * f, axis=1)
    G_Dl = -2.0 * T * np.sum(r * fp, axis=1)
    G_Pmu = -T * G_T
    G_Pde = st.kappa * radon.deriv_T(G_Dl)
    nn = st.n * st.n
    g = np.zeros(p.size)
    if st.hmode:
        g[:nn] = (radon.backproject(G_Pmu + st.gamma * G_Pde, st.theta, st.n)
                  + 2.0 * lam_mu * mu).ravel()
        off = nn
        S = float(np.sum(r * r) + lam_mu * np.sum(mu * mu))
    else:
        g[:nn] = (radon.backproject(G_Pmu, st.theta, st.n) + 2.0 * lam_mu * mu).ravel()
        g[nn:2 * nn] = (radon.backproject(G_Pde, st.theta, st.n) + 2.0 * lam_delta * de).ravel()
        off = 2 * nn
        S = float(np.sum(r * r) + lam_mu * np.sum(mu * mu) + lam_delta * np.sum(de * de))
    if st.fit_mo:
        g[off:off + st.theta.size] = G_Dl.sum(axis=1)
        off += st.theta.size
    if st.fit_mr:
        g[off:off + st.n_det] = G_Dl.sum(axis=0)
    return S, g


class ScaledProblem:
    """The cost in scaled unknowns for the optimiser: maps divided by map_scale (two-map mode:
    (mu_s, delta_s); h-mode: h_s), offsets by offset_scale; lam weights ||z_maps||^2, i.e. in
    raw units lam/mu_s^2 and lam/delta_s^2 (h-mode: lam/h_s^2)."""

    def __init__(self, st: Setup, s_exp, lam: float, map_scale, offset_scale: float = 1.0):
        self.st = st
        self.s_exp = np.asarray(s_exp, dtype=np.float64)
        nn = st.n * st.n
        sc = np.full(st.n_params, float(offset_scale))
        ms = np.atleast_1d(np.asarray(map_scale, dtype=np.float64))
        for c in range(st.n_maps):
            sc[c * nn:(c + 1) * nn] = ms[c]
        self.scale = sc
        self.lam_raw = [lam / ms[c] ** 2 for c in range(st.n_maps)]

    def to_z(self, p):
        return np.asarray(p, dtype=np.float64).ravel() / self.scale

    def to_p(self, z):
        return np.asarray(z, dtype=np.float64).ravel() * self.scale

    def __call__(self, z):
        S, g = cost_and_grad(self.st, self.to_p(z), self.s_exp, *self.lam_raw)
        return S, g * self.scale
