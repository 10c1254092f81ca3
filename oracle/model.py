"""Oracle: edge-illumination forward model, least-squares cost and its analytic gradient.

TEST INFRASTRUCTURE ONLY (FP64 NumPy, shares no code with the HIP path).

Forward model (theory section, eq. 2, and eq. 4 with the drift m_o and ring term m_r
set to zero, the configuration the paper recommends once flats are well sampled):
    P_mu = R mu,  P_delta = R delta                         (eq. 1)
    T = exp(-P_mu)                                          (attenuation)
    Delta = kappa * D P_delta                               (refraction shift, z d/dt R[delta])
    s_mod[a][j][k] = T[a][k] * f_k(m_j - Delta[a][k]),  f_k(u) = A_k exp(-(u - c_k)^2 / (2 s_k^2))
Cost (eq. 5, with the regulariser split over the two maps):
    S = sum_{a,j,k} (s_mod - s_exp)^2 + lam_mu ||mu||^2 + lam_delta ||delta||^2
Gradient (the paper defers it to earlier work; derived by the chain rule), r = s_mod - s_exp:
    G_T     = 2 sum_j r f_k(m_j - Delta)
    G_Delta = -2 T sum_j r f_k'(m_j - Delta),   f_k'(u) = -(u - c_k)/s_k^2 f_k(u)
    G_Pmu   = -T G_T
    G_Pdelta = kappa D^T G_Delta
    grad_mu = R^T G_Pmu + 2 lam_mu mu,   grad_delta = R^T G_Pdelta + 2 lam_delta delta
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np

from . import radon


@dataclass
class Geometry:
    n: int
    theta: np.ndarray            # [n_theta] radians (FP64)
    n_det: int
    mask_pos: np.ndarray         # [n_mask]
    flat_amp: np.ndarray         # [n_det]
    flat_ctr: np.ndarray         # [n_det]
    flat_sigma: np.ndarray       # [n_det]
    kappa: float

    @property
    def rows(self):
        return radon.row_flags(self.theta)


def flat_ic(geo: Geometry, u: np.ndarray) -> np.ndarray:
    """f_k(u) broadcast over a trailing detector axis."""
    return geo.flat_amp * np.exp(-(u - geo.flat_ctr) ** 2 / (2.0 * geo.flat_sigma ** 2))


def flat_ic_deriv(geo: Geometry, u: np.ndarray) -> np.ndarray:
    return -(u - geo.flat_ctr) / geo.flat_sigma ** 2 * flat_ic(geo, u)


def ic_model(P_mu: np.ndarray, P_de: np.ndarray, geo: Geometry):
    """IC model on the sinogram grid: (T, Delta, s_mod[n_theta][n_mask][n_det])."""
    T = np.exp(-P_mu)
    Dl = geo.kappa * radon.deriv(P_de)
    u = geo.mask_pos[None, :, None] - Dl[:, None, :]
    s_mod = T[:, None, :] * flat_ic(geo, u)
    return T, Dl, s_mod


def forward(mu: np.ndarray, delta: np.ndarray, geo: Geometry):
    """Returns (P_mu, P_delta, T, Delta, s_mod[n_theta][n_mask][n_det])."""
    P_mu = radon.project(mu, geo.theta, geo.n_det, geo.rows)
    P_de = radon.project(delta, geo.theta, geo.n_det, geo.rows)
    T, Dl, s_mod = ic_model(P_mu, P_de, geo)
    return P_mu, P_de, T, Dl, s_mod


def cost(mu, delta, s_exp, geo: Geometry, lam_mu: float, lam_delta: float) -> float:
    *_, s_mod = forward(mu, delta, geo)
    r = s_mod - np.asarray(s_exp, dtype=np.float64)
    return float(np.sum(r * r) + lam_mu * np.sum(mu * mu) + lam_delta * np.sum(delta * delta))


def sinogram_seeds(mu, delta, s_exp, geo: Geometry):
    """Cost data term and the adjoint seeds (G_Pmu, G_Pdelta) on the sinogram grid."""
    _, _, T, Dl, s_mod = forward(mu, delta, geo)
    r = s_mod - np.asarray(s_exp, dtype=np.float64)
    u = geo.mask_pos[None, :, None] - Dl[:, None, :]
    f = flat_ic(geo, u)
    fp = flat_ic_deriv(geo, u)
    G_T = 2.0 * np.sum(r * f, axis=1)
    G_Dl = -2.0 * T * np.sum(r * fp, axis=1)
    G_Pmu = -T * G_T
    G_Pde = geo.kappa * radon.deriv_T(G_Dl)
    return float(np.sum(r * r)), G_Pmu, G_Pde


def cost_and_grad(mu, delta, s_exp, geo: Geometry, lam_mu: float, lam_delta: float):
    """S and (grad_mu, grad_delta) in raw units."""
    data, G_Pmu, G_Pde = sinogram_seeds(mu, delta, s_exp, geo)
    g_mu = radon.backproject(G_Pmu, geo.theta, geo.n, geo.rows) + 2.0 * lam_mu * mu
    g_de = radon.backproject(G_Pde, geo.theta, geo.n, geo.rows) + 2.0 * lam_delta * delta
    S = data + lam_mu * float(np.sum(mu * mu)) + lam_delta * float(np.sum(delta * delta))
    return S, g_mu, g_de


class ScaledProblem:
    """The cost in the scaled unknowns z = [mu/mu_s ; delta/delta_s] with weight lam on
    ||z||^2 (lam_mu = lam/mu_s^2, lam_delta = lam/delta_s^2 in raw units).
    F(z) = S(mu_s z_mu, delta_s z_delta); grad_z F = [mu_s grad_mu ; delta_s grad_delta]."""

    def __init__(self, s_exp, geo: Geometry, lam: float, mu_scale: float, delta_scale: float):
        self.s_exp = np.asarray(s_exp, dtype=np.float64)
        self.geo = geo
        self.lam = lam
        self.scale = np.array([mu_scale, delta_scale], dtype=np.float64)
        self.n_evals = 0

    def to_z(self, x):
        return np.asarray(x, dtype=np.float64) / self.scale[:, None, None]

    def to_x(self, z):
        return np.asarray(z, dtype=np.float64) * self.scale[:, None, None]

    def __call__(self, z):
        self.n_evals += 1
        x = self.to_x(z)
        data, G_Pmu, G_Pde = sinogram_seeds(x[0], x[1], self.s_exp, self.geo)
        g = np.empty_like(x)
        g[0] = self.scale[0] * radon.backproject(G_Pmu, self.geo.theta, self.geo.n, self.geo.rows)
        g[1] = self.scale[1] * radon.backproject(G_Pde, self.geo.theta, self.geo.n, self.geo.rows)
        g += 2.0 * self.lam * z
        return data + self.lam * float(np.sum(z * z)), g
