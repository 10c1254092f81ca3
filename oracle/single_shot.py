"""Oracle: non-iterative ("single shot") reconstruction used as the warm-start input.

TEST INFRASTRUCTURE ONLY (FP64 NumPy, shares no code with the HIP path).

The paper's single-shot route retrieves projections from the IC data and then applies a
filtered backprojection (scikit-image's inverse Radon transform, experiment section).
Its eq. 3 (one mask position, homogeneous object) is garbled in the source; with several
mask positions per IC the two channels can be retrieved independently, which is the
reading used here:

Retrieval, per projection pixel (a, k): from s_j = T A_k exp(-(m_j - Delta - c_k)^2/(2 s_k^2)),
    y_j = log s_j - log A_k + (m_j - c_k)^2 / (2 s_k^2) = alpha + beta (m_j - c_k)
with beta = Delta / s_k^2 and alpha = log T - Delta^2/(2 s_k^2). A least-squares line fit
weighted by w_j = s_j (Poisson: var(log s) ~ 1/s) gives
    Delta_hat = beta s_k^2,   log T_hat = alpha + Delta_hat^2 / (2 s_k^2).
Samples with s_j <= 0 get zero weight; a singular fit gives T_hat = 1, Delta_hat = 0.

Reconstruction: filtered backprojection with the Ram-Lak kernel of Kak & Slaney (cited for
eq. 1): h[0] = 1/4, h[n odd] = -1/(pi^2 n^2), h[n even != 0] = 0, linear (zero-padded)
convolution along t, then (pi / N_theta) R^T.
    mu_hat    = (pi/N_theta) R^T (h * (-log T_hat))
    delta_hat = (pi/N_theta) R^T (h * P_hat),  P_hat = trapezoid integral of Delta_hat/kappa
                along t minus the linear ramp that makes both ends zero.
"""
from __future__ import annotations

import numpy as np

from . import radon


def retrieve(s_exp: np.ndarray, mask_pos, amp, ctr, sig):
    """(log T_hat, Delta_hat) [n_theta][n_det] from s_exp [n_theta][n_mask][n_det]."""
    s = np.asarray(s_exp, dtype=np.float64)
    x = mask_pos[None, :, None] - ctr[None, None, :]
    pos = s > 0.0
    w = np.where(pos, s, 0.0)
    y = np.where(pos, np.log(np.where(pos, s, 1.0)), 0.0) - np.log(amp)[None, None, :] \
        + x * x / (2.0 * sig[None, None, :] ** 2)
    S0 = w.sum(1)
    S1 = (w * x).sum(1)
    S2 = (w * x * x).sum(1)
    Y0 = (w * y).sum(1)
    Y1 = (w * x * y).sum(1)
    det = S0 * S2 - S1 * S1
    ok = det > 1e-12 * np.maximum(S0 * S2, 1e-300)
    sdet = np.where(ok, det, 1.0)
    alpha = np.where(ok, (S2 * Y0 - S1 * Y1) / sdet, 0.0)
    beta = np.where(ok, (S0 * Y1 - S1 * Y0) / sdet, 0.0)
    s2 = sig[None, :] ** 2
    dl = beta * s2
    logT = alpha + dl * dl / (2.0 * s2)
    return logT, dl


def ramlak(n_det: int) -> np.ndarray:
    """Kernel values h[n] for n = -(n_det-1) ... (n_det-1)."""
    n = np.arange(-(n_det - 1), n_det)
    h = np.zeros(n.size)
    h[n == 0] = 0.25
    odd = (n % 2) != 0
    h[odd] = -1.0 / (np.pi ** 2 * n[odd].astype(np.float64) ** 2)
    return h


def ramp_filter(p: np.ndarray) -> np.ndarray:
    """Row-wise linear convolution with the Ram-Lak kernel, same length as the input."""
    n_det = p.shape[-1]
    h = ramlak(n_det)
    out = np.empty_like(p, dtype=np.float64)
    for a in range(p.shape[0]):
        full = np.convolve(p[a], h)                  # length 3 n_det - 2
        out[a] = full[n_det - 1: 2 * n_det - 1]
    return out


def integrate_refraction(dl: np.ndarray, kappa: float) -> np.ndarray:
    q = dl / kappa
    P = np.zeros_like(q)
    P[:, 1:] = np.cumsum(0.5 * (q[:, 1:] + q[:, :-1]), axis=1)
    n = q.shape[1]
    ramp = np.arange(n, dtype=np.float64) / max(n - 1, 1)
    return P - P[:, -1:] * ramp[None, :]


def fbp(p: np.ndarray, theta: np.ndarray, n: int) -> np.ndarray:
    return (np.pi / theta.size) * radon.backproject(ramp_filter(p), theta, n)


def reconstruct(s_exp, theta, n, mask_pos, amp, ctr, sig, kappa):
    logT, dl = retrieve(s_exp, mask_pos, amp, ctr, sig)
    mu = fbp(-logT, theta, n)
    de = fbp(integrate_refraction(dl, kappa), theta, n)
    return np.stack([mu, de])


# ---------------------------------------------------------------------------------------
# eq. 3: single-shot retrieval from ONE mask position for a homogeneous object (h-mode).
# Read (the printed equation carries gamma^-1 where eq. 4 and the homogeneity assumption
# put gamma): linearising s = T f(m - Delta) with Delta = kappa gamma d/dt R[h] and
# T d/dt R[h] = -d/dt T gives s/f = T + kappa gamma (f'/f) d/dt T, so in Fourier space along t
#   T = F^-1[ F[s/f] / (1 + i kappa gamma (f'(m)/f(m)) sin q) ],   R[h] = -log T,
# with f(m), f'(m) the detector-averaged flat and its slope at the mask position (the paper's
# definition) and i sin q the symbol of the central difference D (i q in the continuous
# equation). The division by the flat in F[s/f] is per pixel. Transmissions below
# EQ3_T_FLOOR are held at the floor before the logarithm.
EQ3_T_FLOOR = 1e-6


def eq3_symbol(n_det: int, beta: float) -> np.ndarray:
    """1 / (1 + i beta sin q_l), q_l = 2 pi l / n_det (numpy's DFT frequency order)."""
    q = 2.0 * np.pi * np.arange(n_det) / n_det
    return 1.0 / (1.0 + 1j * beta * np.sin(q))


def retrieve_eq3(s_m: np.ndarray, f_px: np.ndarray, f_mean: float, fp_mean: float,
                 kappa_gamma: float) -> np.ndarray:
    """R[h] [n_theta][n_det] from the data at one mask position s_m [n_theta][n_det], the flat
    at that position per pixel f_px [n_det], and the detector-averaged flat and slope."""
    r = np.asarray(s_m, dtype=np.float64) / np.asarray(f_px, dtype=np.float64)[None, :]
    sym = eq3_symbol(r.shape[1], kappa_gamma * fp_mean / f_mean)
    T = np.real(np.fft.ifft(np.fft.fft(r, axis=1) * sym[None, :], axis=1))
    return -np.log(np.maximum(T, EQ3_T_FLOOR))


def reconstruct_eq3(s_exp, theta, n, mask_index, flat_f, flat_fp, kappa_gamma):
    """h from eq. 3 at mask position mask_index and the filtered backprojection of R[h].
    flat_f, flat_fp: [n_det] flat IC and slope of every pixel at that position."""
    s_m = np.asarray(s_exp, dtype=np.float64)[:, mask_index, :]
    P = retrieve_eq3(s_m, flat_f, float(np.mean(flat_f)), float(np.mean(flat_fp)), kappa_gamma)
    return fbp(P, theta, n)
