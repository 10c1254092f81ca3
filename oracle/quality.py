"""Oracle: image-quality measures of the combined-results and experiment sections.

TEST INFRASTRUCTURE ONLY (FP64 NumPy, shares no code with the HIP path).

Fourier ring correlation (eq. 6, as used for the resolution comparison of the experiment
section; the printed equation omits the sums over a ring and the real part, read here as the
standard definition): for two images of the same region with independent noise,
    FRC(r) = sum_{|k| in ring r} Re(F1(k) F2(k)^*) / sqrt(sum |F1(k)|^2 * sum |F2(k)|^2),
F the 2-D DFT of the N x N crop, ring r holding the frequencies (kx, ky) (integers in
[-N/2, N/2), DFT order) with round(sqrt(kx^2 + ky^2)) = r, r = 0 .. N/2 (beyond N/2 rings are
incomplete and dropped). The curve is smoothed by a Gaussian of one ring (the paper smooths
it; the width is not stated) over rings 1 .. N/2 with the weights renormalised at the ends, and
the resolution is N / r_c pixels, r_c the first ring (linear interpolation between rings) at
which the smoothed curve drops below the cutoff (0.5 in the paper).

Contrast-to-noise ratio (eq. 7): CNR = |mean_1 - mean_2| / sqrt(std_1^2 + std_2^2) over two
discs of radius rho around given centres (pixels whose centre lies within rho), population
standard deviations.
"""
from __future__ import annotations

import numpy as np

FRC_SMOOTH_RINGS = 1.0


def frc_curve(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """FRC(r) for r = 0 .. N/2 of two N x N images."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = a.shape[0]
    assert a.shape == b.shape == (n, n)
    F1, F2 = np.fft.fft2(a), np.fft.fft2(b)
    k = np.fft.fftfreq(n) * n
    r = np.rint(np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)).astype(np.int64)
    nr = n // 2 + 1
    num = np.zeros(nr)
    d1 = np.zeros(nr)
    d2 = np.zeros(nr)
    for q in range(nr):
        m = r == q
        num[q] = np.sum(np.real(F1[m] * np.conj(F2[m])))
        d1[q] = np.sum(np.abs(F1[m]) ** 2)
        d2[q] = np.sum(np.abs(F2[m]) ** 2)
    den = np.sqrt(d1 * d2)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)


def smooth(curve: np.ndarray, sigma: float = FRC_SMOOTH_RINGS) -> np.ndarray:
    """Gaussian smoothing over rings 1 .. end (ring 0 kept), weights renormalised."""
    out = curve.copy()
    r = np.arange(1, curve.size)
    for q in r:
        w = np.exp(-0.5 * ((r - q) / sigma) ** 2)
        out[q] = np.sum(w * curve[1:]) / np.sum(w)
    return out


def resolution(curve: np.ndarray, n: int, cutoff: float = 0.5, sigma: float = FRC_SMOOTH_RINGS):
    """(resolution in pixels, crossing ring) from an FRC curve; if the smoothed curve stays at
    or above the cutoff up to ring N/2, the Nyquist limit (n / (N/2), N/2)."""
    s = smooth(curve, sigma)
    for q in range(1, s.size):
        if s[q] < cutoff:
            if q == 1:
                rc = 1.0
            else:
                rc = (q - 1) + (s[q - 1] - cutoff) / (s[q - 1] - s[q])
            return n / rc, rc
    rc = float(s.size - 1)
    return n / rc, rc


def disc_mask(n: int, x0: float, y0: float, rho: float) -> np.ndarray:
    """Pixels (i, j) of an n x n image whose centres (i - (n-1)/2, j - (n-1)/2) lie within rho
    of (x0, y0) (the library's centred coordinates; the image is stored [j][i])."""
    c = (n - 1) / 2.0
    jj, ii = np.mgrid[0:n, 0:n]
    return (ii - c - x0) ** 2 + (jj - c - y0) ** 2 <= rho * rho


def cnr(img: np.ndarray, c1, c2, rho: float) -> float:
    img = np.asarray(img, dtype=np.float64)
    n = img.shape[0]
    v1 = img[disc_mask(n, c1[0], c1[1], rho)]
    v2 = img[disc_mask(n, c2[0], c2[1], rho)]
    return float(abs(v1.mean() - v2.mean()) / np.sqrt(v1.var() + v2.var()))
