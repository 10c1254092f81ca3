"""Pins for the oracle projector R, its transpose and the detector derivative D.

Each check is fixed by something other than the oracle itself: exact discrete special
cases, closed-form line integrals (Kak & Slaney's ellipse formula), analytic refraction
profiles of cylinders, the transpose identity and an independently derived closed form of
the system-matrix element.
"""
import numpy as np
import pytest

from oracle import radon
from paper_2202_08627_amd import synth
from helpers import rel_l2


def _asym_image(n, seed=0):
    rng = np.random.default_rng(seed)
    h = rng.standard_normal((n, n))
    h[: n // 3, :] += 3.0        # break every symmetry (rows vs columns, flips)
    return h


@pytest.mark.parametrize("n", [8, 17, 32])
def test_axis_angles_are_column_and_row_sums(n):
    """P1: theta = 0 integrates along y (column sums), theta = 90 deg along x (row sums)."""
    h = _asym_image(n)
    theta = np.array([0.0, np.pi / 2])
    P = radon.project(h, theta, n)
    assert np.allclose(P[0], h.sum(axis=0), rtol=0, atol=1e-12 * np.abs(h).sum())
    assert np.allclose(P[1], h.sum(axis=1), rtol=0, atol=1e-12 * np.abs(h).sum())


def test_row_flag_tie_rule():
    """|cos| >= |sin| decided in FP64; 45 deg is row-stepping, 135 deg column-stepping."""
    th = radon.angles(4)
    assert list(radon.row_flags(th)) == [True, True, False, False]
    assert np.cos(np.pi / 4) > np.sin(np.pi / 4)


def test_closed_form_matrix_element():
    """R[(a,k),(i,j)] = (1/w) max(0, 1 - |t_k - tau|/w), tau = x_i cos + y_j sin,
    w = |cos| (row-stepping) or |sin| (column-stepping): derived from the interpolation
    weight, independent of the ray loop."""
    n, nd = 9, 11
    th = np.concatenate([radon.angles(12), [0.3, 2.0, 2.6]])
    A = radon.system_matrix(n, th, nd)
    c = (n - 1) / 2
    x = np.arange(n) - c
    t = np.arange(nd) - (nd - 1) / 2
    rows = radon.row_flags(th)
    B = np.zeros_like(A)
    for a, tt in enumerate(th):
        w = abs(np.cos(tt)) if rows[a] else abs(np.sin(tt))
        tau = x[None, :] * np.cos(tt) + x[:, None] * np.sin(tt)     # [j][i]
        el = np.maximum(0.0, 1.0 - np.abs(t[:, None, None] - tau[None]) / w) / w
        B[a * nd:(a + 1) * nd] = el.reshape(nd, n * n)
    assert np.max(np.abs(A - B)) < 1e-13


@pytest.mark.parametrize("n,sb,tol", [(64, 4.0, 5e-3), (128, 8.0, 1.5e-3)])
def test_gaussian_blob_closed_form(n, sb, tol):
    """P2: point-sampled Gaussian projects to sqrt(2 pi) sb exp(-t^2 / 2 sb^2)."""
    c = (n - 1) / 2
    x = np.arange(n) - c
    h = np.exp(-(x[None, :] ** 2 + x[:, None] ** 2) / (2 * sb * sb))
    th = np.concatenate([radon.angles(36), [0.123, 1.0, 2.2]])
    P = radon.project(h, th, n)
    t = np.arange(n) - (n - 1) / 2
    ref = np.sqrt(2 * np.pi) * sb * np.exp(-t ** 2 / (2 * sb * sb))
    assert rel_l2(P, np.broadcast_to(ref, P.shape)) < tol


def test_gaussian_blob_second_order():
    errs = []
    for n, sb in ((64, 4.0), (128, 8.0)):
        c = (n - 1) / 2
        x = np.arange(n) - c
        h = np.exp(-(x[None, :] ** 2 + x[:, None] ** 2) / (2 * sb * sb))
        th = radon.angles(36)
        P = radon.project(h, th, n)
        t = np.arange(n) - (n - 1) / 2
        ref = np.sqrt(2 * np.pi) * sb * np.exp(-t ** 2 / (2 * sb * sb))
        errs.append(rel_l2(P, np.broadcast_to(ref, P.shape)))
    assert errs[0] / errs[1] > 3.5


def test_disk_and_ellipses_against_chord_formula():
    """P3: 4x4 area-fraction voxelisations against the analytic ellipse projections."""
    out = {}
    for n in (64, 128):
        th = radon.angles(36)
        t = np.arange(n) - (n - 1) / 2
        disk = np.array([[0.0, 0.0, 0.35 * n, 0.35 * n, 0.0, 1.0, 0.0]])
        ell = synth.random_ellipses(n, 5, np.random.default_rng(3))
        for name, e in (("disk", disk), ("ell", ell)):
            P = radon.project(synth.rasterize(e, n, 5), th, n)
            out[name, n] = rel_l2(P, synth.ellipse_line_integrals(e, 5, th, t))
    assert out["disk", 64] < 2.5e-2 and out["disk", 128] < 5e-3
    assert out["ell", 64] < 5e-2 and out["ell", 128] < 2.5e-2
    assert out["disk", 128] < out["disk", 64] and out["ell", 128] < out["ell", 64]


@pytest.mark.parametrize("n", [128, 256])
def test_uniform_cylinder_refraction(n):
    """P4: kappa D R[disk] against the analytic -2 kappa c t / sqrt(R^2 - t^2), |t| <= 0.8 R.
    The voxelised edge keeps this near 6 % at every N."""
    R, kappa, c0 = 0.35 * n, 10.0, 1.0
    e = np.array([[0.0, 0.0, R, R, 0.0, 0.0, c0]])
    P = radon.project(synth.rasterize(e, n, 6), radon.angles(12), n)
    t = np.arange(n) - (n - 1) / 2
    m = np.abs(t) <= 0.8 * R
    D = kappa * radon.deriv(P)[:, m]
    ref = -2 * kappa * c0 * t[m] / np.sqrt(R * R - t[m] ** 2)
    assert rel_l2(D, np.broadcast_to(ref, D.shape)) < 0.08


def test_smooth_cylinder_second_order():
    """P4': (1 - r^2/R^2)^2 projects to (16/15)(R^2-t^2)^(5/2)/R^4 with slope
    -(16/3) t (R^2-t^2)^(3/2)/R^4; the central difference converges at second order."""
    tol = {64: (1e-3, 1e-2), 128: (2.5e-4, 2.5e-3), 256: (7e-5, 7e-4)}
    for n in (64, 128, 256):
        R = 0.4 * n
        x = np.arange(n) - (n - 1) / 2
        r2 = x[None, :] ** 2 + x[:, None] ** 2
        h = np.where(r2 < R * R, (1 - r2 / (R * R)) ** 2, 0.0)
        P = radon.project(h, radon.angles(12), n)
        L2 = np.maximum(R * R - x ** 2, 0.0)
        refp = 16 / 15 * L2 ** 2.5 / R ** 4
        refd = -16 / 3 * x * L2 ** 1.5 / R ** 4
        assert rel_l2(P, np.broadcast_to(refp, P.shape)) < tol[n][0]
        assert rel_l2(radon.deriv(P), np.broadcast_to(refd, P.shape)) < tol[n][1]


@pytest.mark.parametrize("n,nd,nt", [(16, 16, 24), (21, 27, 17), (32, 40, 33)])
def test_adjoint_identity(n, nd, nt):
    """P5: <R x, y> = <x, R^T y> for the scatter transpose, and <D p, g> = <p, D^T g>."""
    rng = np.random.default_rng(n)
    th = np.sort(rng.uniform(0, np.pi, nt))
    x = rng.standard_normal((n, n))
    y = rng.standard_normal((nt, nd))
    Rx = radon.project(x, th, nd)
    RTy = radon.backproject(y, th, n)
    lhs, rhs = float(np.vdot(Rx, y)), float(np.vdot(x, RTy))
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(Rx) * np.linalg.norm(y)
    p = rng.standard_normal((nt, nd))
    g = rng.standard_normal((nt, nd))
    assert abs(np.vdot(radon.deriv(p), g) - np.vdot(p, radon.deriv_T(g))) < 1e-12 * nt * nd
    assert np.allclose(radon.deriv_T(g), -radon.deriv(g), atol=1e-15)


def test_backproject_matches_dense_transpose():
    n, nd = 7, 9
    th = radon.angles(10)
    A = radon.system_matrix(n, th, nd)
    y = np.random.default_rng(1).standard_normal((10, nd))
    assert np.allclose(radon.backproject(y, th, n).ravel(), A.T @ y.ravel(), atol=1e-13)


def test_derivative_of_linear_ramp():
    """D of a linear profile is its slope away from the zero-padded ends."""
    p = 0.3 * np.arange(20.0) + 1.0
    d = radon.deriv(p[None])[0]
    assert np.allclose(d[1:-1], 0.3, atol=1e-15)
    assert d[0] == pytest.approx(p[1] / 2) and d[-1] == pytest.approx(-p[-2] / 2)
