"""Oracle: parallel-beam projector R, its literal transpose, and the detector derivative D.

TEST INFRASTRUCTURE ONLY. Plain, slow, FP64 NumPy written from the paper; only the
test suite, the smoke check and the benchmark's CPU-baseline leg may use it. It
shares no code with the HIP path.

Radon transform (theory section, eq. 1): R[h](t, theta) is the integral of h along the
line L(t, theta). The paper fixes no discretisation beyond "linear interpolation with
indices computed on the fly" (algorithmic-improvements section). The reading used here
is Joseph's ray-driven method:

  voxel (i, j) (column i = x, row j = y) has centre (x_i, y_j) = (i - (N-1)/2, j - (N-1)/2),
  stored h[j][i]; detector pixel k is at t_k = k - (Nt-1)/2; angle theta_a; the ray is the
  line x cos(theta) + y sin(theta) = t.

  Row-stepping angle (|cos| >= |sin|, flag decided once in FP64): for every row j the ray
  crosses x = (t - y_j sin)/cos, i.e. fractional column u = x + (N-1)/2; the sample is the
  linear interpolation of row j at u (voxels outside the grid read as 0); the sum over rows
  is multiplied by the step length 1/|cos|.
  Column-stepping angle: the same with rows and columns exchanged (v = (t - x_i cos)/sin
  + (N-1)/2, interpolation along j, weight 1/|sin|).

The transpose is the literal scatter of that loop (every sample's two interpolation weights
are added back into the voxels they were read from), a deliberately different algorithm from
a per-voxel gather.

Detector derivative (finite differences, experimental-improvements section): central
difference with zero padding, (D p)[k] = (p[k+1] - p[k-1]) / 2, so D^T = -D.
"""
from __future__ import annotations

import numpy as np


def angles(n_theta: int) -> np.ndarray:
    """theta_a = a*pi/n_theta (uniform over 180 degrees, endpoint excluded)."""
    return np.arange(n_theta, dtype=np.float64) * (np.pi / n_theta)


def row_flags(theta: np.ndarray) -> np.ndarray:
    """True where the ray steps over rows: |cos| >= |sin| in FP64 (ties to rows)."""
    return np.abs(np.cos(theta)) >= np.abs(np.sin(theta))


def _axis_samples(n: int, n_det: int, th: float, row: bool):
    """Fractional interpolation coordinate u[step, k] and step weight for one angle."""
    c = (n - 1) / 2.0
    t = np.arange(n_det, dtype=np.float64) - (n_det - 1) / 2.0
    p = np.arange(n, dtype=np.float64) - c          # coordinate of the stepped axis
    cs, sn = np.cos(th), np.sin(th)
    if row:
        u = (t[None, :] - p[:, None] * sn) / cs + c
        w = 1.0 / abs(cs)
    else:
        u = (t[None, :] - p[:, None] * cs) / sn + c
        w = 1.0 / abs(sn)
    return u, w


def project(h: np.ndarray, theta: np.ndarray, n_det: int, rows: np.ndarray | None = None) -> np.ndarray:
    """R h for one map h[N][N] -> sinogram [n_theta][n_det] (Joseph, FP64)."""
    h = np.asarray(h, dtype=np.float64)
    n = h.shape[0]
    assert h.shape == (n, n)
    rows = row_flags(theta) if rows is None else rows
    out = np.zeros((theta.size, n_det), dtype=np.float64)
    steps = np.arange(n)[:, None]
    for a, th in enumerate(theta):
        u, w = _axis_samples(n, n_det, th, bool(rows[a]))
        i0 = np.floor(u).astype(np.int64)
        phi = u - i0
        src = h if rows[a] else h.T                 # src[step][interp]
        acc = np.zeros(u.shape)
        for off, wt in ((0, 1.0 - phi), (1, phi)):
            ii = i0 + off
            ok = (ii >= 0) & (ii < n)
            vals = np.where(ok, src[steps, np.clip(ii, 0, n - 1)], 0.0)
            acc += wt * vals
        out[a] = acc.sum(axis=0) * w
    return out


def backproject(g: np.ndarray, theta: np.ndarray, n: int, rows: np.ndarray | None = None) -> np.ndarray:
    """R^T g: scatter every sample weight of `project` back into its voxel."""
    g = np.asarray(g, dtype=np.float64)
    n_det = g.shape[1]
    rows = row_flags(theta) if rows is None else rows
    out_rows = np.zeros(n * n)   # image indexed [j][i]
    out_cols = np.zeros(n * n)   # transposed image indexed [i][j]
    steps = np.broadcast_to(np.arange(n)[:, None], (n, n_det))
    for a, th in enumerate(theta):
        u, w = _axis_samples(n, n_det, th, bool(rows[a]))
        i0 = np.floor(u).astype(np.int64)
        phi = u - i0
        ga = np.broadcast_to(g[a][None, :] * w, u.shape)
        target = out_rows if rows[a] else out_cols
        for off, wt in ((0, 1.0 - phi), (1, phi)):
            ii = i0 + off
            ok = (ii >= 0) & (ii < n)
            flat = steps[ok] * n + ii[ok]
            target += np.bincount(flat, weights=(wt * ga)[ok], minlength=n * n)
    return out_rows.reshape(n, n) + out_cols.reshape(n, n).T


def system_matrix(n: int, theta: np.ndarray, n_det: int, rows: np.ndarray | None = None) -> np.ndarray:
    """Dense R [(a,k), (j,i)] assembled column by column from `project` (tiny grids)."""
    A = np.zeros((theta.size * n_det, n * n))
    e = np.zeros((n, n))
    for q in range(n * n):
        e.flat[q] = 1.0
        A[:, q] = project(e, theta, n_det, rows).ravel()
        e.flat[q] = 0.0
    return A


def deriv(p: np.ndarray) -> np.ndarray:
    """Central difference along the last (detector) axis with zero padding."""
    q = np.zeros_like(p, dtype=np.float64)
    q[..., 1:-1] = (p[..., 2:] - p[..., :-2]) * 0.5
    q[..., 0] = p[..., 1] * 0.5
    q[..., -1] = -p[..., -2] * 0.5
    return q


def deriv_T(g: np.ndarray) -> np.ndarray:
    """Literal transpose of `deriv`: scatter +1/2 to k-1 and -1/2 to k+1 from each output k."""
    out = np.zeros_like(g, dtype=np.float64)
    nk = g.shape[-1]
    for k in range(nk):
        if k + 1 < nk:
            out[..., k + 1] += 0.5 * g[..., k]
        if k - 1 >= 0:
            out[..., k - 1] -= 0.5 * g[..., k]
    return out
