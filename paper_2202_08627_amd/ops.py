"""Python binding over libeitomo.so: torch tensors provide device memory and the stream,
every step runs in the library's HIP kernels. No CPU fallback exists: without the built
library or a GPU these functions raise."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _require(t, shape, dtype=torch.float32, name="tensor"):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _f64(a, n):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).ravel())
    if a.size < max(n, 0):
        raise ValueError(f"array of {a.size} values, {n} needed")
    return a


@dataclass
class Geometry:
    n: int
    n_theta: int
    n_det: int
    n_mask: int
    kappa: float
    theta: np.ndarray
    mask_pos: np.ndarray
    flat_amp: np.ndarray
    flat_ctr: np.ndarray
    flat_sigma: np.ndarray

    @classmethod
    def from_case(cls, case):
        c = case.cfg
        return cls(c.n, c.n_theta, c.n_det, c.n_mask, c.kappa, case.theta, case.mask_pos,
                   case.flat_amp, case.flat_ctr, case.flat_sigma)

    def c_args(self):
        """(dims, setup, arrays to keep alive); Gaussian flat parameters may be None when a
        model plan brings a measured flat table."""
        arrs = [_f64(self.theta, self.n_theta), _f64(self.mask_pos, self.n_mask)]
        arrs += [None if a is None else _f64(a, self.n_det)
                 for a in (self.flat_amp, self.flat_ctr, self.flat_sigma)]
        dims = L.Dims(self.n, self.n_theta, self.n_det, self.n_mask, float(self.kappa))
        setup = L.Setup(*[L.dptr(a) for a in arrs])
        return dims, setup, arrs


@dataclass
class Model:
    """Full-model options of eq. 4 (eit_model): h-mode (mu = h, delta = gamma h), fitted
    per-angle drift and per-pixel ring offsets, a measured flat table [n_det][Q] at
    u_q = table_u0 + q table_du."""
    hmode: bool = False
    gamma: float = 5.0
    fit_drift: bool = False
    fit_ring: bool = False
    flat_table: np.ndarray | None = None
    table_u0: float = -0.5
    table_du: float = 1.0 / 32.0
    offset_scale: float = 1.0
    eq3_mask: int = 0

    @classmethod
    def from_case(cls, case, hmode=None, fit_drift=False, fit_ring=False, use_table=None, **kw):
        """Options matching a simulated case: h-mode when the object is homogeneous, the
        measured flat table when the case has one (use_table=None)."""
        cfg = case.cfg
        hm = cfg.gamma_h > 0 if hmode is None else hmode
        tab = case.flat_table if (use_table is None or use_table) else None
        return cls(hmode=hm, gamma=cfg.gamma_h if cfg.gamma_h > 0 else 5.0, fit_drift=fit_drift,
                   fit_ring=fit_ring, flat_table=tab, table_u0=case.table_u0,
                   table_du=case.table_du if tab is not None else 1.0 / 32.0, **kw)

    def c_args(self, n_det: int):
        tab = None
        if self.flat_table is not None:
            tab = np.ascontiguousarray(np.asarray(self.flat_table, dtype=np.float64))
            if tab.ndim != 2 or tab.shape[0] != n_det:
                raise ValueError(f"flat_table must be [n_det][Q], got {tab.shape}")
        m = L.Model(1 if self.hmode else 0, 1 if self.fit_drift else 0, 1 if self.fit_ring else 0,
                    0 if tab is None else tab.shape[1], float(self.gamma), L.dptr(tab),
                    float(self.table_u0), float(self.table_du), float(self.offset_scale),
                    int(self.eq3_mask), 0)
        return m, tab


def inspect(geo: Geometry, proj_variant: int = -1, adj_variant: int = -1, adj_splits: int = 0,
            tables: bool = False):
    """Host-only plan diagnostics (no GPU needed): sizes and, optionally, the FP64 tables."""
    dims, setup, keep = geo.c_args()
    til = L.Tiling(proj_variant, adj_variant, adj_splits)
    info = L.PlanInfo()
    L.check(L.lib().eit_plan_inspect(C.byref(dims), C.byref(setup), C.byref(til), C.byref(info),
                                     None, None, None, None))
    out = {f: getattr(info, f) for f, _ in L.PlanInfo._fields_}
    if tables:
        pa = np.zeros(6 * geo.n_theta)
        gr = np.zeros(info.n_groups * info.proj_a, dtype=np.int32)
        wl = np.zeros(info.n_groups * info.n_dblk * info.n_strips, dtype=np.int32)
        aa = np.zeros(10 * geo.n_theta)
        L.check(L.lib().eit_plan_inspect(C.byref(dims), C.byref(setup), C.byref(til), C.byref(info),
                                         L.dptr(pa), gr.ctypes.data_as(L.IP), wl.ctypes.data_as(L.IP),
                                         L.dptr(aa)))
        out["proj_angles"] = pa.reshape(-1, 6)
        out["groups"] = gr.reshape(info.n_groups, info.proj_a)
        out["win_lo"] = wl.reshape(info.n_groups, info.n_dblk, info.n_strips)
        out["adj_angles"] = aa.reshape(-1, 10)
    del keep
    return out


def variants(kind: int):
    """Tile shapes of the compiled variants: projector (kind 0) as (angles per group,
    detectors per block, rows per strip, duplicated 16-byte LDS entries 0/1); adjoint
    (kind 1) as (tile x, tile y, angles -- or angle pairs -- per chunk, voxels per thread,
    mirror-pair kernel 0/1)."""
    n = L.lib().eit_variant_info(kind, -1, None, None, None, None)
    out = []
    for v in range(n):
        a, b, c, e = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        L.lib().eit_variant_info(kind, v, C.byref(a), C.byref(b), C.byref(c), C.byref(e))
        if kind == 0:
            dup = C.c_int32()
            L.lib().eit_variant_info(2, v, C.byref(dup), None, None, None)
            out.append((a.value, b.value, c.value, dup.value))
        else:
            mir = C.c_int32()
            L.lib().eit_variant_info(3, v, C.byref(mir), None, None, None)
            out.append((a.value, b.value, c.value, e.value, mir.value))
    return out


class Plan:
    """Owns one eit_plan (device angle/detector tables) for a slice geometry."""

    def __init__(self, geo: Geometry, proj_variant: int = -1, adj_variant: int = -1,
                 adj_splits: int = 0, model: Model | None = None):
        """adj_splits: blocks per adjoint voxel tile (0 = the library's automatic choice).
        model: full-model options of eq. 4 (None: the plain two-map model)."""
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required")
        self.geo = geo
        self.model = model
        dims, setup, keep = geo.c_args()
        til = L.Tiling(proj_variant, adj_variant, adj_splits)
        h = C.c_void_p()
        torch.cuda.current_device()
        if model is None:
            L.check(L.lib().eit_plan_create(C.byref(dims), C.byref(setup), C.byref(til), C.byref(h)))
        else:
            m, tab = model.c_args(geo.n_det)
            L.check(L.lib().eit_plan_create_model(C.byref(dims), C.byref(setup), C.byref(m),
                                                  C.byref(til), C.byref(h)))
            del tab
        del keep
        self._h = h
        self.n_params = int(L.lib().eit_param_count(h))
        self.device = torch.device("cuda", torch.cuda.current_device())

    @classmethod
    def from_case(cls, case, **kw):
        return cls(Geometry.from_case(case), **kw)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan destroyed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            L.lib().eit_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- helpers
    @property
    def x_shape(self):
        return (2, self.geo.n, self.geo.n)

    @property
    def param_shape(self):
        """Shape of x / gradient / reconstruction: [2][n][n] for the plain model, the flat
        parameter vector (maps, then offsets) for a model plan."""
        return self.x_shape if self.model is None else (self.n_params,)

    @property
    def sino_shape(self):
        return (2, self.geo.n_theta, self.geo.n_det)

    @property
    def data_shape(self):
        return (self.geo.n_theta, self.geo.n_mask, self.geo.n_det)

    def workspace_bytes(self, op: int, m: int = 10) -> int:
        return int(L.lib().eit_workspace_bytes(self.handle, op, m))

    def workspace(self, op: int, m: int = 10):
        nb = self.workspace_bytes(op, m)
        if nb == 0:
            raise ValueError("invalid workspace request")
        return torch.empty(nb, dtype=torch.uint8, device=self.device)

    # -------------------------------------------------------------- operators
    def project(self, x, out=None, ws=None):
        _require(x, self.x_shape, name="x")
        out = torch.empty(self.sino_shape, dtype=torch.float32, device=x.device) if out is None else out
        ws = self.workspace(L.EIT_OP_PROJECT) if ws is None else ws
        L.check(L.lib().eit_project(self.handle, _ptr(x), _ptr(out), _ptr(ws), ws.numel(), _stream()))
        return out

    def backproject(self, sino, out=None, ws=None):
        _require(sino, self.sino_shape, name="sino")
        out = torch.empty(self.x_shape, dtype=torch.float32, device=sino.device) if out is None else out
        ws = self.workspace(L.EIT_OP_BACKPROJECT) if ws is None else ws
        L.check(L.lib().eit_backproject(self.handle, _ptr(sino), _ptr(out), _ptr(ws), ws.numel(),
                                        _stream()))
        return out

    def cost_and_grad(self, x, s_exp, lam_mu: float, lam_delta: float, want_grad: bool = True,
                      ws=None):
        """(cost as a 0-d float64 device tensor, gradient of param_shape or None)."""
        _require(x, self.param_shape, name="x")
        _require(s_exp, self.data_shape, name="s_exp")
        cost = torch.empty((), dtype=torch.float64, device=x.device)
        grad = torch.empty(self.param_shape, dtype=torch.float32, device=x.device) if want_grad else None
        ws = self.workspace(L.EIT_OP_COST_GRAD) if ws is None else ws
        L.check(L.lib().eit_cost_and_grad(self.handle, _ptr(x), _ptr(s_exp), float(lam_mu),
                                          float(lam_delta), _ptr(cost), _ptr(grad), _ptr(ws),
                                          ws.numel(), _stream()))
        return cost, grad

    def single_shot(self, s_exp, out=None, ws=None):
        """Single-shot (retrieve + filtered backprojection) reconstruction of param_shape."""
        _require(s_exp, self.data_shape, name="s_exp")
        out = torch.empty(self.param_shape, dtype=torch.float32, device=s_exp.device) if out is None else out
        ws = self.workspace(L.EIT_OP_SINGLE_SHOT) if ws is None else ws
        L.check(L.lib().eit_single_shot(self.handle, _ptr(s_exp), _ptr(out), _ptr(ws), ws.numel(),
                                        _stream()))
        return out

    def reconstruct(self, s_exp, x0=None, iters: int = 50, lam: float = 1e-2, mu_scale: float = 0.05,
                    delta_scale: float = 1e-3, m: int = 10, max_ls: int = 20, tol_rel_step: float = 0.0,
                    c1: float = 1e-4, use_graph: bool = True, cost_hist: bool = False, ws=None,
                    profile: bool = False):
        """L-BFGS reconstruction; returns (x_K, report dict, cost history or None)."""
        _require(s_exp, self.data_shape, name="s_exp")
        if x0 is None:
            x = torch.zeros(self.param_shape, dtype=torch.float32, device=s_exp.device)
        else:
            _require(x0, self.param_shape, name="x0")
            x = x0.clone()
        hist = torch.zeros(iters + 1, dtype=torch.float64, device=s_exp.device) if cost_hist else None
        opts = L.Opts(iters, m, max_ls, 1 if use_graph else 0, lam, mu_scale, delta_scale,
                      tol_rel_step, c1, 1 if profile else 0, 0)
        rep = L.Report()
        # sized with a valid memory so that the library itself validates `m`
        ws = self.workspace(L.EIT_OP_RECONSTRUCT, min(max(m, 1), 20)) if ws is None else ws
        rc = L.lib().eit_reconstruct(self.handle, _ptr(s_exp), C.byref(opts), _ptr(x), _ptr(hist),
                                     C.byref(rep), _ptr(ws), ws.numel(), _stream())
        report = {f: getattr(rep, f) for f, _ in L.Report._fields_ if f not in ("phase_ms", "pad")}
        report["phase_ms"] = dict(zip(L.PHASES, list(rep.phase_ms)))
        if rc not in (L.EIT_OK, L.EIT_ERR_LINESEARCH, L.EIT_ERR_NONFINITE):
            L.check(rc)
        report["rc"] = rc
        return x, report, hist


def reconstruct_batch(plans, s_exps, x0s=None, iters: int = 50, lam: float = 1e-2,
                      mu_scale=0.05, delta_scale=1e-3, m: int = 10, max_ls: int = 20,
                      tol_rel_step: float = 0.0, c1: float = 1e-4, use_graph: bool = True,
                      profile: bool = False, ws=None):
    """Many independent slices (any mix of sizes) in one sequence of persistent launches.
    The optimiser options are shared; mu_scale/delta_scale may be scalars (all slices share
    one scaling; pass per-size scalings by grouping batches). Returns (list of x_K, reports)."""
    n = len(plans)
    if n == 0 or len(s_exps) != n:
        raise ValueError("plans and s_exps must be non-empty and of equal length")
    xs = []
    for i, (p, s) in enumerate(zip(plans, s_exps)):
        _require(s, p.data_shape, name=f"s_exps[{i}]")
        if x0s is None:
            xs.append(torch.zeros(p.param_shape, dtype=torch.float32, device=s.device))
        else:
            _require(x0s[i], p.param_shape, name=f"x0s[{i}]")
            xs.append(x0s[i].clone())
    H = (C.c_void_p * n)(*[p.handle for p in plans])
    SP = (C.c_void_p * n)(*[s.data_ptr() for s in s_exps])
    XP = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
    mm = min(max(m, 1), 20)
    nb = int(L.lib().eit_batch_workspace_bytes(n, H, mm))
    if nb == 0:
        L.check(L.EIT_ERR_INVALID_ARG)
    ws = torch.empty(nb, dtype=torch.uint8, device=s_exps[0].device) if ws is None else ws
    opts = L.Opts(iters, m, max_ls, 1 if use_graph else 0, lam, float(mu_scale), float(delta_scale),
                  tol_rel_step, c1, 1 if profile else 0, 0)
    reps = (L.Report * n)()
    rc = L.lib().eit_reconstruct_batch(n, H, SP, XP, C.byref(opts), reps, _ptr(ws), ws.numel(),
                                       _stream())
    if rc not in (L.EIT_OK, L.EIT_ERR_LINESEARCH, L.EIT_ERR_NONFINITE):
        L.check(rc)
    out = []
    for r in reps:
        d = {f: getattr(r, f) for f, _ in L.Report._fields_ if f not in ("phase_ms", "pad")}
        d["phase_ms"] = dict(zip(L.PHASES, list(r.phase_ms)))
        out.append(d)
    return xs, out


class EITCost(torch.autograd.Function):
    """S(x) of eq. 5 as an autograd node. Forward computes the cost only and saves x;
    backward recomputes the projections (checkpointed) and runs the adjoint kernel."""

    @staticmethod
    def forward(ctx, x, s_exp, plan: Plan, lam_mu: float, lam_delta: float):
        cost, _ = plan.cost_and_grad(x.detach(), s_exp, lam_mu, lam_delta, want_grad=False)
        ctx.save_for_backward(x, s_exp)
        ctx.plan = plan
        ctx.lam = (lam_mu, lam_delta)
        return cost

    @staticmethod
    def backward(ctx, g_out):
        x, s_exp = ctx.saved_tensors
        _, grad = ctx.plan.cost_and_grad(x.detach(), s_exp, *ctx.lam, want_grad=True)
        return (g_out.to(grad.dtype) * grad), None, None, None, None


def eit_cost(x, s_exp, plan: Plan, lam_mu: float, lam_delta: float):
    return EITCost.apply(x, s_exp, plan, lam_mu, lam_delta)


def frc(a, b, cutoff: float = 0.5, sigma: float = 1.0):
    """Fourier ring correlation (eq. 6) of two n x n device images on the device: (curve,
    smoothed curve, resolution in pixels, crossing ring), the curves as float64 device tensors."""
    n = int(a.shape[-1])
    _require(a, (n, n), name="a")
    _require(b, (n, n), name="b")
    nr = n // 2 + 1
    curve = torch.empty(nr, dtype=torch.float64, device=a.device)
    smooth = torch.empty(nr, dtype=torch.float64, device=a.device)
    res = torch.empty(2, dtype=torch.float64, device=a.device)
    nb = int(L.lib().eit_frc_workspace_bytes(n))
    if nb == 0:
        L.check(L.EIT_ERR_SHAPE)
    ws = torch.empty(nb, dtype=torch.uint8, device=a.device)
    L.check(L.lib().eit_frc(n, _ptr(a), _ptr(b), _ptr(curve), _ptr(smooth), _ptr(res), float(cutoff),
                            float(sigma), _ptr(ws), nb, _stream()))
    r = res.cpu()
    return curve, smooth, float(r[0]), float(r[1])


def cnr(img, c1, c2, rho: float) -> float:
    """Contrast-to-noise ratio (eq. 7) between two discs of radius rho (centred coordinates)
    of an n x n device image, computed on the device."""
    n = int(img.shape[-1])
    _require(img, (n, n), name="img")
    out = torch.empty(1, dtype=torch.float64, device=img.device)
    L.check(L.lib().eit_cnr(n, _ptr(img), float(c1[0]), float(c1[1]), float(c2[0]), float(c2[1]),
                            float(rho), _ptr(out), _stream()))
    return float(out.cpu()[0])
