"""Slice-level entry points over the C ABI, for callers that hold a simulated or measured case
rather than a plan: project, cost_and_grad (an autograd node), reconstruct, reconstruct_batch
and warmstart. Each builds (and caches) the plan of the case's geometry with the autotuned
tiles and forwards to `ops`; every step runs in the library's kernels.

A case is anything with `cfg` (a `configs.SliceConfig`: sizes, kappa, lam, mu_scale,
delta_scale, iters), `s_exp` (host or device, [n_theta][n_mask][n_det]) and the geometry arrays
`theta`, `mask_pos`, `flat_amp`, `flat_ctr`, `flat_sigma`, as `synth.make_case` returns.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import autotune, ops

_plans: dict = {}


@dataclass
class Opts:
    """Optimiser options of `reconstruct` (defaults from the case's config when None)."""
    iters: int | None = None
    m: int = 10
    max_ls: int = 20
    lam: float | None = None
    tol_rel_step: float = 0.0


def clear_plans() -> None:
    """Releases the cached plans (their device tables) of every geometry seen so far."""
    for p in _plans.values():
        p.close()
    _plans.clear()


def plan_for(case) -> ops.Plan:
    """The case's plan with the autotuned tiles; one per geometry, kept for reuse until
    `clear_plans`."""
    c = case.cfg
    key = (c.n, c.n_theta, c.n_det, c.n_mask, float(c.kappa),
           np.asarray(case.theta, np.float64).tobytes(), np.asarray(case.mask_pos, np.float64).tobytes(),
           np.asarray(case.flat_amp, np.float64).tobytes(), np.asarray(case.flat_ctr, np.float64).tobytes(),
           np.asarray(case.flat_sigma, np.float64).tobytes())
    p = _plans.get(key)
    if p is None:
        geo = ops.Geometry.from_case(case)
        p = ops.Plan(geo, *autotune.tiling_for(geo))
        _plans[key] = p
    return p


def _data(case) -> torch.Tensor:
    s = case.s_exp
    if isinstance(s, torch.Tensor) and s.is_cuda:
        return s
    return torch.as_tensor(np.ascontiguousarray(s, dtype=np.float32), device="cuda")


def project(x: torch.Tensor, case) -> torch.Tensor:
    """R x for both maps: [2][n][n] -> [2][n_theta][n_det] (eq. 1)."""
    return plan_for(case).project(x)


def cost_and_grad(x: torch.Tensor, case, lam_mu: float | None = None, lam_delta: float | None = None):
    """S(x) of eq. 5 as a differentiable scalar (FP64, on the device); its backward pass gives
    the gradient through the adjoint kernel."""
    c = case.cfg
    return ops.eit_cost(x, _data(case), plan_for(case), c.lam_mu if lam_mu is None else lam_mu,
                        c.lam_delta if lam_delta is None else lam_delta)


def _recon_kw(case, opts: Opts | None):
    c = case.cfg
    o = opts or Opts()
    return dict(iters=c.iters if o.iters is None else o.iters, m=o.m, max_ls=o.max_ls,
                lam=c.lam if o.lam is None else o.lam, mu_scale=c.mu_scale,
                delta_scale=c.delta_scale, tol_rel_step=o.tol_rel_step)


def reconstruct(case, opts: Opts | None = None, x0: torch.Tensor | None = None):
    """The plain method (L-BFGS on the scaled unknowns) from zero or from x0; returns
    (x_K [2][n][n], report dict)."""
    x, rep, _ = plan_for(case).reconstruct(_data(case), x0=x0, **_recon_kw(case, opts))
    return x, rep


def reconstruct_batch(cases, opts: Opts | None = None):
    """Independent slices of any sizes in one launch sequence. The optimiser options and the
    (mu, delta) scaling are shared: the first case's config supplies them."""
    kw = _recon_kw(cases[0], opts)
    return ops.reconstruct_batch([plan_for(c) for c in cases], [_data(c) for c in cases], **kw)


def warmstart(case, net, opts: Opts | None = None):
    """Learned warm start: x0 = the network applied to the single-shot reconstruction, kept
    only if its cost is not above the single shot's and zero's (else the cheaper of those),
    then the plain method from x0. Returns (x_K, report, choice)."""
    from . import warmstart as ws
    plan = plan_for(case)
    s = _data(case)
    c = case.cfg
    x0, choice, _ = ws.warm_start(plan, s, net, c, lam=None if opts is None else opts.lam)
    x, rep = reconstruct(case, opts, x0=x0)
    return x, rep, choice
