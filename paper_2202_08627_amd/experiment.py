"""The paper's experiment on synthetic data, on the device (combined-results section).

Workload: the granule stack of synth.make_stack at the paper's acquisition (configs.PAPER_220:
homogeneous object, gamma = 5, one mask position on the IC slope, 400 projections over 360
degrees, 220^2 slices, lambda = 1e-2, mask drift fitted per angle), with the flat IC measured
by 1 or 20 flat scans and the ring term m_r fitted or not (Table 2's four columns).
Measures, all computed by the library's kernels:
  * iterations and time to 1e-3 (relative L2 of h) of the converged solution x*, the run from
    zero until no step passes the sufficient-decrease test (the paper's 36 / 87 steps are its
    own SciPy criterion on its data: context only);
  * CNR (eq. 7) between the three granule materials in x*, discs at granule centres;
  * FRC resolution (eq. 6) of the iterative x* and of the eq. 3 single shot, from two
    independent noise realisations of the same slice (the paper's resolution comparison).
Nothing here runs on the CPU except bookkeeping."""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import torch

from . import autotune, configs, ops, synth
from .warmstart import first_stable_crossing

MATERIAL_NAMES = ("A", "B", "C")      # the three granule materials, brightest first


def model_plan(case, fit_drift=True, fit_ring=False, use_table=True):
    """h-mode plan (two maps if the case's object is not homogeneous) with the case's flat table."""
    geo = ops.Geometry.from_case(case)
    model = ops.Model.from_case(case, fit_drift=fit_drift, fit_ring=fit_ring, use_table=use_table)
    return ops.Plan(geo, *autotune.tiling_for(geo), model=model)


def map_error(x, x_ref, n: int, n_maps: int) -> float:
    """Larger over the maps of ||x - x_ref|| / ||x_ref|| (offsets excluded)."""
    nn = n * n
    e = 0.0
    for c in range(n_maps):
        a, b = x[c * nn:(c + 1) * nn], x_ref[c * nn:(c + 1) * nn]
        e = max(e, float((a - b).norm() / b.norm()))
    return e


def solve_kw(cfg):
    return dict(lam=cfg.lam, mu_scale=cfg.mu_scale, delta_scale=cfg.delta_scale, m=10)


def converge(plan, s_exp, cfg, k_max: int = 3000):
    """x* = the run from zero until no step passes the sufficient-decrease test (or k_max)."""
    x, rep, _ = plan.reconstruct(s_exp, iters=k_max, **solve_kw(cfg))
    return x, rep


def iterations_to_tol(plan, s_exp, x_star, cfg, tol: float = 1e-3, k_max: int = 3000):
    n_maps = 1 if plan.model is not None and plan.model.hmode else 2
    x0 = torch.zeros(plan.param_shape, dtype=torch.float32, device=s_exp.device)

    def err(k):
        x, _, _ = plan.reconstruct(s_exp, iters=k, **solve_kw(cfg))
        return map_error(x, x_star, cfg.n, n_maps)
    return first_stable_crossing(err, map_error(x0, x_star, cfg.n, n_maps), tol, k_max)


def time_iterations(plan, s_exp, cfg, k: int, reps: int = 3) -> float:
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        plan.reconstruct(s_exp, iters=k, **solve_kw(cfg))
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts))


def material_discs(granules, z: float, frac: float = 0.6):
    """Per material present in slice z: (centre, radius) of a disc inside its largest
    cross-section (radius frac times the smaller semi-axis)."""
    best = {}
    for g in granules:
        t = 1.0 - ((z - g.z0) / g.c) ** 2
        if t <= 0.0:
            continue
        r = frac * min(g.a, g.b) * np.sqrt(t)
        if r >= 2.0 and r > best.get(g.material, (None, 0.0))[1]:
            best[g.material] = ((g.x0, g.y0), r)
    return best


def cnr_table(h_img, granules, z: float):
    """CNR between every pair of materials present (eq. 7), on the device."""
    discs = material_discs(granules, z)
    out = {}
    mats = sorted(discs)
    for i, a in enumerate(mats):
        for b in mats[i + 1:]:
            (ca, ra), (cb, rb) = discs[a], discs[b]
            rho = min(ra, rb)
            out[f"{MATERIAL_NAMES[a]}-{MATERIAL_NAMES[b]}"] = round(ops.cnr(h_img, ca, cb, rho), 3)
    return out


def h_image(x, n: int):
    return x[: n * n].reshape(n, n).contiguous()


def table2(cfg=configs.PAPER_220, n_slices: int = 75, z: int | None = None, k_max: int = 3000,
           log=print):
    """Table 2's four columns on slice z of the synthetic granule stack: 1 or 20 flat scans,
    ring term fitted or not (drift fitted in all)."""
    z = n_slices // 2 if z is None else z
    rows = []
    for scans in (1, 20):
        c_cfg = dataclasses.replace(cfg, flat_scans=scans)
        cases, granules = synth.make_stack(c_cfg, n_slices)
        case = cases[z]
        s_exp = torch.as_tensor(case.s_exp, device="cuda")
        for ring in (True, False):
            plan = model_plan(case, fit_drift=True, fit_ring=ring)
            x_star, rep = converge(plan, s_exp, c_cfg, k_max)
            k, e_k, _ = iterations_to_tol(plan, s_exp, x_star, c_cfg, 1e-3, rep["iters"])
            t_it = time_iterations(plan, s_exp, c_cfg, 50) / 50
            truth = torch.as_tensor(case.mu_true.astype(np.float32), device="cuda")
            err_truth = float((h_image(x_star, cfg.n) - truth).norm() / truth.norm())
            row = {"flat_scans": scans, "ring_term": ring, "x_star_iters": rep["iters"],
                   "x_star_status": rep["rc"], "iters_to_1e-3": k,
                   "ms_per_iter": round(1e3 * t_it, 4),
                   "ms_to_1e-3": round(1e3 * t_it * k, 3) if k is not None else None,
                   "rel_err_to_phantom": round(err_truth, 4),
                   "cnr": cnr_table(h_image(x_star, cfg.n), granules, z)}
            log(f"# table2 flats={scans} ring={ring}: {row}")
            rows.append(row)
            plan.close()
    return rows


def resolution_comparison(cfg=configs.PAPER_220, n_slices: int = 75, z: int | None = None,
                          k_max: int = 3000, counts: float | None = None, log=print):
    """FRC resolution (eq. 6) of the iterative solution and of the eq. 3 single shot, from two
    independent noise realisations of slice z (20 flat scans, drift fitted, no ring term),
    at the configuration's photon count or at `counts`."""
    z = n_slices // 2 if z is None else z
    if counts is not None:
        cfg = dataclasses.replace(cfg, counts=counts)
    it_imgs, ss_imgs = [], []
    for noise in (101, 202):
        cases, _ = synth.make_stack(cfg, n_slices, noise_seed=noise)
        case = cases[z]
        s_exp = torch.as_tensor(case.s_exp, device="cuda")
        plan = model_plan(case, fit_drift=True, fit_ring=False)
        x_star, _ = converge(plan, s_exp, cfg, k_max)
        it_imgs.append(h_image(x_star, cfg.n))
        ss_imgs.append(h_image(plan.single_shot(s_exp), cfg.n))
        plan.close()
    _, _, r_it, _ = ops.frc(*it_imgs)
    _, _, r_ss, _ = ops.frc(*ss_imgs)
    out = {"counts": cfg.counts, "iterative_px": round(r_it, 3), "single_shot_px": round(r_ss, 3),
           "iterative_over_single_shot": round(r_it / r_ss, 4)}
    log(f"# FRC resolution: {out}")
    return out


def stack_batch(cfg=configs.PAPER_220, n_slices: int = 75, iters: int = 36, warmup: int = 2,
                fit_ring: bool = False, log=print):
    """The whole stack through one batch call (every slice its own optimiser): wall time of
    `iters` iterations, slice-iterations per second, and the mean CNR over the slices."""
    cases, granules = synth.make_stack(cfg, n_slices)
    plans = [model_plan(c, fit_drift=True, fit_ring=fit_ring) for c in cases]
    s_dev = [torch.as_tensor(c.s_exp, device="cuda") for c in cases]
    kw = solve_kw(cfg)
    t_w = time.perf_counter()
    while True:         # untimed, repeated for 0.25 s so that the clocks have settled
        ops.reconstruct_batch(plans, s_dev, iters=warmup, **kw)
        torch.cuda.synchronize()
        if time.perf_counter() - t_w >= 0.25:
            break
    t0 = time.perf_counter()
    xs, reps = ops.reconstruct_batch(plans, s_dev, iters=iters, **kw)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    done = sum(r["iters"] for r in reps)
    return {"slices": n_slices, "iters": iters, "wall_s": round(t, 4),
            "slice_iters_per_s": round(done / t, 1),
            "stopped_early": sum(1 for r in reps if r["iters"] < iters)}, xs, cases, granules, plans
