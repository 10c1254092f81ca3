"""Tile-shape autotuner for the projector and adjoint kernels.

For a slice geometry (grid size, angles, detector pixels) every compiled variant that fits
the geometry is timed through the C ABI (eit_project / eit_backproject, HIP events around
repeated launches on the current stream) and the fastest pair is stored in a JSON cache keyed
by the size class. The adjoint is timed for every variant and angle split (blocks per voxel
tile); the fastest few are then timed inside the optimiser step, where a split adjoint's
partial sums are added by the update pass instead of a separate one, and the choice is the
fastest per evaluation there. `tiling_for(geo)` returns the cached (projector variant,
adjoint variant, adjoint split), or (-1, -1, 0) = library defaults.

With --hmode the optimiser step is that of the paper's acquisition at this size (h-mode,
single-map kernels, one mask position, drift fitted, measured flat table): every split of
the fastest adjoint variants is a step candidate, then the fastest projector variants are
timed in the step with the chosen adjoint, and the entry records the mode. A size class
whose slices are h-mode (the paper-shaped 220 x 400 x 220) is tuned that way.

    python -m paper_2202_08627_amd.autotune --n 512 --n-theta 720 [--cache tiles.json] [--angle-span 2] [--hmode]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os

import numpy as np

from . import _lib as L
from . import ops, synth

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiles.json")
SPLITS = (1, 2, 4, 8)
SOLVER_CANDIDATES = 4
PROJ_STEP_CANDIDATES = 6      # h-mode: projector variants timed in the step
SOLVER_ITERS = 40
SOLVER_REPS = 3
STEP_TIE = 0.01


def size_key(geo) -> str:
    return f"{geo.n}x{geo.n_theta}x{geo.n_det}"


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _fits(geo, pv: int, av: int, ag: int) -> bool:
    """Whether the library accepts these tiles for this geometry (host-only check)."""
    try:
        ops.inspect(geo, pv, av, ag)
        return True
    except L.EitError:
        return False


def tiling_for(geo, path: str = DEFAULT_CACHE):
    """Cached tiles of the geometry's size class, checked against this geometry's angle list.
    The cache is keyed by size only; a variant tuned on angles over 180 degrees can be too
    narrow for other angle lists (over 360 degrees, irregular), whose projector windows are
    wider. Then the next fastest timed variant that fits is taken (the cache keeps every
    variant's time), and the library's default if none does."""
    ent = load_cache(path).get(size_key(geo))
    if not ent:
        return -1, -1, 0
    pv, av, ag = int(ent["proj_variant"]), int(ent["adj_variant"]), int(ent.get("adj_splits", 1))
    if _fits(geo, pv, av, ag):
        return pv, av, ag
    projs = [pv] + [int(k) for k, _ in sorted(ent.get("proj_us", {}).items(), key=lambda kv: kv[1])]
    adjs = [(av, ag)] + [tuple(int(v) for v in k.split("/"))
                         for k, _ in sorted(ent.get("adj_us", {}).items(), key=lambda kv: kv[1])]
    p_ok = next((p for p in projs if _fits(geo, p, -1, 0)), -1)
    a_ok = next((a for a in adjs if _fits(geo, -1, *a)), (-1, 0))
    if _fits(geo, p_ok, *a_ok):
        return (p_ok, *a_ok)
    return -1, -1, 0


def _time(fn, reps: int):
    import torch
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def pick_adjoint(step: dict, kernel: dict, tie: float = STEP_TIE):
    """Fastest adjoint (variant, split) inside the optimiser step; candidates within `tie`
    (relative) of the fastest step are ranked by their own kernel time, which is measured with
    less noise than the step."""
    best = min(step.values())
    close = [k for k, v in step.items() if v <= best * (1.0 + tie)]
    return min(close, key=lambda k: kernel[k])


def _hmode_case(geo):
    """The paper's acquisition (configs.PAPER_220's settings) at this geometry's size."""
    from . import configs
    cfg = dataclasses.replace(configs.PAPER_220, n=geo.n, n_theta=geo.n_theta, n_det=geo.n_det,
                              mu_scale=configs.PAPER_220.mu_scale * configs.PAPER_220.n / geo.n)
    return cfg, synth.make_case(cfg, seed=12345)


def tune(geo, reps: int = 20, verbose: bool = True, hmode: bool = False) -> dict:
    """Times every applicable variant; returns the record stored in the cache."""
    import torch
    rng = np.random.default_rng(0)
    x = torch.as_tensor(rng.standard_normal((2, geo.n, geo.n)).astype(np.float32), device="cuda")
    y = torch.as_tensor(rng.standard_normal((2, geo.n_theta, geo.n_det)).astype(np.float32),
                        device="cuda")
    res = {"proj": {}, "adj": {}}
    for v, shape in enumerate(ops.variants(0)):
        try:
            plan = ops.Plan(geo, proj_variant=v, adj_variant=0)
        except L.EitError:
            continue                      # window wider than this variant's pitch
        out = torch.empty(plan.sino_shape, device="cuda")
        ws = plan.workspace(L.EIT_OP_PROJECT)
        ms = _time(lambda: plan.project(x, out=out, ws=ws), reps)
        res["proj"][v] = ms
        if verbose:
            print(f"  project variant {v} {shape}: {ms * 1e3:.1f} us", flush=True)
        plan.close()
    for v, shape in enumerate(ops.variants(1)):
        units = geo.n_theta // 2 + 1 if shape[4] else geo.n_theta   # angle pairs if mirrored
        nchunks = -(-units // shape[2])
        for g in SPLITS:
            if g > 1 and g > nchunks // 2:
                continue
            try:
                plan = ops.Plan(geo, adj_variant=v, adj_splits=g)
            except L.EitError:
                break
            out = torch.empty(plan.x_shape, device="cuda")
            ws = plan.workspace(L.EIT_OP_BACKPROJECT)
            ms = _time(lambda: plan.backproject(y, out=out, ws=ws), reps)
            res["adj"][(v, g)] = ms
            if verbose:
                print(f"  backproject variant {v} {shape} split {g}: {ms * 1e3:.1f} us", flush=True)
            plan.close()
    pv = min(res["proj"], key=res["proj"].get)
    # optimiser-step timing of the best adjoint candidates on a simulated slice of this size
    # (a run that keeps iterating; flat data would stop within a few steps): random ellipses
    # with the plain model, or the paper's acquisition with the h-mode model
    model = None
    if hmode:
        cfg, case = _hmode_case(geo)
        model = ops.Model.from_case(case, fit_drift=True, fit_ring=False)
        kw = dict(lam=cfg.lam, mu_scale=cfg.mu_scale, delta_scale=cfg.delta_scale)
        top = sorted(res["adj"], key=res["adj"].get)[:SOLVER_CANDIDATES]
        cands = sorted({(v, g) for v, _ in top for g in SPLITS if _fits(geo, pv, v, g)})
    else:
        from . import warmstart
        cfg = warmstart.slice_config(geo.n, geo.n_theta, geo.n_mask)
        cfg = dataclasses.replace(cfg, n_det=geo.n_det)
        case = synth.make_case(cfg, seed=12345)
        kw = dict(lam=cfg.lam, mu_scale=cfg.mu_scale, delta_scale=cfg.delta_scale)
        cands = sorted(res["adj"], key=res["adj"].get)[:SOLVER_CANDIDATES]
    sgeo = ops.Geometry.from_case(case)
    s_exp = torch.as_tensor(case.s_exp, device="cuda")
    def time_step(pv_, av_, ag_):
        plan = ops.Plan(sgeo, proj_variant=pv_, adj_variant=av_, adj_splits=ag_, model=model)
        ws = plan.workspace(L.EIT_OP_RECONSTRUCT, 10)
        plan.reconstruct(s_exp, iters=2, ws=ws, **kw)
        best = float("inf")
        for _ in range(SOLVER_REPS):
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            _, rep, _ = plan.reconstruct(s_exp, iters=SOLVER_ITERS, ws=ws, **kw)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) / max(rep["evals"], 1))
        plan.close()
        return best

    step = {}
    for key in cands:
        step[key] = time_step(pv, *key)
        if verbose:
            print(f"  optimiser step with adjoint {key[0]} split {key[1]}: {step[key] * 1e3:.1f} us"
                  " per evaluation", flush=True)
    pstep = {}
    if hmode:       # the two-map kernel times say nothing about the single-map kernels
        av, ag = min(step, key=step.get)
        for v in sorted(res["proj"], key=res["proj"].get)[:PROJ_STEP_CANDIDATES]:
            pstep[v] = step[(av, ag)] if v == pv else time_step(v, av, ag)
            if verbose:
                print(f"  optimiser step with projector {v}: {pstep[v] * 1e3:.1f} us per evaluation",
                      flush=True)
        pv = min(pstep, key=pstep.get)
    else:
        av, ag = pick_adjoint(step, res["adj"])
    rec = {"proj_variant": pv, "adj_variant": av, "adj_splits": ag,
           "proj_us": {str(k): round(v * 1e3, 2) for k, v in res["proj"].items()},
           "adj_us": {f"{k[0]}/{k[1]}": round(v * 1e3, 2) for k, v in res["adj"].items()},
           "step_us_per_eval": {f"{k[0]}/{k[1]}": round(v * 1e3, 2) for k, v in step.items()}}
    if hmode:
        rec["step_model"] = "h-mode (paper's acquisition, drift fitted, measured flat table)"
        rec["proj_step_us_per_eval"] = {str(k): round(v * 1e3, 2) for k, v in pstep.items()}
    return rec


def tune_and_store(geo, path: str = DEFAULT_CACHE, reps: int = 20, verbose: bool = True,
                   hmode: bool = False) -> dict:
    rec = tune(geo, reps, verbose, hmode)
    cache = load_cache(path)
    cache[size_key(geo)] = rec
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    return rec


def geometry_for(n: int, n_theta: int, n_det: int | None = None, n_mask: int = 8,
                 angle_span: float = 1.0):
    nd = n if n_det is None else n_det
    return ops.Geometry(n, n_theta, nd, n_mask, 10.0, synth.angles(n_theta, angle_span),
                        synth.mask_positions(n_mask), np.ones(nd), np.zeros(nd), np.full(nd, 0.6))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", default=[512])
    ap.add_argument("--n-theta", type=int, nargs="+", default=[720])
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--angle-span", type=float, default=1.0,
                    help="angles a * span * pi / n_theta (2 for 360 degrees)")
    ap.add_argument("--hmode", action="store_true",
                    help="time the adjoint candidates in the h-mode optimiser step")
    a = ap.parse_args()
    for n, nt in zip(a.n, a.n_theta):
        geo = geometry_for(n, nt, angle_span=a.angle_span)
        print(f"tuning {size_key(geo)}" + (" (h-mode step)" if a.hmode else ""), flush=True)
        rec = tune_and_store(geo, a.cache, a.reps, hmode=a.hmode)
        print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
