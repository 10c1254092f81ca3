#!/usr/bin/env python3
"""Benchmark: plain iterative EI reconstruction of one 512^2 slice (720 angles over 180 deg,
512 detector pixels, 8 mask positions, Shepp-Logan-style phantom, Poisson at 1e4 counts),
FP32 projector/adjoint with FP64 cost and optimiser reductions, L-BFGS m = 10; and the time
to 1e-3 relative L2 of the plain solution from the zero, single-shot and learned starts.

A step is one accepted L-BFGS iteration of the slice (its line-search evaluations
included): projector, IC model/residual, FP64 cost reduction, adjoint backprojection and the
optimiser's vector updates. `--steps K` iterations are timed from the zero start with the
inputs resident in HBM; the value is slice-iterations per second.

Printed as one JSON line. Extra keys:
  roofline      the dominant kernel's algorithmic FLOP rate against the FP32 vector peak,
                from per-launch device times of hipEvents recorded on the library's stream
                around every kernel of a replay of the same K iterations; `traffic` = HBM
                bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes scaled by a
                plain copy's counts (recorded with the kernel source's hash: null once the
                source differs);
  roofline.project_plus_adjoint
                algorithmic HBM bytes of projector and adjoint (maps and sinograms in and out)
                over their summed launch time, against 8 TB/s;
  roofline.valu_issue
                the dominant kernel's VALU wavefront instructions per launch (rocprofv3
                SQ_INSTS_VALU, recorded with the source hash like `traffic`) over the chip's
                issue rate (one per SIMD per 4 cycles), against its launch time: how close the
                kernel is to the bound that binds it;
  cpu_baseline  the FP64 oracle on this host, single thread, two cost+gradient evaluations
                of the same slice, scaled to slice-iterations/s; `host`: one oracle process per
                host core (at most 16) at the same time, the host's aggregate rate;
  paper_context the paper's own CPU timings and hardware (context, not a target);
  time_to_tol   iterations and wall time to 1e-3 relative L2 (the larger over the two maps)
                of the plain run's converged solution, per start, on this slice and three held-out
                random-ellipse 512^2 slices (learned start: committed trained weights, guard on).

Other workloads (`--workload`): batch256 (256 independent slices of mixed size),
unet_train / unet_infer (the warm-start network), autograd1024 (cost and gradient through the
autograd node at 1024^2, 1800 angles, M = 12), paper220 (the paper's acquisition on a
synthetic granule slice: h-mode, one mask position, 400 angles over 360 deg, drift fitted;
slice-iters/s and Table 2's four columns: 1 or 20 flat scans, ring term fitted or not, with
iterations to 1e-3, CNR and the FRC resolution of iterative vs eq. 3 single shot), stack220
(the 220 x 220 x 75 granule stack through one batch call), sweeps (projector-only times at
Table 1's four sinogram shapes, and iteration times at N_t = N_theta = 360 / 720 / 1440).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "slice-iters/s (512², 720 angles) and time-to-1e-3 tol, plain vs warm start"
PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak (counts packed FP32)
PEAK_FP32_UNPACKED = 78.6     # 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP x 2.4 GHz, one FMA per lane
PEAK_LDS_TBS = 78.6           # 256 CUs x 128 B/clk x 2.4 GHz
PEAK_HBM_GBS = 8000.0
# Algorithmic work per unit (the useful arithmetic, not the instructions issued):
#   projector fused sample (one ray, one row, both maps): per map the interpolation
#     x_c + phi (x_(c+1) - x_c) is one multiply-add on the staged (value, difference) entry and
#     the ray sum one add: 3 FLOP per map, 6 per sample (about 1.0-1.1 GFLOP per 512^2/720
#     projection);
#   adjoint voxel-angle pair (both maps): the two triangle weights of the voxel's two detector
#     bins (one multiply-add each, 4 FLOP) and per map two multiply-adds of weight and seed
#     (8 FLOP): 12 FLOP per pair (about 2.3 GFLOP per 512^2/720 backprojection).
FLOPS_PER_SAMPLE = 6.0
FLOPS_PER_VOXEL_ANGLE = 12.0
KERNEL_SRC = os.path.join(ROOT, "paper_2202_08627_amd", "csrc", "kernels.hip")
WEIGHTS = os.path.join(ROOT, "paper_2202_08627_amd", "weights", "unet_b32_256.npz")
# HBM bytes per launch at this workload from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE,
# each scaled by the counts of a plain 256 MiB copy; valid only for the kernel source with
# this SHA-256 (first 16 hex digits). Filled from the committed traffic summary.
TRAFFIC = {
    "project": {"src": "8bae7ef64b4443db", "variant": 23, "bytes": 24.98e6},
    "backproject": {"src": "8bae7ef64b4443db", "variant": 12, "bytes": 22.92e6},
}


# VALU wavefront instructions per launch at this workload (rocprofv3 --pmc SQ_INSTS_VALU,
# medians over working launches, same source and tiles as TRAFFIC). A SIMD has 16 lanes, so a
# wavefront of 64 issues one VALU instruction per 4 cycles: the chip issues at most
# 1024 SIMDs x 2.4 GHz / 4 = 6.14e11 wavefront instructions per second, and the kernel's VALU
# issue fraction is its instruction count over that rate and its launch time.
VALU_INSTS = {
    "project": {"src": "8bae7ef64b4443db", "variant": 23, "insts": 3.2235e7},
    "backproject": {"src": "8bae7ef64b4443db", "variant": 12, "insts": 2.7450e7},
}
VALU_ISSUE_PER_S = 1024 * 2.4e9 / 4


def _src_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


# The paper's own timings (CPU only; its workload is a 220^2 slice, 400 angles over 360 deg,
# one mask position, single-map h-mode), quoted beside the measured rates as context.
PAPER_CONTEXT = {
    "hardware": "Intel Core i5 at 2.10 GHz workstation, single thread (Radon transform in "
                "Numba; SciPy L-BFGS-B)",
    "final_method": "Numba, no ring term, 20 flat scans: 36 iterations in 6.62 % of 219 s = "
                    "14.5 s for a 220^2 slice, 400 angles, M = 1 (Table 2), i.e. 2.5 slice-iters/s",
    "per_voxel_angle": "about 20 ns per voxel-angle pair per iteration (14.5 s / 36 / (220^2 x 400))",
    "extrapolated_to_this_workload": "about 0.26 slice-iters/s at 512^2 x 720 angles at the same "
                                     "rate per voxel-angle pair (not measured by the paper)",
    "simulated_total_iteration_time_s": {"N_t = N_theta = 360": 31, "720": 290, "1440": 2700},
    "full_3d_stack": "220 x 220 x 75 voxels in 23 min, single thread",
}


def cpu_cores():
    """CPU model and the cores this process may use (at most 16, the host share of one GPU)."""
    import platform
    cpu = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return cpu, max(1, min(n, 16))


# Minimum length of the untimed warm-up. The GPU raises its clocks over the first ~100 ms
# of load and lowers them again within tens of ms of idling: a timed region of a few ms that
# starts from idle runs about 13 % slower than the same work back to back (measured on the
# 512^2 slice: 0.222 ms per iteration cold, 0.196 after 200 ms of load, 0.218 after 50 ms
# idle). The warm-up therefore repeats its W steps until this much time has passed, and the
# timed K steps follow without a gap; the K steps themselves are timed as they run.
WARM_MIN_S = 0.25


def warm_up(run, min_s: float = WARM_MIN_S) -> int:
    """Run the untimed warm-up `run` (W steps) once, then again until `min_s` have passed
    since it started; returns the number of repetitions."""
    import torch
    t0 = time.perf_counter()
    n = 0
    while True:
        run()
        torch.cuda.synchronize()
        n += 1
        if time.perf_counter() - t0 >= min_s:
            return n


def cpu_baseline_child(n_evals: int):
    """Time the CPU oracle on n_evals cost+gradient evaluations of the benchmark slice."""
    import numpy as np
    from paper_2202_08627_amd import configs, synth
    from oracle import model
    cfg = configs.SLICE_512
    c = synth.make_case(cfg)
    geo = model.Geometry(cfg.n, c.theta, cfg.n_det, c.mask_pos, c.flat_amp, c.flat_ctr,
                         c.flat_sigma, cfg.kappa)
    prob = model.ScaledProblem(c.s_exp, geo, cfg.lam, cfg.mu_scale, cfg.delta_scale)
    rng = np.random.default_rng(0)
    zs = [np.zeros((2, cfg.n, cfg.n))] + [rng.uniform(0, 1, (2, cfg.n, cfg.n)) for _ in range(n_evals - 1)]
    w0 = time.time()
    t0 = time.perf_counter()
    for z in zs:
        prob(z)
    t = (time.perf_counter() - t0) / len(zs)
    cpu, _ = cpu_cores()
    print(json.dumps({"eval_s": t, "n_evals": len(zs), "cores": 1, "cpu": cpu,
                      "t_start": w0, "t_end": time.time()}), flush=True)


def cpu_host_baseline(log):
    """The oracle on the whole host share: one single-threaded process per core, each running
    one cost+gradient evaluation of the benchmark slice at the same time (slices are
    independent, so this is the host's slice throughput). Returns (evaluations/s, cores, cpu,
    wall seconds) or None."""
    cpu, p = cpu_cores()
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child",
                               "--cpu-evals", "1"], env=env, stdout=subprocess.PIPE,
                              stderr=subprocess.PIPE, text=True) for _ in range(p)]
    res = []
    for q in procs:
        out, err = q.communicate(timeout=900)
        if q.returncode != 0 or not out.strip():
            log(f"host baseline process failed: {err[-1000:]}")
            return None
        res.append(json.loads(out.strip().splitlines()[-1]))
    # the evaluations overlap; the aggregate rate is evaluations over the span they covered
    span = max(r["t_end"] for r in res) - min(r["t_start"] for r in res)
    return p / span, p, cpu, span


def time_to_tol(plan, s_exp, cfg, extra_seeds, log):
    """Warm-start comparison on this slice plus held-out random slices (medians)."""
    import numpy as np
    import torch
    from paper_2202_08627_amd import autotune, ops, warmstart as WS
    net = WS.load_net(WEIGHTS)
    recs = []
    r = WS.evaluate_case(plan, s_exp, net, cfg, tol=1e-3)
    r["slice"] = "bench slice"
    recs.append(r)
    wcfg = WS.slice_config(cfg.n, cfg.n_theta, cfg.n_mask)
    for seed in extra_seeds:
        _, s, g = WS._make_case((wcfg, seed))
        geo = WS._geometry(wcfg, g)
        p = ops.Plan(geo, *autotune.tiling_for(geo))
        r = WS.evaluate_case(p, torch.tensor(s, device="cuda"), net, wcfg, tol=1e-3)
        r["slice"] = f"random ellipses, seed {seed}"
        recs.append(r)
        p.close()
        log(f"# time-to-tol seed {seed}: " + ", ".join(f"{k} {r[k]['iters']}" for k in ("zero", "single_shot", "unet")))
    starts = ("zero", "single_shot", "unet")

    def med(key, k):
        v = [rr[k][key] for rr in recs if rr[k]["iters"] is not None]
        return float(np.median(v)) if v else None
    out = {"tol": 1e-3, "error": "max over the mu and delta maps of the relative L2 distance to "
                                 "the plain run from zero (run until no step passes)",
           "slices": [rr["slice"] for rr in recs],
           "median_iters": {k: med("iters", k) for k in starts},
           "median_ms": {k: (round(1e3 * med("t_total_s", k), 3) if med("t_total_s", k) else None) for k in starts},
           "median_err0": {k: round(float(np.median([rr[k]["err0"] for rr in recs])), 4) for k in starts},
           "guard_choices": [rr["unet"]["choice"] for rr in recs]}
    both = [rr for rr in recs if rr["zero"]["iters"] and rr["unet"]["iters"] is not None]
    out["ratio_time_warm_vs_plain"] = round(float(np.median(
        [rr["unet"]["t_total_s"] / rr["zero"]["t_total_s"] for rr in both])), 4) if both else None
    out["ratio_iters_warm_vs_plain"] = round(float(np.median(
        [rr["unet"]["iters"] / rr["zero"]["iters"] for rr in both])), 4) if both else None
    return out


def _case_for_batch(cfg):
    from paper_2202_08627_amd import synth
    c = synth.make_case(cfg)
    return c.s_exp, (c.theta, c.mask_pos, c.flat_amp, c.flat_ctr, c.flat_sigma)


def batch_main(args, log):
    """256 independent slices of mixed size ({256^2/360, 512^2/720, 768^2/1080}, M = 8, seeded
    random ellipses, seeded shuffle of the classes) in one sequence of graph-replayed launches,
    tiles per size class from the autotuner's cache. One shared (mu, delta) scaling: the
    512^2 class's."""
    from concurrent.futures import ProcessPoolExecutor
    import numpy as np
    import torch
    from paper_2202_08627_amd import autotune, configs, ops
    cfgs = configs.BATCH_256.slice_configs()
    log(f"# simulating {len(cfgs)} slices")
    with ProcessPoolExecutor(16) as ex:
        data = list(ex.map(_case_for_batch, cfgs, chunksize=2))
    torch.cuda.set_device(0)
    plans, s_dev = [], []
    for cfg, (s, g) in zip(cfgs, data):
        geo = ops.Geometry(cfg.n, cfg.n_theta, cfg.n_det, cfg.n_mask, cfg.kappa, *g)
        plans.append(ops.Plan(geo, *autotune.tiling_for(geo)))
        s_dev.append(torch.as_tensor(s, device="cuda"))
    mid = configs.SLICE_512
    kw = dict(lam=mid.lam, mu_scale=configs.mu_range_for(512), delta_scale=mid.delta_scale, m=10)
    log("# warmup")
    warm_up(lambda: ops.reconstruct_batch(plans, s_dev, iters=max(args.warmup, 1), **kw))
    log("# timed")
    t0 = time.perf_counter()
    xs, reps = ops.reconstruct_batch(plans, s_dev, iters=args.steps, **kw)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    iters = sum(r["iters"] for r in reps)
    evals = sum(r["evals"] for r in reps)
    work = sum(float(c.n) ** 2 * c.n_theta * r["iters"] for c, r in zip(cfgs, reps))
    c2 = 512.0 ** 2 * 720
    classes = {}
    for c in cfgs:
        classes[f"{c.n}x{c.n_theta}"] = classes.get(f"{c.n}x{c.n_theta}", 0) + 1
    line = {
        "metric": "slice-iters/s (256 mixed slices, one launch sequence)", "value": round(iters / t, 2),
        "unit": "slice-iters/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * t / args.steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch_256: 256 independent slices, classes " + json.dumps(classes)
                               + ", M = 8, 6 random ellipses each, L-BFGS m = 10",
                   "slice_iters": iters, "evals": evals,
                   "stopped_early": sum(1 for r in reps if r["iters"] < args.steps),
                   "voxel_angle_iters_per_s": round(work / t, 1),
                   "equivalent_512x720_iters_per_s": round(work / t / c2, 1)},
    }
    print(json.dumps(line), flush=True)
    return 0


def unet_flops(net, h, w, train):
    """Multiply-add FLOPs of one sample: forward convolutions (3x3 at their level's
    resolution, 2x2 transposed at the coarser input's), and for training the data gradients
    of every layer but the first plus the weight gradients (each the size of the forward)."""
    res = [h, h, h // 2, h // 2, h // 4, h // 4, h // 8, h // 8, h // 8, h // 4, h // 4, h // 4,
           h // 2, h // 2, h // 2, h, h, h]
    fwd = dgrad = 0.0
    for i, (l, r) in enumerate(zip(net.layers, res)):
        px = float(r) * r * w / h
        taps = {"conv3x3": 9, "upconv2x2": 4, "head1x1": 1}[l["kind"]]
        f = 2.0 * px * taps * l["cin"] * l["cout"]
        fwd += f
        if i > 0:
            dgrad += f
    return fwd * 2 + dgrad if train else fwd


def unet_main(args, log, train):
    """Warm-start network on the device: training steps (batch 16 at 256^2, the training
    resolution) or inference (one 512^2 image, the evaluation resolution)."""
    import numpy as np
    import torch
    from paper_2202_08627_amd.unet import UNet
    torch.cuda.set_device(0)
    net = UNet(32)
    net.init_he(0)
    B, H = (16, 256) if train else (1, 512)
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.rand((B, 2, H, H), device="cuda", generator=g)
    y = x + 0.1 * torch.rand((B, 2, H, H), device="cuda", generator=g)

    def step():
        if train:
            net.train_step(x, y, lr=1e-4)
        else:
            net(x)
    def warm():
        for _ in range(max(args.warmup, 1)):
            step()
    warm_up(warm)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    flops = unet_flops(net, H, H, train) * B
    achieved = flops / t / 1e12
    line = {
        "metric": "U-Net training samples/s (256^2, batch 16)" if train else "U-Net inference images/s (512^2)",
        "value": round(B / t, 2), "unit": "samples/s" if train else "images/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * t, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": ("unet_train: 4-level U-Net, 32 base channels, MSE + Adam, batch 16, 256x256"
                                if train else "unet_infer: 4-level U-Net, 32 base channels, one 512x512 image"),
                   "params": net.n_params, "gflop_per_step": round(flops / 1e9, 2)},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": round(achieved / 2500.0, 4), "traffic": None,
                     "note": "whole step (all kernels), dense BF16 MFMA peak"},
    }
    print(json.dumps(line), flush=True)
    return 0


def autograd_main(args, log):
    """Differentiation workload: S(x) and its gradient through the autograd node EITCost at
    1024^2, 1800 angles, 1024 detector pixels, M = 12 (forward: projections and IC model;
    backward: recomputed projections, IC seeds and the adjoint), plus the projector and
    adjoint launches timed alone on the same plan."""
    import torch
    from paper_2202_08627_amd import _lib, autotune, configs, ops, synth
    cfg = configs.SLICE_1024
    log(f"# building inputs {cfg.n}^2 x {cfg.n_theta} x {cfg.n_det} x M={cfg.n_mask}")
    case = synth.make_case(cfg)
    torch.cuda.set_device(0)
    geo = ops.Geometry.from_case(case)
    tiling = autotune.tiling_for(geo)
    plan = ops.Plan(geo, *tiling)
    s_exp = torch.as_tensor(case.s_exp, device="cuda")
    x = torch.as_tensor((0.9 * case.x_true).astype("float32"), device="cuda").requires_grad_()

    def step():
        x.grad = None
        ops.eit_cost(x, s_exp, plan, cfg.lam_mu, cfg.lam_delta).backward()
    def warm():
        for _ in range(max(args.warmup, 1)):
            step()
    warm_up(warm)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps

    def kernel_ms(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps
    xd = x.detach()
    sino = torch.empty(plan.sino_shape, device="cuda")
    out = torch.empty(plan.x_shape, device="cuda")
    wsp = plan.workspace(_lib.EIT_OP_PROJECT)
    wsb = plan.workspace(_lib.EIT_OP_BACKPROJECT)
    ms_p = kernel_ms(lambda: plan.project(xd, out=sino, ws=wsp))
    ms_b = kernel_ms(lambda: plan.backproject(sino, out=out, ws=wsb))
    units = float(cfg.n) * cfg.n_theta * cfg.n_det
    fp = FLOPS_PER_SAMPLE * units / (ms_p * 1e-3) / 1e12
    fb = FLOPS_PER_VOXEL_ANGLE * float(cfg.n) ** 2 * cfg.n_theta / (ms_b * 1e-3) / 1e12
    line = {
        "metric": "autograd cost+gradient evaluations/s (1024^2, 1800 angles)",
        "value": round(1.0 / t, 2), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * t, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "autograd_1024: EITCost forward + backward, 1024x1024 slice, "
                               "1800 angles over 180 deg, 1024 detector pixels, 12 mask positions",
                   "tiling": {"proj_variant": tiling[0], "adj_variant": tiling[1],
                              "adj_splits": tiling[2]}},
        "roofline": {"bound": "alu", "kernel": "k_project (call incl. launch)",
                     "achieved": round(fp, 3), "peak": 157.3, "unit": "TFLOP/s",
                     "frac": round(fp / 157.3, 4), "traffic": None,
                     "project_call_ms": round(ms_p, 4), "backproject_call_ms": round(ms_b, 4),
                     "backproject_tflops": round(fb, 3)},
    }
    print(json.dumps(line), flush=True)
    return 0


def paper220_main(args, log):
    """The paper's acquisition on slice 37 of the synthetic 220 x 220 x 75 granule stack
    (configs.PAPER_220): timed iterations with 20 flat scans, drift fitted, no ring term (the
    paper's final method), then Table 2's four columns and the FRC resolution comparison."""
    import torch
    from paper_2202_08627_amd import configs, experiment, synth
    cfg = configs.PAPER_220
    torch.cuda.set_device(0)
    cases, granules = synth.make_stack(cfg, 75)
    case = cases[37]
    s_exp = torch.as_tensor(case.s_exp, device="cuda")
    plan = experiment.model_plan(case, fit_drift=True, fit_ring=False)
    kw = experiment.solve_kw(cfg)
    warm_up(lambda: plan.reconstruct(s_exp, iters=max(args.warmup, 1), **kw))
    t0 = time.perf_counter()
    x, rep, _ = plan.reconstruct(s_exp, iters=args.steps, **kw)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    _, prep, _ = plan.reconstruct(s_exp, iters=args.steps, profile=True, **kw)
    rows = frc = None
    if not args.no_experiment:
        rows = experiment.table2(cfg, log=log)
        frc = [experiment.resolution_comparison(cfg, counts=c, log=log) for c in (cfg.counts, 1e3)]
    line = {
        "metric": "slice-iters/s (220^2, 400 angles over 360 deg, M = 1, h-mode)",
        "value": round(rep["iters"] / t, 2), "unit": "slice-iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * t / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "paper220: h-mode (mu = h, delta = 5 h), one mask position on the "
                               "IC slope, 400 angles over 360 deg, 220x220 slice of a 3-material "
                               "granule stack, tabulated flat from 20 scans, drift fitted, no ring "
                               "term, lambda = 1e-2, from zero",
                   "iterations": rep["iters"], "evals": rep["evals"],
                   "phase_ms_per_iter": {k: round(v / max(prep["iters"], 1), 5)
                                         for k, v in prep["phase_ms"].items()}},
        "table2": rows,
        "frc_resolution": frc,
        "paper_context": {"table2": "Numba columns: 1 flat scan 87 steps with m_r, 37 without; "
                                    "20 flat scans 51 with m_r, 36 without (6.62 % of 219 s = "
                                    "14.5 s on one i5 core); CNR PMMA-PP 12.6, PMMA-PS 9.6, PS-PP "
                                    "2.6 with 20 scans and no m_r",
                          "frc": "iterative resolution 30 % better than single shot"},
    }
    print(json.dumps(line), flush=True)
    return 0


def stack220_main(args, log):
    """The 220 x 220 x 75 granule stack (paper acquisition, 20 flat scans, drift fitted, no ring
    term) in one batch call of `--steps` iterations per slice."""
    import torch
    from paper_2202_08627_amd import configs, experiment
    torch.cuda.set_device(0)
    res, xs, cases, granules, plans = experiment.stack_batch(configs.PAPER_220, 75, iters=args.steps,
                                                             warmup=max(args.warmup, 1))
    line = {
        "metric": "slice-iters/s (220 x 220 x 75 stack, 400 angles over 360 deg, M = 1, h-mode)",
        "value": res["slice_iters_per_s"], "unit": "slice-iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * res["wall_s"] / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "stack220: 75 slices of the synthetic granule stack, one batch call",
                   **res},
        "paper_context": "220 x 220 x 75 voxels in 23 min on one i5 core",
    }
    print(json.dumps(line), flush=True)
    return 0


def gemm_ref_main(args, log):
    """Calibration, not part of the path: the library GEMM (torch.matmul, which calls
    hipBLASLt) at the warm-start network's layer shapes as plain BF16 GEMMs (no im2col), for
    comparison with the network's own implicit-GEMM and weight-gradient kernels (whose
    per-layer times come from the kernel trace of `--workload unet_train`)."""
    import torch
    torch.cuda.set_device(0)
    shapes = [("3x3 conv 32->32 at 256^2, batch 16 (pixels x Co x 9Ci)", 1048576, 32, 288),
              ("3x3 conv 64->32 (concatenation input) at 256^2", 1048576, 32, 576),
              ("3x3 conv 64->64 at 128^2", 262144, 64, 576),
              ("3x3 conv 128->128 at 64^2", 65536, 128, 1152),
              ("3x3 conv 256->256 at 32^2", 16384, 256, 2304),
              ("weight gradient 128->128 at 64^2 (Co x 9Ci x pixels)", 128, 1152, 65536),
              ("weight gradient 32->32 at 256^2", 32, 288, 1048576)]
    rows = []
    for name, M, N, K in shapes:
        a = torch.randn(M, K, device="cuda", dtype=torch.bfloat16)
        b = torch.randn(K, N, device="cuda", dtype=torch.bfloat16)
        warm_up(lambda: a @ b)
        reps = max(args.steps, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            a @ b
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        rows.append({"shape": name, "M": M, "N": N, "K": K, "us": round(1e6 * dt, 1),
                     "tflops": round(2.0 * M * N * K / dt / 1e12, 1)})
        log(f"# {name}: {1e6 * dt:.1f} us, {2.0 * M * N * K / dt / 1e12:.0f} TFLOP/s")
    print(json.dumps({"metric": "library BF16 GEMM at the warm-start network's layer shapes",
                      "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "dtype": "bf16",
                      "data": "synthetic", "config": {"workload": "gemm_ref", "library": "torch.matmul (hipBLASLt)"},
                      "rows": rows}), flush=True)
    return 0


def sweeps_main(args, log):
    """Secondary sweeps (context, not targets): the projector alone at Table 1's sinogram shapes
    (N_t detector pixels = grid size, N_theta angles over 180 deg, both maps), and full h-mode
    iterations (one mask position, 360 deg, drift fitted, 20-scan flat table) at
    N_t = N_theta = 360, 720, 1440."""
    import dataclasses
    import torch
    from paper_2202_08627_amd import _lib, autotune, configs, experiment, ops, synth
    torch.cuda.set_device(0)
    out = {"projector": [], "iteration": []}
    for nt_det, n_th in ((90, 45), (180, 90), (360, 180), (720, 360)):
        cfg = dataclasses.replace(configs.SMALL_64, n=nt_det, n_theta=n_th, n_det=nt_det,
                                  mu_scale=configs.mu_range_for(nt_det))
        c = synth.make_case(cfg)
        geo = ops.Geometry.from_case(c)
        plan = ops.Plan(geo, *autotune.tiling_for(geo))
        x = torch.as_tensor(c.x_true.astype("float32"), device="cuda")
        sino = torch.empty(plan.sino_shape, device="cuda")
        ws = plan.workspace(_lib.EIT_OP_PROJECT)
        for _ in range(3):
            plan.project(x, out=sino, ws=ws)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 50
        e0.record()
        for _ in range(reps):
            plan.project(x, out=sino, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out["projector"].append({"N_t": nt_det, "N_theta": n_th, "ms": round(ms, 5),
                                 "samples_per_s": round(float(nt_det) ** 2 * n_th / (ms * 1e-3), 1)})
        log(f"# projector {nt_det} x {n_th}: {ms:.4f} ms")
    for N in (360, 720, 1440):
        cfg = dataclasses.replace(configs.PAPER_220, n=N, n_det=N, n_theta=N,
                                  mu_scale=configs.mu_range_for(N))
        c = synth.make_case(cfg)
        plan = experiment.model_plan(c, fit_drift=True, fit_ring=False)
        s_exp = torch.as_tensor(c.s_exp, device="cuda")
        k = 36
        t = experiment.time_iterations(plan, s_exp, cfg, k)
        out["iteration"].append({"N": N, "iters": k, "total_ms": round(1e3 * t, 3),
                                 "ms_per_iter": round(1e3 * t / k, 4)})
        log(f"# iteration N = {N}: {1e3 * t / k:.4f} ms per iteration")
    line = {
        "metric": "secondary sweeps (projector at Table 1 shapes; h-mode iterations at N = 360/720/1440)",
        "value": None, "unit": "ms", "n_gpus": 1, "steps": None, "warmup": None,
        "higher_is_better": False, "dtype": "f32", "data": "synthetic", "sweeps": out,
        "paper_context": {"table1_relative": "lookup / Numba / OpenMP (3 threads), lookup at "
                                             "720 x 360 = 100: 90x45 0.74/0.18/0.27, 180x90 3.5/1.4/1.2, "
                                             "360x180 18/11/5.6, 720x360 100/88/27",
                          "total_iteration_time_s": {"360": 31, "720": 290, "1440": 2700}},
    }
    print(json.dumps(line), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["slice512", "batch256", "unet_train", "unet_infer",
                                           "autograd1024", "paper220", "stack220", "sweeps",
                                           "gemm_ref"],
                    default="slice512",
                    help="slice512 (default): the headline slice; batch256: 256 mixed slices; "
                         "unet_train / unet_infer: the warm-start network; autograd1024: "
                         "cost and gradient through the autograd node at 1024^2")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-warm-start", action="store_true")
    ap.add_argument("--no-host-baseline", action="store_true",
                    help="skip the oracle run on every host core")
    ap.add_argument("--no-experiment", action="store_true",
                    help="paper220: time the iterations only (no Table 2 columns, no FRC)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="finish with a plain 256 MiB device copy (HBM counter scaling)")
    ap.add_argument("--cpu-evals", type=int, default=2)
    ap.add_argument("--cpu-baseline-child", action="store_true")
    args = ap.parse_args()
    if args.cpu_baseline_child:
        cpu_baseline_child(args.cpu_evals)
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library runs one slice problem per GPU and "
              "has no multi-GPU path (slices shard across GPUs without communication).",
              file=sys.stderr)
        return 2

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.workload == "batch256":
        return batch_main(args, log)
    if args.workload in ("unet_train", "unet_infer"):
        return unet_main(args, log, args.workload == "unet_train")
    if args.workload == "autograd1024":
        return autograd_main(args, log)
    if args.workload == "paper220":
        return paper220_main(args, log)
    if args.workload == "stack220":
        return stack220_main(args, log)
    if args.workload == "sweeps":
        return sweeps_main(args, log)
    if args.workload == "gemm_ref":
        return gemm_ref_main(args, log)

    child = None
    if not args.no_cpu_baseline:
        env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
        # started before this process touches the GPU
        child = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child",
                                  "--cpu-evals", str(args.cpu_evals)],
                                 env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)

    import torch
    from paper_2202_08627_amd import _lib, autotune, configs, ops, synth

    cfg = configs.SLICE_512
    log(f"# building inputs {cfg.n}^2 x {cfg.n_theta} x {cfg.n_det} x M={cfg.n_mask}")
    case = synth.make_case(cfg)
    torch.cuda.set_device(0)
    geo = ops.Geometry.from_case(case)
    tiling = autotune.tiling_for(geo)
    plan = ops.Plan(geo, *tiling)
    info = ops.inspect(geo, *tiling)
    s_exp = torch.as_tensor(case.s_exp, device="cuda")
    ws = plan.workspace(_lib.EIT_OP_RECONSTRUCT, 10)
    kw = dict(lam=cfg.lam, mu_scale=cfg.mu_scale, delta_scale=cfg.delta_scale, m=10, ws=ws)

    log("# warmup")
    warm_up(lambda: plan.reconstruct(s_exp, iters=max(args.warmup, 1), **kw))

    log("# timed")
    t0 = time.perf_counter()
    x, rep, _ = plan.reconstruct(s_exp, iters=args.steps, **kw)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    if rep["rc"] != 0 or rep["iters"] != args.steps:
        log(f"reconstruction stopped early: {rep}")
        return 1
    value = rep["iters"] / t

    log("# replay with per-kernel hipEvents")
    _, prep, _ = plan.reconstruct(s_exp, iters=args.steps, profile=True, **kw)
    n, nt, nd = cfg.n, cfg.n_theta, cfg.n_det
    evals = max(prep["phase_steps"], 1)        # projector launches (one per evaluation)
    accepted = prep["iters"] + 1               # adjoint launches that do work (accepted trials)
    kern = {
        "project": (float(n) * nt * nd * FLOPS_PER_SAMPLE, prep["phase_ms"]["project"] / evals,
                    f"k_project<{info['proj_a']}, {info['proj_w']}, {info['proj_r']}, ...>"),
        "backproject": (float(n) * n * nt * FLOPS_PER_VOXEL_ANGLE, prep["phase_ms"]["backproject"] / accepted,
                        f"k_backproject<{info['adj_tx']}, {info['adj_ty']}, {info['adj_ac']}, ...>"),
    }
    dom = max(kern, key=lambda k: kern[k][1] * (evals if k == "project" else accepted))
    flops, ms, kname = kern[dom]
    achieved = flops / (ms * 1e-3) / 1e12
    # algorithmic HBM bytes: maps in + sinograms out (projector); seeds in + gradient out +
    # iterate in (adjoint)
    hbm_alg = {"project": 4.0 * (2 * n * n + 2 * nt * nd), "backproject": 4.0 * (2 * nt * nd + 4 * n * n)}
    tr = TRAFFIC.get(dom)
    traffic = None
    if tr and tr.get("src") == _src_hash() and tr.get("variant") == (info["proj_variant"] if dom == "project" else info["adj_variant"]):
        traffic = tr["bytes"]
    units = float(n) * nt * nd if dom == "project" else float(n) * n * nt
    lds_bytes = 16.0 * units                   # one 16-byte read of both neighbours per unit
    # HBM roofline of projector + adjoint together: maps in and sinograms out, seeds in and
    # gradient out (2.10 + 2.95 + 2.95 + 2.10 MB at 512^2 / 720), over their summed launch time
    pa_bytes = 4.0 * (2 * n * n + 2 * nt * nd) * 2
    pa_ms = kern["project"][1] + kern["backproject"][1]
    # kernels whose roofline is HBM: algorithmic bytes per launch and the achieved rate.
    #   ic: projections in, IC data in, seeds out;
    #   lb_update (accepted trials): trial point, gradient (FP64 partial planes when the adjoint
    #     is split), iterate and gradient, the m history pairs in; new pair, iterate, gradient out;
    #   lb_direction: new direction (gradient, iterate and the m pairs in; direction, trial
    #     point and its transpose out) or backtrack (direction and iterate in; trial point and
    #     its transpose out), weighted by how often each ran.
    nv = 2.0 * n * n
    mh = kw["m"]
    G = info["adj_splits"]
    b_ic = 4.0 * nt * nd * (4 + cfg.n_mask)
    b_up = nv * (4 + (8 * G if G > 1 else 4) + 8 + 8 * mh + 16)
    b_new, b_bt = nv * (4 + 4 + 8 * mh + 12), nv * (4 + 4 + 12)
    b_dir = (accepted * b_new + max(evals - accepted, 0) * b_bt) / evals
    hbm_kernels = {}
    for k, b, launches in (("ic", b_ic, evals), ("update", b_up, accepted), ("direction", b_dir, evals)):
        ms_k = prep["phase_ms"][k] / launches
        gbs = b / (ms_k * 1e-3) / 1e9
        hbm_kernels[k] = {"launch_us": round(ms_k * 1e3, 2), "alg_bytes": round(b),
                          "GB/s": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4)}
    roof = {
        "bound": "alu", "kernel": kname,
        "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
        "peak_unpacked": PEAK_FP32_UNPACKED, "frac_unpacked": round(achieved / PEAK_FP32_UNPACKED, 4),
        "lds_alg_bytes": lds_bytes, "lds_frac": round(lds_bytes / (ms * 1e-3) / 1e12 / PEAK_LDS_TBS, 4),
        "launch_us": round(ms * 1e3, 2),
        "hbm_alg_bytes": hbm_alg[dom],
        "hbm_frac": round(hbm_alg[dom] / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 5),
        "flop_per_unit": FLOPS_PER_SAMPLE if dom == "project" else FLOPS_PER_VOXEL_ANGLE,
        "units_per_launch": units,
        "project_plus_adjoint": {"alg_bytes": pa_bytes, "launch_us": round(pa_ms * 1e3, 2),
                                 "GB/s": round(pa_bytes / (pa_ms * 1e-3) / 1e9, 1),
                                 "hbm_frac": round(pa_bytes / (pa_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 5)},
        "other_kernel": {k: {"launch_us": round(v[1] * 1e3, 2),
                             "tflops": round(v[0] / (v[1] * 1e-3) / 1e12, 3)} for k, v in kern.items() if k != dom},
        "phase_ms_per_iter": {k: round(v / max(prep["iters"], 1), 5) for k, v in prep["phase_ms"].items()},
        "hbm_kernels": hbm_kernels,
        "tiling": {"proj_variant": info["proj_variant"], "adj_variant": info["adj_variant"],
                   "adj_splits": info["adj_splits"]},
    }
    vi = VALU_INSTS.get(dom)
    if vi and vi["src"] == _src_hash() and vi["variant"] == (info["proj_variant"] if dom == "project" else info["adj_variant"]):
        issue_us = vi["insts"] / VALU_ISSUE_PER_S * 1e6
        roof["valu_issue"] = {"insts_per_launch": vi["insts"], "per_unit": round(vi["insts"] * 64 / units, 2),
                              "issue_bound_us": round(issue_us, 2), "frac": round(issue_us / (ms * 1e3), 4)}

    ttt = None
    if not args.no_warm_start:
        log("# time to tolerance (zero / single-shot / learned start)")
        ttt = time_to_tol(plan, s_exp, cfg, [1_000_000, 1_000_001, 1_000_002], log)

    if args.copy_calibration:
        a = torch.ones(64 * 1024 * 1024, device="cuda")        # 256 MiB read + 256 MiB written
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    cpu = None
    if child is not None:
        out, err = child.communicate(timeout=900)
        if child.returncode == 0 and out.strip():
            cb = json.loads(out.strip().splitlines()[-1])
            evals_per_iter = rep["evals"] / max(rep["iters"], 1)
            cpu = {"value": round(1.0 / (cb["eval_s"] * evals_per_iter), 6), "unit": "slice-iters/s",
                   "cores": cb["cores"], "kind": "oracle",
                   "sample": (f"{cb['n_evals']} FP64 cost+gradient evaluations of the same slice "
                              f"(zero and a random point) at {cb['eval_s']:.1f} s each on 1 thread "
                              f"({cb['cpu']}); scaled by the {evals_per_iter:.3f} evaluations per "
                              f"iteration of the timed run")}
            if not args.no_host_baseline:
                log("# oracle on every host core")
                hb = cpu_host_baseline(log)
                if hb:
                    eps, p, cpu_model, span = hb
                    cpu["host"] = {"value": round(eps / evals_per_iter, 6), "unit": "slice-iters/s",
                                   "cores": p, "cpu": cpu_model,
                                   "sample": (f"{p} single-threaded oracle processes, one FP64 "
                                              f"cost+gradient evaluation of the slice each, "
                                              f"overlapping in {span:.1f} s; scaled by the "
                                              f"{evals_per_iter:.3f} evaluations per iteration"),
                                   "gpu_over_host": round(value / (eps / evals_per_iter), 1)}
            cpu["gpu_over_core"] = round(value / cpu["value"], 1)
        else:
            log(f"cpu baseline failed: {err[-2000:]}")

    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "slice-iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * t / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "slice_512: plain L-BFGS (m=10) reconstruction of a 512x512 mu/delta "
                               "slice, 720 angles over 180 deg, 512 detector pixels, 8 mask positions, "
                               "Shepp-Logan-style phantom, Poisson 1e4 counts, from zero",
                   "n": n, "n_theta": nt, "n_det": nd, "n_mask": cfg.n_mask,
                   "iterations": args.steps, "evals": rep["evals"],
                   "warmup_policy": (f"the {args.warmup}-iteration warm-up call repeated for at least "
                                     f"{WARM_MIN_S} s (clocks settled), then the timed call"),
                   "evals_per_s": round(rep["evals"] / t, 1), "final_cost": rep["cost"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "paper_context": PAPER_CONTEXT,
        "time_to_tol": ttt,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
