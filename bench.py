#!/usr/bin/env python3
"""Benchmark: plain iterative EI reconstruction of one 512^2 slice (720 angles over 180 deg,
512 detector pixels, 8 mask positions, Shepp-Logan-style phantom, Poisson at 1e4 counts),
FP32 projector/adjoint with FP64 cost and optimiser reductions, L-BFGS m = 10.

A step is one accepted L-BFGS iteration of the slice (its line-search evaluations
included): projector, IC model/residual, FP64 cost reduction, adjoint backprojection and the
optimiser's vector updates. `--steps K` iterations are timed from the zero start with the
inputs resident in HBM; the value is slice-iterations per second.

Printed as one JSON line. Extra keys: `roofline` for the dominant kernel (per-launch device
time from hipEvent phase timers of a profiled replay of the same workload), `cpu_baseline`
(the FP64 oracle on this host's cores, one cost+gradient evaluation as the sample)."""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "slice-iters/s (512², 720 angles) and time-to-1e-3 tol, plain vs warm start"
PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0
# algorithmic work per unit: projector fused sample (both maps) and
# adjoint voxel-angle pair (both maps)
FLOPS_PER_SAMPLE = 12.0
FLOPS_PER_VOXEL_ANGLE = 18.0


def cpu_baseline_child():
    """Time the CPU oracle on one cost+gradient evaluation of the benchmark slice."""
    import platform
    import numpy as np
    from paper_2202_08627_amd import configs, synth
    from oracle import model
    cfg = configs.SLICE_512
    c = synth.make_case(cfg)
    geo = model.Geometry(cfg.n, c.theta, cfg.n_det, c.mask_pos, c.flat_amp, c.flat_ctr,
                         c.flat_sigma, cfg.kappa)
    prob = model.ScaledProblem(c.s_exp, geo, cfg.lam, cfg.mu_scale, cfg.delta_scale)
    z = np.zeros((2, cfg.n, cfg.n))
    t0 = time.perf_counter()
    prob(z)
    t = time.perf_counter() - t0
    cpu = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    print(json.dumps({"eval_s": t, "cores": 1, "cpu": cpu}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-child", action="store_true")
    args = ap.parse_args()
    if args.cpu_baseline_child:
        cpu_baseline_child()
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build runs one slice problem per GPU and "
              "has no multi-GPU path (slices shard across GPUs without communication).",
              file=sys.stderr)
        return 2

    child = None
    if not args.no_cpu_baseline:
        env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
        # started before this process touches the GPU
        child = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child"],
                                 env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)

    import numpy as np
    import torch
    from paper_2202_08627_amd import _lib, configs, ops, synth

    cfg = configs.SLICE_512
    print(f"# building inputs {cfg.n}^2 x {cfg.n_theta} x {cfg.n_det} x M={cfg.n_mask}", file=sys.stderr, flush=True)
    case = synth.make_case(cfg)
    torch.cuda.set_device(0)
    plan = ops.Plan.from_case(case)
    s_exp = torch.as_tensor(case.s_exp, device="cuda")
    ws = plan.workspace(_lib.EIT_OP_RECONSTRUCT, 10)
    kw = dict(lam=cfg.lam, mu_scale=cfg.mu_scale, delta_scale=cfg.delta_scale, m=10, ws=ws)

    print("# warmup", file=sys.stderr, flush=True)
    plan.reconstruct(s_exp, iters=max(args.warmup, 1), **kw)
    torch.cuda.synchronize()

    print("# timed", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    x, rep, _ = plan.reconstruct(s_exp, iters=args.steps, **kw)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    if rep["rc"] != 0 or rep["iters"] != args.steps:
        print(f"reconstruction stopped early: {rep}", file=sys.stderr)
        return 1
    value = rep["iters"] / t

    print("# profiled replay", file=sys.stderr, flush=True)
    _, prep, _ = plan.reconstruct(s_exp, iters=args.steps, profile=True, **kw)
    steps = max(prep["phase_steps"], 1)
    ph = {k: v / steps for k, v in prep["phase_ms"].items()}     # ms per launch
    n, nt, nd = cfg.n, cfg.n_theta, cfg.n_det
    units = float(n) * nt * nd
    kern = {
        "project": (units * FLOPS_PER_SAMPLE, ph["project"]),
        "backproject": (float(n) * n * nt * FLOPS_PER_VOXEL_ANGLE, ph["backproject"] * steps / max(prep["iters"], 1)),
    }
    # the adjoint runs only for accepted trials: its per-launch time is its total over the
    # accepted evaluations (one launch each)
    accepted = prep["iters"] + 1
    kern["backproject"] = (float(n) * n * nt * FLOPS_PER_VOXEL_ANGLE,
                           prep["phase_ms"]["backproject"] / accepted)
    dom = max(kern, key=lambda k: kern[k][1])
    flops, ms = kern[dom]
    achieved = flops / (ms * 1e-3) / 1e12
    # HBM view of the same two kernels: algorithmic bytes = maps in + sinograms out (projector),
    # seeds in + gradient out + iterate in (adjoint)
    hbm_bytes = {"project": 4.0 * (2 * n * n + 2 * nt * nd),
                 "backproject": 4.0 * (2 * nt * nd + 4 * n * n)}
    roof = {
        "bound": "alu", "kernel": "k_project" if dom == "project" else "k_backproject",
        "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
        "launch_ms": round(ms, 5),
        "hbm_frac": round(hbm_bytes[dom] / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 5),
        "phase_ms_per_step": {k: round(v, 5) for k, v in ph.items()},
    }

    cpu = None
    if child is not None:
        out, err = child.communicate(timeout=900)
        if child.returncode == 0 and out.strip():
            cb = json.loads(out.strip().splitlines()[-1])
            evals_per_iter = rep["evals"] / max(rep["iters"], 1)
            cpu = {"value": round(1.0 / (cb["eval_s"] * evals_per_iter), 6), "unit": "slice-iters/s",
                   "cores": cb["cores"], "kind": "oracle",
                   "sample": (f"one FP64 cost+gradient evaluation of the same slice at z=0 took "
                              f"{cb['eval_s']:.1f} s on 1 thread ({cb['cpu']}); scaled by the "
                              f"{evals_per_iter:.3f} evaluations per iteration of the timed run")}
        else:
            print(f"cpu baseline failed: {err[-2000:]}", file=sys.stderr)

    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "slice-iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * t / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "slice_512: plain L-BFGS (m=10) reconstruction of a 512x512 mu/delta "
                               "slice, 720 angles over 180 deg, 512 detector pixels, 8 mask positions, "
                               "Shepp-Logan-style phantom, Poisson 1e4 counts, from zero",
                   "n": n, "n_theta": nt, "n_det": nd, "n_mask": cfg.n_mask,
                   "iterations": args.steps, "evals": rep["evals"], "final_cost": rep["cost"]},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
