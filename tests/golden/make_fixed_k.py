"""Write the FP64 oracle's fixed-K reconstructions used as stored expected values by the GPU
fixed-K parity tests.

Every value written here comes from `oracle/` (the FP64 NumPy L-BFGS over the FP64 model)
on inputs from the seeded simulator `paper_2202_08627_amd.synth`; nothing comes from the HIP
path. Each fixture holds x_K (stored FP32: the parity bound is 1e-3 relative L2, FP32
storage adds ~1e-7), the per-iteration trace (accepted cost, step length, trials) and the
run's settings.

    python tests/golden/make_fixed_k.py slice512       # 512^2 / 720 / M = 8, K = 100
    python tests/golden/make_fixed_k.py batch_classes  # one slice per batch size class, K = 5

The optimiser reading (theory section: L-BFGS through SciPy, settings unstated) is the
oracle's: memory 10, first trial 1/||g||, Armijo c1 = 1e-4 with halving, at most 20
trials, pair stored when s^T y > 1e-10 ||s|| ||y||.
"""
from __future__ import annotations

import json
import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
os.environ.setdefault("MKL_NUM_THREADS", "1")

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_2202_08627_amd import configs, synth  # noqa: E402
from oracle import lbfgs as olbfgs  # noqa: E402
from oracle import model as omodel  # noqa: E402

# Shared option set of a mixed batch: one (lam, mu_s, delta_s) for every slice, taken from
# the 512^2 class (the batch entry point takes one option set for all slices).
BATCH_LAM = 1e-2
BATCH_MU_SCALE = configs.mu_range_for(512)
BATCH_DELTA_SCALE = 1e-3


def batch_class_slices(per_class: int = 1):
    """Indices and configs of the first `per_class` slices of each size class in the seeded
    256-slice mixed batch."""
    cfgs = configs.BATCH_256.slice_configs()
    out = {}
    for s, c in enumerate(cfgs):
        key = (c.n, c.n_theta)
        out.setdefault(key, [])
        if len(out[key]) < per_class:
            out[key].append((s, c))
    return [item for k in sorted(out) for item in out[k]]


def run_oracle(case, lam, mu_scale, delta_scale, iters, m=10):
    cfg = case.cfg
    geo = omodel.Geometry(cfg.n, case.theta, cfg.n_det, case.mask_pos, case.flat_amp,
                          case.flat_ctr, case.flat_sigma, cfg.kappa)
    prob = omodel.ScaledProblem(case.s_exp, geo, lam, mu_scale, delta_scale)
    t0 = time.time()
    x, st, tr = olbfgs.reconstruct(prob, np.zeros((2, cfg.n, cfg.n)), iters, m=m)
    return x, st, tr, time.time() - t0


def save(path, x, st, tr, meta):
    np.savez_compressed(path, x=x.astype(np.float32), cost=np.asarray(tr.cost),
                        alpha=np.asarray(tr.alpha), trials=np.asarray(tr.trials, dtype=np.int32),
                        status=np.int32(tr.status), evals=np.int32(st.evals),
                        meta=json.dumps(meta))
    print(f"wrote {path}: {meta}", flush=True)


def make_slice512(iters=100):
    cfg = configs.SLICE_512
    case = synth.make_case(cfg)
    x, st, tr, dt = run_oracle(case, cfg.lam, cfg.mu_scale, cfg.delta_scale, iters)
    meta = dict(workload="512x512, 720 angles, 512 detector pixels, M=8, Shepp-Logan-style "
                "phantom, seed 0, Poisson 1e4, from zero", n=cfg.n, n_theta=cfg.n_theta,
                n_mask=cfg.n_mask, seed=cfg.seed, iters=iters, m=10, lam=cfg.lam,
                mu_scale=cfg.mu_scale, delta_scale=cfg.delta_scale, oracle_s=round(dt, 1),
                command="python tests/golden/make_fixed_k.py slice512")
    save(os.path.join(HERE, "slice512_k100.npz"), x, st, tr, meta)


def make_batch_classes(iters=5):
    for s, cfg in batch_class_slices(1):
        case = synth.make_case(cfg)
        x, st, tr, dt = run_oracle(case, BATCH_LAM, BATCH_MU_SCALE, BATCH_DELTA_SCALE, iters)
        meta = dict(workload=f"batch slice {s}: {cfg.n}x{cfg.n}, {cfg.n_theta} angles, M={cfg.n_mask}, "
                    f"random ellipses seed {cfg.seed}, from zero", slice_index=s, n=cfg.n,
                    n_theta=cfg.n_theta, n_mask=cfg.n_mask, seed=cfg.seed, iters=iters, m=10,
                    lam=BATCH_LAM, mu_scale=BATCH_MU_SCALE, delta_scale=BATCH_DELTA_SCALE,
                    oracle_s=round(dt, 1), command="python tests/golden/make_fixed_k.py batch_classes")
        save(os.path.join(HERE, f"batch_slice{s}_{cfg.n}_k{iters}.npz"), x, st, tr, meta)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "slice512"
    {"slice512": make_slice512, "batch_classes": make_batch_classes}[what]()
