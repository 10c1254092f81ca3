"""Write the FP64 oracle's fixed-K reconstructions used as stored expected values by the GPU
fixed-K parity tests.

Every value written here comes from `oracle/` (the FP64 NumPy L-BFGS over the FP64 model)
on inputs from the seeded simulator `paper_2202_08627_amd.synth`; nothing comes from the HIP
path. Each fixture holds x_K (stored FP32: the parity bound is 1e-3 relative L2, FP32
storage adds ~1e-7), the per-iteration trace (accepted cost, step length, trials) and the
run's settings.

    python tests/golden/make_fixed_k.py slice512 [K ...]  # 512^2 / 720 / M = 8, x_K (default K = 100)
    python tests/golden/make_fixed_k.py batch_classes  # one slice per batch size class, K = 5
    python tests/golden/make_fixed_k.py paper220       # the paper's acquisition (eq. 4 model), K = 50

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
from oracle import full_model as ofull  # noqa: E402
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


def run_oracle(case, lam, mu_scale, delta_scale, iters, m=10, snapshots=(), on_snapshot=None):
    """The oracle's run from zero; x at each iteration count in `snapshots` is passed to
    on_snapshot(k, x, state) on the way."""
    cfg = case.cfg
    geo = omodel.Geometry(cfg.n, case.theta, cfg.n_det, case.mask_pos, case.flat_amp,
                          case.flat_ctr, case.flat_sigma, cfg.kappa)
    prob = omodel.ScaledProblem(case.s_exp, geo, lam, mu_scale, delta_scale)
    t0 = time.time()

    def cb(st):
        if st.k in snapshots and on_snapshot is not None:
            on_snapshot(st.k, prob.to_x(st.z), st)
    z, st, tr = olbfgs.minimize(prob, prob.to_z(np.zeros((2, cfg.n, cfg.n))), iters, m=m,
                                callback=cb)
    return prob.to_x(z), st, tr, time.time() - t0


def save(path, x, st, tr, meta):
    np.savez_compressed(path, x=x.astype(np.float32), cost=np.asarray(tr.cost),
                        alpha=np.asarray(tr.alpha), trials=np.asarray(tr.trials, dtype=np.int32),
                        status=np.int32(tr.status), evals=np.int32(st.evals),
                        meta=json.dumps(meta))
    print(f"wrote {path}: {meta}", flush=True)


def make_slice512(iters=100, snapshots=(), out_dir=HERE):
    """x_iters of the benchmark slice (slice512_k<iters>.npz), and x_k for every k in
    snapshots on the way (slice512_k<k>.npz)."""
    cfg = configs.SLICE_512
    case = synth.make_case(cfg)
    t0 = time.time()

    def meta_for(k, dt):
        return dict(workload="512x512, 720 angles, 512 detector pixels, M=8, Shepp-Logan-style "
                    "phantom, seed 0, Poisson 1e4, from zero", n=cfg.n, n_theta=cfg.n_theta,
                    n_mask=cfg.n_mask, seed=cfg.seed, iters=k, m=10, lam=cfg.lam,
                    mu_scale=cfg.mu_scale, delta_scale=cfg.delta_scale, oracle_s=round(dt, 1),
                    command=f"python tests/golden/make_fixed_k.py slice512 {k}")

    class _Tr:      # trace prefix of a snapshot
        def __init__(self, tr, k):
            self.cost, self.alpha, self.trials, self.status = tr.cost[:k], tr.alpha[:k], tr.trials[:k], 0

    trace = olbfgs.Trace()

    def snap(k, x, st):
        save(os.path.join(out_dir, f"slice512_k{k}.npz"), x, st, _Tr(trace, k), meta_for(k, time.time() - t0))
    geo = omodel.Geometry(cfg.n, case.theta, cfg.n_det, case.mask_pos, case.flat_amp,
                          case.flat_ctr, case.flat_sigma, cfg.kappa)
    prob = omodel.ScaledProblem(case.s_exp, geo, cfg.lam, cfg.mu_scale, cfg.delta_scale)

    def cb(st):
        if st.k in snapshots:
            snap(st.k, prob.to_x(st.z), st)
    z, st, tr = olbfgs.minimize(prob, prob.to_z(np.zeros((2, cfg.n, cfg.n))), iters, m=10,
                                trace=trace, callback=cb)
    save(os.path.join(out_dir, f"slice512_k{iters}.npz"), prob.to_x(z), st, tr,
         meta_for(iters, time.time() - t0))


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


def make_paper220(iters=50, z=37):
    """Slice z of the 220 x 220 x 75 granule stack at the paper's acquisition: h-mode
    (gamma = 5), one mask position, 400 angles over 360 deg, 20-scan flat table, drift m_o
    fitted, no ring term; x_K is the parameter vector [h (n^2), m_o (n_theta)]."""
    cfg = configs.PAPER_220
    cases, _ = synth.make_stack(cfg, 75)
    c = cases[z]
    st = ofull.Setup(cfg.n, c.theta, cfg.n_det, c.mask_pos, c.flat_amp, c.flat_ctr, c.flat_sigma,
                     cfg.kappa, hmode=True, gamma=cfg.gamma_h, fit_mo=True, fit_mr=False,
                     flat_table=c.flat_table, table_u0=c.table_u0, table_du=c.table_du)
    prob = ofull.ScaledProblem(st, c.s_exp, cfg.lam, cfg.mu_scale, 1.0)
    t0 = time.time()
    zk, stt, tr = olbfgs.minimize(prob, np.zeros(st.n_params), iters, m=10)
    meta = dict(workload=f"paper acquisition, granule stack slice {z}: 220x220, 400 angles over "
                "360 deg, M=1, h-mode gamma=5, 20-scan flat table, drift fitted, from zero",
                n=cfg.n, n_theta=cfg.n_theta, n_mask=cfg.n_mask, slice=z, iters=iters, m=10,
                lam=cfg.lam, mu_scale=cfg.mu_scale, offset_scale=1.0, oracle_s=round(time.time() - t0, 1),
                command="python tests/golden/make_fixed_k.py paper220")
    save(os.path.join(HERE, f"paper220_k{iters}.npz"), prob.to_p(zk), stt, tr, meta)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "slice512"
    if what == "slice512":
        ks = [int(a) for a in sys.argv[2:]] or [100]
        make_slice512(max(ks), snapshots=tuple(k for k in ks if k != max(ks)))
    elif what == "paper220":
        make_paper220()
    else:
        make_batch_classes()
