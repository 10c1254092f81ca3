"""Learned warm start for the iterative reconstruction (not part of the paper's method).

Pipeline, all compute on the device through the library:
  1. training data: seeded random-ellipse slices (host simulation of the EI data, eq. 2),
     inputs = single-shot reconstructions (eit_single_shot), targets = plain iterative
     solutions after a fixed number of L-BFGS iterations from zero (eit_reconstruct_batch),
     both in scaled units z = [mu / mu_scale ; delta / delta_scale];
  2. training of the U-Net (eit_unet_train_step, MSE, Adam);
  3. warm start with a guard: the network's estimate is used only if its cost (eq. 5) is no
     larger than the single-shot start's and the zero start's, else the better of those;
  4. time to tolerance: iterations and wall time until the relative L2 distance (the larger
     over the two maps) to the plain run's converged solution falls to a tolerance.

The plain iteration from zero stays the reference solution and the fallback.
"""
from __future__ import annotations

import os
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import torch

from . import autotune, configs, ops, synth
from .unet import UNet


def slice_config(n: int, n_theta: int, n_mask: int = 8, seed: int = 0,
                 axis_max: float = 0.4) -> configs.SliceConfig:
    """Random-ellipse slice with per-pixel sigma jitter, the warm-start workload."""
    return configs.SliceConfig(n=n, n_theta=n_theta, n_det=n, n_mask=n_mask, phantom="random",
                               n_ellipses=6, axis_max=axis_max, sigma=0.6, sigma_jitter=0.05,
                               mu_scale=configs.mu_range_for(n), seed=seed)


def _make_case(args):
    cfg, seed = args
    c = synth.make_case(cfg, seed=seed)
    return seed, c.s_exp, (c.theta, c.mask_pos, c.flat_amp, c.flat_ctr, c.flat_sigma)


def generate_cases(cfg: configs.SliceConfig, seeds, workers: int = 8):
    """Yield (seed, s_exp, geometry arrays) in seed order; host simulation in a process pool."""
    seeds = list(seeds)
    if workers <= 1:
        for s in seeds:
            yield _make_case((cfg, s))
        return
    with ProcessPoolExecutor(workers) as ex:
        yield from ex.map(_make_case, [(cfg, s) for s in seeds], chunksize=4)


def _geometry(cfg, arrays):
    theta, m, amp, ctr, sig = arrays
    return ops.Geometry(cfg.n, cfg.n_theta, cfg.n_det, cfg.n_mask, cfg.kappa, theta, m, amp, ctr, sig)


def scales(cfg) -> torch.Tensor:
    return torch.tensor([cfg.mu_scale, cfg.delta_scale], dtype=torch.float32).view(2, 1, 1)


def build_training_set(cfg: configs.SliceConfig, seeds, target_iters: int = 300, chunk: int = 256,
                       m: int = 10, workers: int = 8, tiling=(-1, -1, 0), log=print):
    """(inputs, targets) as device tensors [N][2][n][n] in scaled units, and statistics."""
    seeds = list(seeds)
    dev = torch.device("cuda")
    X = torch.empty((len(seeds), 2, cfg.n, cfg.n), dtype=torch.float32, device=dev)
    Y = torch.empty_like(X)
    sc = scales(cfg).to(dev)
    gen = generate_cases(cfg, seeds, workers)
    t0 = time.time()
    # "stalled": runs that ended before target_iters because no step passed the sufficient-
    # decrease test any more (converged to the precision of the FP32 gradient)
    stats = {"slices": 0, "iters": 0, "evals": 0, "gpu_s": 0.0, "stalled": 0, "nonfinite": 0}
    for c0 in range(0, len(seeds), chunk):
        part = [next(gen) for _ in range(min(chunk, len(seeds) - c0))]
        plans = [ops.Plan(_geometry(cfg, g), *tiling) for _, _, g in part]
        s_dev = [torch.tensor(s, device=dev) for _, s, _ in part]
        torch.cuda.synchronize()
        tg = time.time()
        for i, (p, s) in enumerate(zip(plans, s_dev)):
            X[c0 + i] = p.single_shot(s) / sc
        xs, reps = ops.reconstruct_batch(plans, s_dev, iters=target_iters, lam=cfg.lam,
                                         mu_scale=cfg.mu_scale, delta_scale=cfg.delta_scale, m=m)
        for i, x in enumerate(xs):
            Y[c0 + i] = x / sc
        torch.cuda.synchronize()
        stats["gpu_s"] += time.time() - tg
        stats["slices"] += len(part)
        stats["iters"] += sum(r["iters"] for r in reps)
        stats["evals"] += sum(r["evals"] for r in reps)
        stats["stalled"] += sum(1 for r in reps if r["status"] == -6)
        stats["nonfinite"] += sum(1 for r in reps if r["status"] == -5)
        for p in plans:
            p.close()
        log(f"[data] {stats['slices']}/{len(seeds)} slices, {time.time() - t0:.1f}s "
            f"(device {stats['gpu_s']:.1f}s, {stats['iters'] / max(stats['gpu_s'], 1e-9):.0f} slice-iters/s)")
    return X, Y, stats


def train(net: UNet, X: torch.Tensor, Y: torch.Tensor, epochs: int, batch: int = 16,
          lr: float = 1e-3, lr_min: float = 1e-5, seed: int = 0, log=print, val=None):
    """Adam on the MSE with a cosine learning-rate schedule; returns per-epoch mean losses."""
    n = X.shape[0]
    g = torch.Generator().manual_seed(seed)
    steps = epochs * (n // batch)
    hist = []
    k = 0
    t0 = time.time()
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g)
        tot = torch.zeros((), dtype=torch.float64, device=X.device)
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch].to(X.device)
            xb, yb = X.index_select(0, idx).contiguous(), Y.index_select(0, idx).contiguous()
            a = lr_min + 0.5 * (lr - lr_min) * (1 + np.cos(np.pi * k / max(steps, 1)))
            tot += net.train_step(xb, yb, lr=a)
            k += 1
        mean = float(tot.cpu()) / (n // batch)
        hist.append(mean)
        msg = f"[train] epoch {ep + 1}/{epochs} loss {mean:.4e} ({time.time() - t0:.1f}s)"
        if val is not None:
            msg += f" val {evaluate_loss(net, *val):.4e}"
        log(msg)
    return hist


def evaluate_loss(net: UNet, X: torch.Tensor, Y: torch.Tensor, batch: int = 16) -> float:
    tot, cnt = 0.0, 0
    for b0 in range(0, X.shape[0], batch):
        xb = X[b0:b0 + batch].contiguous()
        out = net(xb)
        tot += float(((out - Y[b0:b0 + batch]) ** 2).sum().cpu())
        cnt += out.numel()
    return tot / cnt


def save_weights(net: UNet, path: str, meta: dict | None = None):
    np.savez_compressed(path, params=net.params.cpu().numpy(), base=net.base,
                        meta=np.array(repr(meta or {})))


def load_net(path: str) -> UNet:
    d = np.load(path, allow_pickle=False)
    return UNet(int(d["base"]), d["params"])


# --------------------------------------------------------------------------- warm start
def warm_start(plan: ops.Plan, s_exp: torch.Tensor, net: UNet | None, cfg, lam: float | None = None):
    """Start point for the plain iteration and the name of the start chosen by the guard.
    Returns (x0 raw units [2][n][n], choice, costs dict)."""
    lam = cfg.lam if lam is None else lam
    lam_mu, lam_de = lam / cfg.mu_scale ** 2, lam / cfg.delta_scale ** 2
    sc = scales(cfg).to(s_exp.device)
    x_ss = plan.single_shot(s_exp)
    cands = {"zero": torch.zeros_like(x_ss), "single_shot": x_ss}
    if net is not None:
        z = (x_ss / sc).unsqueeze(0).contiguous()
        cands["unet"] = (net(z)[0] * sc).contiguous()
    # the candidates' costs stay on the device until one transfer reads them all
    dev_costs = [plan.cost_and_grad(v, s_exp, lam_mu, lam_de, want_grad=False)[0].reshape(1)
                 for v in cands.values()]
    costs = dict(zip(cands.keys(), torch.cat(dev_costs).cpu().tolist()))
    choice = guard_choice(costs)
    return cands[choice], choice, costs


def guard_choice(costs: dict) -> str:
    """The network's start is taken only if its cost is finite and no larger than both the
    single-shot start's and the zero start's; otherwise the cheaper of those two (zero on a
    non-finite single-shot cost)."""
    ss = costs.get("single_shot", float("inf"))
    best = "single_shot" if np.isfinite(ss) and ss <= costs["zero"] else "zero"
    u = costs.get("unet")
    if u is not None and np.isfinite(u) and u <= costs["zero"] and (not np.isfinite(ss) or u <= ss):
        return "unet"
    return best


def rel_err(x: torch.Tensor, x_ref: torch.Tensor, cfg=None) -> float:
    """Tolerance measure: the larger over the two maps of ||x - x_ref|| / ||x_ref||."""
    d = (x - x_ref).flatten(1).norm(dim=1) / x_ref.flatten(1).norm(dim=1)
    return float(d.max().cpu())


STABILITY_PROBES = (1, 5, 20, 50)


def first_stable_crossing(err, e0: float, tol: float, k_max: int, probes=STABILITY_PROBES):
    """Smallest K with err(K) <= tol after which err stays <= tol at the probe points
    K + p (p in probes, up to k_max) and at k_max. L-BFGS gives no guarantee that the error
    falls monotonically, so a bisection alone can land on a crossing that is undone later:
    when a probe fails, the search restarts above the failing probe.
    Returns (K or None if err(k_max) > tol, err(K), checks) where checks holds err(K - 1)
    (> tol, or None for K = 0) and the probe errors."""
    cache = {0: e0}

    def E(k):
        if k not in cache:
            cache[k] = err(k)
        return cache[k]

    if E(k_max) > tol:
        return None, cache[k_max], {"k_max": k_max, "err_k_max": cache[k_max]}
    lo = 0
    while True:
        if E(lo) <= tol:
            k = lo
        else:
            a, b = lo, k_max          # E(a) > tol, E(b) <= tol
            while b - a > 1:
                mid = (a + b) // 2
                if E(mid) <= tol:
                    b = mid
                else:
                    a = mid
            k = b
        later = sorted({min(k + p, k_max) for p in probes} | {k_max})
        bad = [q for q in later if E(q) > tol]
        if not bad:
            checks = {"err_k_minus_1": E(k - 1) if k > 0 else None,
                      "probes": {int(q): E(q) for q in later}}
            return k, E(k), checks
        lo = bad[-1]


def iterations_to_tolerance(plan: ops.Plan, s_exp, x0, x_star, cfg, tol: float = 1e-3,
                            k_max: int = 2000, m: int = 10):
    """Iterations from x0 until rel_err(x_K, x_star) <= tol for good (first_stable_crossing).
    The device iteration is deterministic, so a run of K iterations is the first K iterations
    of a longer run. Returns (K or None if not reached by k_max, error at K, checks)."""
    def err(k):
        x, rep, _ = plan.reconstruct(s_exp, x0=x0, iters=k, lam=cfg.lam, mu_scale=cfg.mu_scale,
                                     delta_scale=cfg.delta_scale, m=m)
        return rel_err(x, x_star, cfg)
    return first_stable_crossing(err, rel_err(x0, x_star, cfg), tol, k_max)


def time_iterations(plan: ops.Plan, s_exp, x0, k: int, cfg, m: int = 10, reps: int = 3) -> float:
    """Median wall time (s) of k plain iterations from x0 (inputs resident on the device)."""
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        plan.reconstruct(s_exp, x0=x0, iters=k, lam=cfg.lam, mu_scale=cfg.mu_scale,
                         delta_scale=cfg.delta_scale, m=m)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts))


def time_warm_start(plan: ops.Plan, s_exp, net, cfg, reps: int = 3) -> float:
    """Median wall time (s) of the warm start itself: single shot, inference, guard costs."""
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        warm_start(plan, s_exp, net, cfg)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts))


# --------------------------------------------------------------------------- evaluation
def evaluate_case(plan: ops.Plan, s_exp, net, cfg, tol: float = 1e-3, k_ref: int = 2000,
                  k_max: int = 1000, m: int = 10, reps: int = 3):
    """Iterations and wall time to rel_err <= tol for the zero, single-shot and (guarded)
    network starts. The reference x* is the plain run from zero after k_ref iterations (it
    stops earlier once no step passes the sufficient-decrease test). Times are medians of
    reps runs with the data resident on the device; a warm start's time includes computing
    the start (single shot, inference and the guard's cost evaluations)."""
    x_star, rep, _ = plan.reconstruct(s_exp, iters=k_ref, lam=cfg.lam, mu_scale=cfg.mu_scale,
                                      delta_scale=cfg.delta_scale, m=m)
    out = {"ref_iters": rep["iters"], "ref_status": rep["rc"], "ref_cost": rep["cost"]}
    x_ss = plan.single_shot(s_exp)
    starts = {"zero": (torch.zeros_like(x_ss), 0.0, "zero"), "single_shot": (x_ss, None, "single_shot")}
    if net is not None:
        x0, choice, costs = warm_start(plan, s_exp, net, cfg)
        starts["unet"] = (x0, None, choice)
        out["guard_costs"] = costs
    for name, (x0, t_start, choice) in starts.items():
        k, e, checks = iterations_to_tolerance(plan, s_exp, x0, x_star, cfg, tol=tol, k_max=k_max, m=m)
        if t_start is None:
            if name == "single_shot":
                ts = []
                for _ in range(reps):
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    plan.single_shot(s_exp)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t)
                t_start = float(np.median(ts))
            else:
                t_start = time_warm_start(plan, s_exp, net, cfg, reps)
        t_iter = time_iterations(plan, s_exp, x0, k, cfg, m, reps) if k else 0.0
        out[name] = {"iters": k, "err": e, "err0": rel_err(x0, x_star, cfg), "choice": choice,
                     "checks": checks,
                     "t_start_s": t_start, "t_iter_s": t_iter,
                     "t_total_s": (t_start + t_iter) if k is not None else None}
    return out


def summarize(records):
    """Medians over slices of iterations and time per start, and warm/plain ratios."""
    s = {"n": len(records)}
    for name in ("zero", "single_shot", "unet"):
        rs = [r[name] for r in records if name in r]
        if not rs:
            continue
        ok = [r for r in rs if r["iters"] is not None]
        s[name] = {"reached": len(ok), "median_iters": float(np.median([r["iters"] for r in ok])) if ok else None,
                   "median_time_s": float(np.median([r["t_total_s"] for r in ok])) if ok else None,
                   "median_err0": float(np.median([r["err0"] for r in rs])),
                   "choices": {c: sum(1 for r in rs if r["choice"] == c) for c in {r["choice"] for r in rs}}}
    if "unet" in s and s["unet"]["median_time_s"] and s["zero"]["median_time_s"]:
        both = [r for r in records if r["zero"]["iters"] is not None and r.get("unet", {}).get("iters") is not None]
        s["ratio_time_unet_vs_zero"] = float(np.median([r["unet"]["t_total_s"] / r["zero"]["t_total_s"] for r in both]))
        s["ratio_iters_unet_vs_zero"] = float(np.median([r["unet"]["iters"] / max(r["zero"]["iters"], 1) for r in both]))
    return s


def _main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="train / evaluate the learned warm start")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--n-train", type=int, default=configs.WARMSTART.n_train)
    t.add_argument("--n-val", type=int, default=configs.WARMSTART.n_val)
    t.add_argument("--target-iters", type=int, default=configs.WARMSTART.target_iters)
    t.add_argument("--epochs", type=int, default=configs.WARMSTART.epochs)
    t.add_argument("--batch", type=int, default=16)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--workers", type=int, default=16)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--axis-max", type=float, default=0.4,
                   help="largest ellipse semi-axis as a fraction of n/2 (0.8 at 256^2 spans the "
                        "pixel sizes of 0.4 at 512^2)")
    t.add_argument("--train-n", type=int, default=configs.WARMSTART.train_n,
                   help="grid size of the training slices")
    t.add_argument("--train-theta", type=int, default=configs.WARMSTART.train_theta,
                   help="angles of the training slices")
    t.add_argument("--seed0", type=int, default=0, help="first phantom seed of the training set")
    t.add_argument("--init", default=None, help="start from these weights instead of He init")
    t.add_argument("--out", required=True, help="weights .npz (a .json log is written beside it)")
    e = sub.add_parser("eval")
    e.add_argument("--weights", default=None)
    e.add_argument("--n-eval", type=int, default=configs.WARMSTART.n_eval)
    e.add_argument("--tol", type=float, default=configs.WARMSTART.tol)
    e.add_argument("--workers", type=int, default=16)
    e.add_argument("--with-shepp", action="store_true", help="also the Shepp-Logan-style 512^2 slice")
    e.add_argument("--out", required=True)
    a = ap.parse_args()
    W = configs.WARMSTART

    def log(msg):
        print(msg, flush=True)

    if a.cmd == "train":
        cfg = slice_config(a.train_n, a.train_theta, W.n_mask, axis_max=a.axis_max)
        t0 = time.time()
        X, Y, st = build_training_set(cfg, range(a.seed0, a.seed0 + a.n_train + a.n_val),
                                      a.target_iters, workers=a.workers, log=log)
        t_data = time.time() - t0
        if a.init:
            net = load_net(a.init)
        else:
            net = UNet(W.base_channels)
            net.init_he(a.seed)
        val = (X[a.n_train:], Y[a.n_train:])
        log(f"[train] identity-map val loss {float(((val[0] - val[1]) ** 2).mean().cpu()):.4e}")
        t1 = time.time()
        hist = train(net, X[:a.n_train], Y[:a.n_train], a.epochs, a.batch, a.lr, seed=a.seed, log=log,
                     val=val)
        t_train = time.time() - t1
        meta = {"n_train": a.n_train, "n_val": a.n_val, "target_iters": a.target_iters,
                "seed0": a.seed0, "init": os.path.basename(a.init) if a.init else None,
                "axis_max": a.axis_max,
                "epochs": a.epochs, "batch": a.batch, "lr": a.lr, "seed": a.seed,
                "train_shape": [a.train_n, a.train_theta, W.n_mask], "data_stats": st,
                "data_s": t_data, "train_s": t_train, "loss_hist": hist,
                "val_loss": evaluate_loss(net, *val),
                "val_identity_loss": float(((val[0] - val[1]) ** 2).mean().cpu())}
        save_weights(net, a.out, meta)
        with open(os.path.splitext(a.out)[0] + ".json", "w") as f:
            json.dump(meta, f, indent=1)
        log(json.dumps({k: v for k, v in meta.items() if k != "loss_hist"}))
    else:
        net = load_net(a.weights) if a.weights else None
        cfg = slice_config(W.eval_n, W.eval_theta, W.n_mask)
        seeds = [W.eval_seed0 + i for i in range(a.n_eval)]
        cases = [(cfg, s, sx, g) for s, sx, g in generate_cases(cfg, seeds, a.workers)]
        if a.with_shepp:
            c = synth.make_case(configs.SLICE_512)
            cases.append((configs.SLICE_512, -1, c.s_exp,
                          (c.theta, c.mask_pos, c.flat_amp, c.flat_ctr, c.flat_sigma)))
        recs = []
        for cf, seed, sx, g in cases:
            geo = _geometry(cf, g)
            plan = ops.Plan(geo, *autotune.tiling_for(geo))
            r = evaluate_case(plan, torch.tensor(sx, device="cuda"), net, cf, tol=a.tol)
            r["seed"] = seed
            recs.append(r)
            plan.close()
            log(f"[eval] seed {seed}: " + ", ".join(
                f"{k} {r[k]['iters']} it {r[k]['t_total_s'] or float('nan'):.4f}s (e0 {r[k]['err0']:.3f}, {r[k]['choice']})"
                for k in ("zero", "single_shot", "unet") if k in r))
        summ = summarize(recs)
        with open(a.out, "w") as f:
            json.dump({"summary": summ, "records": recs, "tol": a.tol,
                       "shape": [W.eval_n, W.eval_theta, W.n_mask]}, f, indent=1)
        log(json.dumps(summ))


if __name__ == "__main__":
    _main()
