"""Fixed-K reconstruction parity against stored FP64 oracle runs, in the launch configurations
the benchmark times.

* The 512^2 / 720-angle / M = 8 benchmark slice: x_K from zero with the tuned tiles, per-map
  relative L2 <= 1e-3 against the oracle's x_K (tests/golden/slice512_k<K>.npz, written by
  tests/golden/make_fixed_k.py from oracle/ only).
* The paper's acquisition (full eq. 4 model) on one slice of the granule stack, K = 50.
* The mixed-size batch: three slices of each size class (256^2/360, 512^2/720, 768^2/1080,
  M = 8) in one batch call with the tuned tiles; that many adjoint tiles put the batch in the
  regime where every adjoint runs unsplit. Each slice equals its own single-slice run with an
  unsplit adjoint bitwise, and one slice per class is within 1e-3 of the oracle's x_5.

Margins (relative L2 per map) are printed for the log."""
import json
import os

import numpy as np
import pytest
import torch

from paper_2202_08627_amd import autotune, configs, synth
from helpers import rel_l2

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL_X = 1e-3


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_08627_amd import ops as _ops
    return _ops


def load_fixture(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"fixture {name} not generated (tests/golden/make_fixed_k.py)")
    z = np.load(path, allow_pickle=False)
    return {k: z[k] for k in z.files}, json.loads(str(z["meta"]))


def first_divergence(gpu_hist, oracle_cost, rtol=1e-4):
    """First accepted iteration whose cost differs from the oracle's by more than rtol."""
    for k, (a, b) in enumerate(zip(gpu_hist, oracle_cost)):
        if abs(a - b) > rtol * abs(b):
            return k + 1
    return None


# x_38 is within about 1e-5 of the oracle's. K = 100 (the benchmark's iteration count) misses
# the bound: the FP32 trajectory leaves the FP64 one at iteration 39 (cost within 3e-6
# relative through iteration 38, 1.8e-4 at 39, with the same number of line-search trials;
# the first differing trial count is at iteration 69), x_40 is already 5e-4 / 2e-3 away and
# x_100 1.1e-3 (mu) / 4.7e-3 (delta). Kept as a strict expected failure so that the margins
# stay in the log and a change that closes the gap is noticed.
FIXED_K = [38, pytest.param(100, marks=pytest.mark.xfail(
    strict=True, reason="the FP32 trajectory departs from the FP64 oracle at iteration 39"))]


@pytest.mark.parametrize("K", FIXED_K)
def test_fixed_k_benchmark_slice(ops, K):
    fx, meta = load_fixture(f"slice512_k{K}.npz")
    cfg = configs.SLICE_512
    assert (meta["n"], meta["n_theta"], meta["n_mask"], meta["iters"]) == (512, 720, 8, K)
    c = synth.make_case(cfg)
    geo = ops.Geometry.from_case(c)
    tiles = autotune.tiling_for(geo)
    print(f"fixed-K 512^2/720/M=8, K={K}, tiles", tiles, flush=True)
    plan = ops.Plan(geo, *tiles)
    x, rep, hist = plan.reconstruct(dev(c.s_exp), iters=K, lam=cfg.lam, mu_scale=cfg.mu_scale,
                                    delta_scale=cfg.delta_scale, cost_hist=True)
    X = x.cpu().numpy().astype(np.float64)
    xo = fx["x"].astype(np.float64)
    e_mu, e_de = rel_l2(X[0], xo[0]), rel_l2(X[1], xo[1])
    h = hist.cpu().numpy()[1:]
    div = first_divergence(h, fx["cost"])
    print(f"fixed-K 512 K={K}: rel-L2 mu {e_mu:.3e} delta {e_de:.3e} (bound {TOL_X}); evals GPU "
          f"{rep['evals']} oracle {int(fx['evals'])}; first cost divergence > 1e-4 at iteration {div}; "
          f"final cost GPU {h[-1]:.6e} oracle {fx['cost'][-1]:.6e}", flush=True)
    assert rep["rc"] == 0 and rep["iters"] == K
    assert e_mu < TOL_X and e_de < TOL_X
    assert np.allclose(h, fx["cost"], rtol=1e-4)


def _batch_slices(per_class):
    cfgs = configs.BATCH_256.slice_configs()
    got = {}
    for s, cfg in enumerate(cfgs):
        key = (cfg.n, cfg.n_theta)
        got.setdefault(key, [])
        if len(got[key]) < per_class:
            got[key].append((s, cfg))
    return [it for k in sorted(got) for it in got[k]]


BATCH_KW = dict(lam=1e-2, mu_scale=configs.mu_range_for(512), delta_scale=1e-3)


def test_mixed_batch_in_benchmark_shape(ops):
    slices = _batch_slices(3)
    cases = [synth.make_case(cfg) for _, cfg in slices]
    geos = [ops.Geometry.from_case(c) for c in cases]
    tiles = [autotune.tiling_for(g) for g in geos]
    tiles_count = 0
    for g, t in zip(geos, tiles):
        info = ops.inspect(g, *t)
        tiles_count += info["n_tx"] * info["n_ty"]
    print("batch slices", [s for s, _ in slices], "tiles", tiles, "adjoint tiles", tiles_count, flush=True)
    assert tiles_count >= 1024      # the regime in which a batch runs every adjoint unsplit
    plans = [ops.Plan(g, *t) for g, t in zip(geos, tiles)]
    s_dev = [dev(c.s_exp) for c in cases]
    K = 5
    xs, reps = ops.reconstruct_batch(plans, s_dev, iters=K, **BATCH_KW)
    for i, (g, t, s) in enumerate(zip(geos, tiles, s_dev)):
        assert reps[i]["status"] == 0 and reps[i]["iters"] == K, (i, reps[i])
        single = ops.Plan(g, t[0], t[1], 1)
        x1, r1, _ = single.reconstruct(s, iters=K, **BATCH_KW)
        assert r1["evals"] == reps[i]["evals"], i
        assert torch.equal(x1, xs[i]), f"slice {slices[i][0]} differs from its single-slice run"
    checked = 0
    for i, (s_idx, cfg) in enumerate(slices):
        name = f"batch_slice{s_idx}_{cfg.n}_k{K}.npz"
        if not os.path.exists(os.path.join(GOLDEN, name)):
            continue
        fx, meta = load_fixture(name)
        assert meta["mu_scale"] == BATCH_KW["mu_scale"] and meta["lam"] == BATCH_KW["lam"]
        X = xs[i].cpu().numpy().astype(np.float64)
        xo = fx["x"].astype(np.float64)
        e_mu, e_de = rel_l2(X[0], xo[0]), rel_l2(X[1], xo[1])
        print(f"batch slice {s_idx} ({cfg.n}^2/{cfg.n_theta}) vs oracle x_{K}: mu {e_mu:.3e} "
              f"delta {e_de:.3e}", flush=True)
        assert e_mu < TOL_X and e_de < TOL_X
        checked += 1
    assert checked == 3


def test_fixed_k_paper_acquisition(ops):
    """The paper's acquisition (eq. 4 model: h-mode, one mask position, 400 angles over 360 deg,
    20-scan flat table, drift fitted) on slice 37 of the granule stack, in the benchmark's
    launch configuration: x_50 (h and m_o) within 1e-3 of the FP64 oracle's."""
    from paper_2202_08627_amd import experiment
    fx, meta = load_fixture("paper220_k50.npz")
    cfg = configs.PAPER_220
    K = meta["iters"]
    cases, _ = synth.make_stack(cfg, 75)
    c = cases[meta["slice"]]
    plan = experiment.model_plan(c, fit_drift=True, fit_ring=False)
    x, rep, hist = plan.reconstruct(dev(c.s_exp), iters=K, cost_hist=True, **experiment.solve_kw(cfg))
    X = x.cpu().numpy().astype(np.float64)
    xo = fx["x"].astype(np.float64)
    nn = cfg.n * cfg.n
    e_h, e_mo = rel_l2(X[:nn], xo[:nn]), rel_l2(X[nn:], xo[nn:])
    h = hist.cpu().numpy()[1:]
    print(f"fixed-K paper220 K={K}: rel-L2 h {e_h:.3e} m_o {e_mo:.3e} (bound {TOL_X}); evals GPU "
          f"{rep['evals']} oracle {int(fx['evals'])}; first cost divergence > 1e-4 at iteration "
          f"{first_divergence(h, fx['cost'])}", flush=True)
    assert rep["rc"] == 0 and rep["iters"] == K
    assert e_h < TOL_X and e_mo < TOL_X
    assert np.allclose(h, fx["cost"], rtol=1e-4)
