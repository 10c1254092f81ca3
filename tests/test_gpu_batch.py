"""Batched reconstruction of independent slices of mixed sizes (3-D as a stack of 2-D
problems): every slice of a batch must equal its own single-slice run bitwise (the per-slice
arithmetic is the same and every reduction has a fixed order), one slice is checked against
the oracle, and a failing slice must not disturb the others."""
import dataclasses
import sys

import numpy as np
import pytest
import torch

from oracle import lbfgs as olbfgs
from oracle import model as omodel
from paper_2202_08627_amd import configs, synth
from helpers import geometry, rel_l2, tiny_cfg

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_08627_amd import ops as _ops
    return _ops


def _cases():
    cfgs = [tiny_cfg(n=32, n_theta=24, n_mask=5),
            tiny_cfg(n=48, n_theta=60, n_mask=8),
            dataclasses.replace(configs.SMALL_64, mu_scale=0.05),
            tiny_cfg(n=40, n_theta=33, n_mask=3, n_det=52),
            tiny_cfg(n=64, n_theta=45, n_mask=2)]
    return [synth.make_case(c, seed=i + 3) for i, c in enumerate(cfgs)]


# (projector variant, adjoint variant, adjoint angle split) per slice. First set: slices 1
# and 3 split their adjoint over 2 and 3 blocks per voxel tile. Second set: interleaved-ray
# projectors and mirror-pair adjoints (split and unsplit), the kinds the tuned size classes use.
VARIANTS = [(-1, -1, 0), (1, 1, 2), (7, 5, 1), (8, 0, 3), (0, 2, 1)]
VARIANTS_IL_MIRROR = [(22, 12, 2), (23, 8, 1), (24, 9, 3), (25, 11, 2), (18, 10, 1)]


@pytest.mark.parametrize("variants", [VARIANTS, VARIANTS_IL_MIRROR], ids=["mixed", "il-mirror"])
def test_batch_equals_single_slice_runs(ops, variants):
    print("batch vs single", variants, flush=True)
    cases = _cases()
    plans = [ops.Plan.from_case(c, proj_variant=pv, adj_variant=av, adj_splits=g)
             for c, (pv, av, g) in zip(cases, variants)]
    s = [dev(c.s_exp) for c in cases]
    kw = dict(iters=20, lam=1e-2, mu_scale=0.05, delta_scale=1e-3)
    xs, reps = ops.reconstruct_batch(plans, s, **kw)
    for i, (p, si) in enumerate(zip(plans, s)):
        x1, r1, _ = p.reconstruct(si, **kw)
        assert reps[i]["status"] == 0 and reps[i]["iters"] == 20
        assert r1["evals"] == reps[i]["evals"]
        assert torch.equal(x1, xs[i]), i


def test_batch_slice_matches_oracle(ops):
    cases = _cases()
    plans = [ops.Plan.from_case(c) for c in cases]
    xs, reps = ops.reconstruct_batch(plans, [dev(c.s_exp) for c in cases], iters=20, lam=1e-2,
                                     mu_scale=0.05, delta_scale=1e-3)
    for i in (1, 3):
        c = cases[i]
        geo = geometry(c, omodel)
        prob = omodel.ScaledProblem(c.s_exp, geo, 1e-2, 0.05, 1e-3)
        xo, st, _ = olbfgs.reconstruct(prob, np.zeros((2, c.cfg.n, c.cfg.n)), 20)
        X = xs[i].cpu().numpy().astype(np.float64)
        assert rel_l2(X[0], xo[0]) < 1e-3 and rel_l2(X[1], xo[1]) < 1e-3


def test_failing_slice_is_isolated(ops):
    cases = _cases()[:3]
    plans = [ops.Plan.from_case(c) for c in cases]
    bad = cases[1].s_exp.copy()
    bad[0, 0, 0] = np.nan
    s = [dev(cases[0].s_exp), dev(bad), dev(cases[2].s_exp)]
    xs, reps = ops.reconstruct_batch(plans, s, iters=10, lam=1e-2, mu_scale=0.05, delta_scale=1e-3)
    assert reps[0]["status"] == 0 and reps[0]["iters"] == 10
    assert reps[1]["status"] == -5 and reps[1]["iters"] == 0
    assert reps[2]["status"] == 0 and reps[2]["iters"] == 10
    x0, _, _ = plans[0].reconstruct(s[0], iters=10, lam=1e-2, mu_scale=0.05, delta_scale=1e-3)
    assert torch.equal(x0, xs[0])
