"""Case-level entry points (`eitomo`): each forwards to the plan API with the autotuned tiles and
must give the plan API's results bitwise, and the oracle's within the usual tolerances."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import lbfgs as olbfgs
from oracle import model as omodel
from oracle import radon as oradon
from paper_2202_08627_amd import configs, synth
from helpers import geometry, rel_l2, tiny_cfg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_08627_amd import eitomo
    return eitomo


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def test_project_and_cost_and_grad(E):
    cfg = configs.SMALL_64
    c = synth.make_case(cfg)
    rng = np.random.default_rng(21)
    x = (c.x_true + 0.2 * np.stack([cfg.mu_scale * rng.standard_normal((cfg.n, cfg.n)),
                                    cfg.delta_scale * rng.standard_normal((cfg.n, cfg.n))]))
    x = x.astype(np.float32).astype(np.float64)
    P = E.project(dev(x), c)
    assert torch.equal(P, E.plan_for(c).project(dev(x)))
    ref = np.stack([oradon.project(x[q], c.theta, cfg.n_det) for q in range(2)])
    assert rel_l2(P.cpu().numpy().astype(np.float64), ref) < 1e-5
    xt = dev(x).requires_grad_(True)
    S = E.cost_and_grad(xt, c)
    S.backward()
    S_o, gm, gd = omodel.cost_and_grad(x[0], x[1], c.s_exp, geometry(c, omodel), cfg.lam_mu, cfg.lam_delta)
    assert float(S.detach()) == pytest.approx(S_o, rel=1e-5)
    G = xt.grad.cpu().numpy().astype(np.float64)
    assert rel_l2(G[0], gm) < 1e-4 and rel_l2(G[1], gd) < 1e-4


def test_reconstruct_and_batch(E):
    cfg = configs.SMALL_64
    c = synth.make_case(cfg)
    x, rep = E.reconstruct(c)
    assert rep["rc"] == 0 and rep["iters"] == cfg.iters
    x2, _, _ = E.plan_for(c).reconstruct(dev(c.s_exp), iters=cfg.iters, lam=cfg.lam,
                                         mu_scale=cfg.mu_scale, delta_scale=cfg.delta_scale)
    assert torch.equal(x, x2)
    prob = omodel.ScaledProblem(c.s_exp, geometry(c, omodel), cfg.lam, cfg.mu_scale, cfg.delta_scale)
    xo, _, _ = olbfgs.reconstruct(prob, np.zeros((2, cfg.n, cfg.n)), cfg.iters)
    X = x.cpu().numpy().astype(np.float64)
    assert rel_l2(X[0], xo[0]) < 1e-3 and rel_l2(X[1], xo[1]) < 1e-3
    # a batch of two geometries gives each slice's own run
    c2 = synth.make_case(dataclasses.replace(tiny_cfg(n=40, n_theta=33, n_mask=3, n_det=52),
                                             mu_scale=cfg.mu_scale), seed=4)
    assert (c2.cfg.mu_scale, c2.cfg.delta_scale) == (cfg.mu_scale, cfg.delta_scale)
    o = E.Opts(iters=12, lam=cfg.lam)
    xs, reps = E.reconstruct_batch([c, c2], o)
    for xi, ci in zip(xs, (c, c2)):
        xs1, _ = E.reconstruct(ci, o)
        assert torch.equal(xi, xs1)


def test_warmstart_without_network(E):
    """With no network the guard chooses between zero and the single shot; the run continues
    from that start exactly as a plain run from it."""
    cfg = configs.SMALL_64
    c = synth.make_case(cfg)
    o = E.Opts(iters=10)
    x, rep, choice = E.warmstart(c, None, o)
    assert choice in ("zero", "single_shot")
    x0 = torch.zeros_like(x) if choice == "zero" else E.plan_for(c).single_shot(dev(c.s_exp))
    x1, _ = E.reconstruct(c, o, x0=x0)
    assert torch.equal(x, x1)
    E.clear_plans()
    assert not E._plans
