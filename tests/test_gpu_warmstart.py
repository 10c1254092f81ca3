"""Learned warm start on the device: the committed trained network against the method
without it (single-shot start, zero start) on held-out 512x720 slices, and the guard's
fallback when the network's estimate is worse. The trained weights themselves have no
oracle (parity unpinned): they are judged by iterations to 1e-3 relative L2 of the plain
solution."""
import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2202_08627_amd", "weights", "unet_b32_256.npz")


def _case(seed):
    from paper_2202_08627_amd import warmstart as WS, ops
    cfg = WS.slice_config(512, 720)
    _, s, g = WS._make_case((cfg, seed))
    return cfg, ops.Plan(WS._geometry(cfg, g)), torch.tensor(s, device="cuda")


@pytest.mark.parametrize("seed", [1_000_040, 1_000_041])
def test_trained_network_beats_starts_without_it(seed):
    print(f"[warm start] seed {seed}", flush=True)
    from paper_2202_08627_amd import warmstart as WS
    net = WS.load_net(WEIGHTS)
    cfg, plan, s = _case(seed)
    r = WS.evaluate_case(plan, s, net, cfg, tol=1e-3, reps=1)
    print({k: (r[k]["iters"], round(r[k]["err0"], 3), r[k]["choice"]) for k in ("zero", "single_shot", "unet")})
    assert r["unet"]["choice"] == "unet"
    # the network's start is much closer to the plain solution than either start without it
    assert r["unet"]["err0"] < 0.5 * min(r["single_shot"]["err0"], r["zero"]["err0"])
    for k in ("zero", "single_shot", "unet"):
        assert r[k]["iters"] is not None and r[k]["err"] <= 1e-3
    assert r["unet"]["iters"] < r["zero"]["iters"]
    assert r["unet"]["iters"] <= r["single_shot"]["iters"]


def test_guard_falls_back_when_network_is_worse():
    print("[warm start] guard fallback", flush=True)
    from paper_2202_08627_amd import warmstart as WS
    net = WS.load_net(WEIGHTS)
    for l in net.layers:                      # a head blown up 100x: estimate far off
        if l["kind"] == "head1x1":
            net.params[l["w_off"]:l["b_off"]] *= 100.0
    cfg, plan, s = _case(1_000_042)
    x0, choice, costs = WS.warm_start(plan, s, net, cfg)
    print(costs, choice)
    assert costs["unet"] > costs["single_shot"]
    assert choice == "single_shot"
    assert torch.equal(x0, plan.single_shot(s))
