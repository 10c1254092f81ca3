"""The no-allocation cost/gradient entry point (static device scratch array) against the
workspace entry point it varies: identical cost and gradient on two calls in a row, the
second on a smaller problem, plus the size limit's error. Calls go through the C ABI."""
import numpy as np
import pytest
import torch

from paper_2202_08627_amd import _lib as L
from paper_2202_08627_amd import configs, ops, synth

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda:0")


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


def _both(plan, x, s, lam_mu, lam_de):
    """(cost, grad) from eit_cost_and_grad with a torch workspace, then from the no-alloc
    entry point; both through the C ABI."""
    lib = L.lib()
    ws = plan.workspace(L.EIT_OP_COST_GRAD)
    c_ws = torch.empty((), dtype=torch.float64, device="cuda:0")
    g_ws = torch.empty(plan.param_shape, dtype=torch.float32, device="cuda:0")
    L.check(lib.eit_cost_and_grad(plan.handle, _ptr(x), _ptr(s), lam_mu, lam_de, _ptr(c_ws),
                                  _ptr(g_ws), _ptr(ws), ws.numel(), _stream()))
    c_na = torch.empty((), dtype=torch.float64, device="cuda:0")
    g_na = torch.full(plan.param_shape, float("nan"), dtype=torch.float32, device="cuda:0")
    L.check(lib.eit_cost_and_grad_noalloc(plan.handle, _ptr(x), _ptr(s), lam_mu, lam_de,
                                          _ptr(c_na), _ptr(g_na), _stream()))
    torch.cuda.synchronize()
    return float(c_ws), g_ws.cpu().numpy(), float(c_na), g_na.cpu().numpy()


def _case(cfg, frac):
    c = synth.make_case(cfg)
    return c, dev(frac * c.x_true), dev(c.s_exp)


def test_noalloc_matches_workspace_entry_two_calls_shrinking():
    torch.cuda.set_device(0)
    big = configs.SLICE_512
    small = configs.SMALL_64
    cb, xb, sb = _case(big, 0.7)
    cs, xs, ss = _case(small, 0.9)
    pb = ops.Plan.from_case(cb, adj_splits=4)
    ps = ops.Plan.from_case(cs)
    print(f"noalloc: 512^2 needs {pb.workspace_bytes(L.EIT_OP_COST_GRAD)} B, "
          f"64^2 needs {ps.workspace_bytes(L.EIT_OP_COST_GRAD)} B, limit {32 << 20} B", flush=True)
    for plan, x, s, cfg in ((pb, xb, sb, big), (ps, xs, ss, small)):
        c_ws, g_ws, c_na, g_na = _both(plan, x, s, cfg.lam_mu, cfg.lam_delta)
        assert np.isfinite(c_ws) and c_ws > 0
        assert c_na == c_ws                      # same kernels, same layout: bit-identical
        assert np.array_equal(g_na, g_ws)
    # the no-gradient form leaves grad untouched
    c = torch.empty((), dtype=torch.float64, device="cuda:0")
    L.check(L.lib().eit_cost_and_grad_noalloc(ps.handle, _ptr(xs), _ptr(ss), small.lam_mu,
                                              small.lam_delta, _ptr(c), None, _stream()))
    torch.cuda.synchronize()
    assert float(c) == c_ws


def test_noalloc_model_plan_matches_workspace_entry():
    """The full model of eq. 4 at the paper's acquisition (h-mode, single-map kernels, drift
    fitted, measured flat table): the parameter vector's gradient, bit for bit."""
    torch.cuda.set_device(0)
    from paper_2202_08627_amd import experiment
    cfg = configs.PAPER_220
    cases, _ = synth.make_stack(cfg, 8)
    c = cases[4]
    plan = experiment.model_plan(c, fit_drift=True, fit_ring=False)
    rng = np.random.default_rng(3)
    nn = cfg.n * cfg.n
    p = np.concatenate([0.9 * c.mu_true.ravel(), 0.01 * rng.standard_normal(cfg.n_theta)])
    assert p.size == plan.n_params
    x, s = dev(p), dev(c.s_exp)
    c_ws, g_ws, c_na, g_na = _both(plan, x, s, cfg.lam_mu, 0.0)
    print(f"noalloc model plan: cost {c_ws:.6e}, |g| {np.linalg.norm(g_ws):.3e}", flush=True)
    assert np.isfinite(c_ws) and c_ws > 0 and np.all(np.isfinite(g_ws[:nn]))
    assert c_na == c_ws
    assert np.array_equal(g_na, g_ws)


def test_noalloc_rejects_problems_over_the_limit():
    torch.cuda.set_device(0)
    cfg = configs.SLICE_1024
    g = ops.Geometry(cfg.n, cfg.n_theta, cfg.n_det, cfg.n_mask, cfg.kappa, synth.angles(cfg.n_theta),
                     synth.mask_positions(cfg.n_mask), np.ones(cfg.n_det), np.zeros(cfg.n_det),
                     np.full(cfg.n_det, 0.6))
    plan = ops.Plan(g, adj_splits=4)
    assert plan.workspace_bytes(L.EIT_OP_COST_GRAD) > (32 << 20)
    x = torch.zeros(plan.x_shape, dtype=torch.float32, device="cuda:0")
    s = torch.ones(plan.data_shape, dtype=torch.float32, device="cuda:0")
    c = torch.empty((), dtype=torch.float64, device="cuda:0")
    rc = L.lib().eit_cost_and_grad_noalloc(plan.handle, _ptr(x), _ptr(s), 0.0, 0.0, _ptr(c), None,
                                           _stream())
    assert rc == L.EIT_ERR_NOMEM
    assert b"static limit" in L.lib().eit_last_error()
