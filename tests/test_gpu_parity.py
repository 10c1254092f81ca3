"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same seeded
inputs. Tolerances: projections 1e-5 relative L2 (FP32), gradients 1e-4 relative L2,
cost 1e-6 relative (FP64 reduction of FP32 residuals), reconstructions after a fixed number
of iterations 1e-3 relative L2 per map."""
import dataclasses
import sys

import numpy as np
import pytest
import torch

from oracle import lbfgs as olbfgs
from oracle import model as omodel
from oracle import radon as oradon
from paper_2202_08627_amd import configs, synth
from helpers import geometry, rel_l2, tiny_cfg

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_08627_amd import ops as _ops
    return _ops


CASES = [
    tiny_cfg(n=16, n_theta=24),
    configs.SMALL_64,
    tiny_cfg(n=37, n_theta=13, n_det=45, n_mask=3),
    tiny_cfg(n=100, n_theta=7, n_det=70, n_mask=1),
    tiny_cfg(n=130, n_theta=181, n_det=131, n_mask=8),
]
IDS = [f"{c.n}x{c.n_theta}x{c.n_det}x{c.n_mask}" for c in CASES]


@pytest.mark.parametrize("cfg", CASES, ids=IDS)
def test_project_parity(ops, cfg):
    say("project", cfg.n, cfg.n_theta, cfg.n_det)
    c = synth.make_case(cfg)
    plan = ops.Plan.from_case(c)
    rng = np.random.default_rng(1)
    for x in (c.x_true, rng.standard_normal((2, cfg.n, cfg.n))):
        P = host(plan.project(dev(x)))
        x32 = x.astype(np.float32).astype(np.float64)
        ref = np.stack([oradon.project(x32[q], c.theta, cfg.n_det) for q in range(2)])
        assert rel_l2(P, ref) < 1e-5


@pytest.mark.parametrize("cfg", CASES, ids=IDS)
def test_backproject_parity(ops, cfg):
    say("backproject", cfg.n, cfg.n_theta, cfg.n_det)
    c = synth.make_case(cfg)
    plan = ops.Plan.from_case(c)
    rng = np.random.default_rng(2)
    y = rng.standard_normal((2, cfg.n_theta, cfg.n_det)).astype(np.float32).astype(np.float64)
    B = host(plan.backproject(dev(y)))
    ref = np.stack([oradon.backproject(y[q], c.theta, cfg.n) for q in range(2)])
    assert rel_l2(B, ref) < 1e-5


def test_adjoint_identity_on_gpu(ops):
    """<R x, y> = <x, R^T y> for the gather kernel against the ray kernel (FP32 operands,
    FP64 dot products on the host)."""
    cfg = configs.SLICE_512
    g = ops.Geometry(cfg.n, cfg.n_theta, cfg.n_det, cfg.n_mask, cfg.kappa, synth.angles(cfg.n_theta),
                     synth.mask_positions(cfg.n_mask), np.ones(cfg.n_det), np.zeros(cfg.n_det),
                     np.full(cfg.n_det, 0.6))
    plan = ops.Plan(g)
    gen = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn((2, cfg.n, cfg.n), device="cuda", generator=gen)
    y = torch.randn((2, cfg.n_theta, cfg.n_det), device="cuda", generator=gen)
    Rx = plan.project(x)
    RTy = plan.backproject(y)
    lhs = float((Rx.double() * y.double()).sum())
    rhs = float((x.double() * RTy.double()).sum())
    scale = float(Rx.double().norm() * y.double().norm())
    assert abs(lhs - rhs) < 1e-5 * scale


def test_no_sample_gives_flat_field(ops):
    """mu = delta = 0 => s_mod = f: the cost equals sum (f - s_exp)^2 (P6 on the device)."""
    cfg = configs.SMALL_64
    c = synth.make_case(cfg)
    plan = ops.Plan.from_case(c)
    z = np.zeros((2, cfg.n, cfg.n))
    cost, grad = plan.cost_and_grad(dev(z), dev(c.s_exp), 0.0, 0.0)
    f = c.flat_amp * np.exp(-(c.mask_pos[:, None] - c.flat_ctr) ** 2 / (2 * c.flat_sigma ** 2))
    ref = float(np.sum((f[None] - c.s_exp.astype(np.float64)) ** 2))
    assert float(cost) == pytest.approx(ref, rel=1e-6)


@pytest.mark.parametrize("cfg", CASES[:4], ids=IDS[:4])
def test_cost_and_grad_parity(ops, cfg):
    say("cost_and_grad", cfg.n, cfg.n_theta)
    c = synth.make_case(cfg)
    plan = ops.Plan.from_case(c)
    geo = geometry(c, omodel)
    rng = np.random.default_rng(3)
    x = c.x_true + 0.3 * np.stack([cfg.mu_scale * rng.standard_normal((cfg.n, cfg.n)),
                                   cfg.delta_scale * rng.standard_normal((cfg.n, cfg.n))])
    x = x.astype(np.float32).astype(np.float64)
    cost, grad = plan.cost_and_grad(dev(x), dev(c.s_exp), cfg.lam_mu, cfg.lam_delta)
    S, gm, gd = omodel.cost_and_grad(x[0], x[1], c.s_exp, geo, cfg.lam_mu, cfg.lam_delta)
    assert float(cost) == pytest.approx(S, rel=1e-5)
    G = host(grad)
    assert rel_l2(G[0], gm) < 1e-4
    assert rel_l2(G[1], gd) < 1e-4


@pytest.mark.parametrize("layout", ["jittered", "narrow"])
def test_cost_and_grad_mask_layouts(ops, layout):
    """The IC stage with mask positions off the equal spacing ('jittered') and with every
    other detector pixel given a flat-field width of 0.02 mask periods ('narrow': Gaussian
    factors down to exp(-600) and below, next to ordinary pixels in one wavefront)."""
    cfg = CASES[4]
    c = synth.make_case(cfg)
    if layout == "jittered":
        rng = np.random.default_rng(11)
        c = dataclasses.replace(c, mask_pos=c.mask_pos + 0.02 * rng.standard_normal(cfg.n_mask))
    else:
        sig = c.flat_sigma.copy()
        sig[::2] = 0.02
        c = dataclasses.replace(c, flat_sigma=sig)
    plan = ops.Plan.from_case(c)
    geo = geometry(c, omodel)
    x = (0.9 * c.x_true).astype(np.float32).astype(np.float64)
    cost, grad = plan.cost_and_grad(dev(x), dev(c.s_exp), cfg.lam_mu, cfg.lam_delta)
    S, gm, gd = omodel.cost_and_grad(x[0], x[1], c.s_exp, geo, cfg.lam_mu, cfg.lam_delta)
    assert float(cost) == pytest.approx(S, rel=1e-6)
    G = host(grad)
    assert rel_l2(G[0], gm) < 1e-4 and rel_l2(G[1], gd) < 1e-4


def test_autograd_function_matches_oracle(ops):
    cfg = configs.SMALL_64
    c = synth.make_case(cfg)
    plan = ops.Plan.from_case(c)
    geo = geometry(c, omodel)
    x = (c.x_true * 0.8).astype(np.float32).astype(np.float64)
    xt = dev(x).requires_grad_(True)
    S = ops.eit_cost(xt, dev(c.s_exp), plan, cfg.lam_mu, cfg.lam_delta)
    (2.0 * S).backward()
    S_o, gm, gd = omodel.cost_and_grad(x[0], x[1], c.s_exp, geo, cfg.lam_mu, cfg.lam_delta)
    assert float(S.detach()) == pytest.approx(S_o, rel=1e-5)
    G = host(xt.grad) / 2.0
    assert rel_l2(G[0], gm) < 1e-4 and rel_l2(G[1], gd) < 1e-4


def _oracle_recon(c, cfg, iters, m=10):
    geo = geometry(c, omodel)
    prob = omodel.ScaledProblem(c.s_exp, geo, cfg.lam, cfg.mu_scale, cfg.delta_scale)
    return olbfgs.reconstruct(prob, np.zeros((2, cfg.n, cfg.n)), iters, m=m)


@pytest.mark.parametrize("use_graph", [True, False])
def test_reconstruct_parity_small(ops, use_graph):
    """Plain method at 64^2 / 90 angles / M = 5: x_50 within 1e-3 relative L2 per map."""
    cfg = configs.SMALL_64
    say("reconstruct small graph=", use_graph)
    c = synth.make_case(cfg)
    plan = ops.Plan.from_case(c)
    x, rep, hist = plan.reconstruct(dev(c.s_exp), iters=cfg.iters, lam=cfg.lam, mu_scale=cfg.mu_scale,
                                    delta_scale=cfg.delta_scale, use_graph=use_graph, cost_hist=True)
    xo, st, tr = _oracle_recon(c, cfg, cfg.iters)
    say("report", rep, "oracle evals", st.evals)
    assert rep["rc"] == 0 and rep["iters"] == cfg.iters
    X = host(x)
    assert rel_l2(X[0], xo[0]) < 1e-3
    assert rel_l2(X[1], xo[1]) < 1e-3
    h = host(hist)
    assert np.allclose(h[1:], tr.cost, rtol=1e-4)
    assert np.all(np.diff(h) <= 0)


@pytest.mark.parametrize("m", [3, 20])
def test_reconstruct_parity_memory_sizes(ops, m):
    """Smallest and largest L-BFGS memory: with m = 20 the update produces 7 + 4*20 = 87
    inner products per block, more than one 64-wide pass of the finalize reduction."""
    cfg = configs.SMALL_64
    iters = 30
    say("reconstruct small m=", m)
    c = synth.make_case(cfg)
    plan = ops.Plan.from_case(c)
    x, rep, hist = plan.reconstruct(dev(c.s_exp), iters=iters, lam=cfg.lam, mu_scale=cfg.mu_scale,
                                    delta_scale=cfg.delta_scale, m=m, cost_hist=True)
    xo, st, tr = _oracle_recon(c, cfg, iters, m=m)
    assert rep["rc"] == 0 and rep["iters"] == iters
    X = host(x)
    assert rel_l2(X[0], xo[0]) < 1e-3
    assert rel_l2(X[1], xo[1]) < 1e-3
    assert np.allclose(host(hist)[1:], tr.cost, rtol=1e-4)


def test_reconstruct_forced_line_search_failure(ops):
    cfg = configs.SMALL_64
    c = synth.make_case(cfg)
    plan = ops.Plan.from_case(c)
    x, rep, _ = plan.reconstruct(dev(c.s_exp), iters=5, max_ls=0)
    assert rep["rc"] == -6 and rep["iters"] == 0


def test_reconstruct_nonfinite_data(ops):
    cfg = configs.SMALL_64
    c = synth.make_case(cfg)
    s = c.s_exp.copy()
    s[3, 1, 7] = np.nan
    plan = ops.Plan.from_case(c)
    x, rep, _ = plan.reconstruct(dev(s), iters=5)
    assert rep["rc"] == -5 and rep["iters"] == 0


def test_reconstruct_zero_iterations_returns_start(ops):
    cfg = configs.SMALL_64
    c = synth.make_case(cfg)
    plan = ops.Plan.from_case(c)
    x0 = dev(c.x_true)
    x, rep, _ = plan.reconstruct(dev(c.s_exp), x0=x0, iters=0)
    assert rep["rc"] == 0 and rep["iters"] == 0
    assert torch.allclose(x, x0, rtol=1e-6, atol=0)


def test_opts_validation(ops):
    from paper_2202_08627_amd import _lib as L
    cfg = configs.SMALL_64
    c = synth.make_case(cfg)
    plan = ops.Plan.from_case(c)
    for kw in (dict(m=0), dict(m=21), dict(lam=-1.0), dict(mu_scale=0.0), dict(c1=1.5),
               dict(iters=-1), dict(max_ls=-2)):
        with pytest.raises(L.EitError) as e:
            plan.reconstruct(dev(c.s_exp), **kw)
        assert e.value.code == L.EIT_ERR_INVALID_ARG


def _bench_plan(ops, c):
    """The plan the benchmark times: tiles from the autotuner's cache for this size class."""
    from paper_2202_08627_amd import autotune
    geo = ops.Geometry.from_case(c)
    return ops.Plan(geo, *autotune.tiling_for(geo))


def test_large_slice_sampled_projection(ops):
    """Full-size 512^2 / 720-angle workload: the projector in the benchmark's launch shape,
    checked against the oracle on 24 sampled angles (the oracle's rows are independent)."""
    cfg = configs.SLICE_512
    say("large projection")
    c = synth.make_case(cfg)
    plan = _bench_plan(ops, c)
    P = host(plan.project(dev(c.x_true)))
    sel = np.linspace(0, cfg.n_theta - 1, 24).astype(int)
    sel = np.unique(np.concatenate([sel, [0, 180, 360, 540]]))
    x32 = c.x_true.astype(np.float32).astype(np.float64)
    for q in range(2):
        ref = oradon.project(x32[q], c.theta[sel], cfg.n_det)
        assert rel_l2(P[q, sel], ref) < 1e-5


def test_large_slice_sampled_backprojection(ops):
    cfg = configs.SLICE_512
    c = synth.make_case(cfg)
    plan = _bench_plan(ops, c)
    rng = np.random.default_rng(4)
    sel = np.unique(np.linspace(0, cfg.n_theta - 1, 20).astype(int))
    y = np.zeros((2, cfg.n_theta, cfg.n_det))
    y[:, sel] = rng.standard_normal((2, sel.size, cfg.n_det)).astype(np.float32)
    B = host(plan.backproject(dev(y)))
    for q in range(2):
        ref = oradon.backproject(y[q, sel], c.theta[sel], cfg.n)
        assert rel_l2(B[q], ref) < 1e-5


def test_768_slice_sampled_parity_in_tuned_configuration(ops):
    """The batch's 768^2 / 1080-angle class in its tuned launch shape (autotuner cache):
    projections of the phantom on 16 sampled angles and the backprojection of a sinogram that
    is non-zero on 16 sampled angles, against the oracle."""
    from paper_2202_08627_amd import autotune
    cfg = configs.SliceConfig(n=768, n_theta=1080, n_det=768, n_mask=8, mu_scale=configs.mu_range_for(768))
    c = synth.make_case(cfg)
    say("768 sampled parity", autotune.tiling_for(ops.Geometry.from_case(c)))
    plan = _bench_plan(ops, c)
    sel = np.unique(np.concatenate([np.linspace(0, cfg.n_theta - 1, 12).astype(int),
                                    [0, 270, 540, 810]]))
    P = host(plan.project(dev(c.x_true)))
    x32 = c.x_true.astype(np.float32).astype(np.float64)
    for q in range(2):
        assert rel_l2(P[q, sel], oradon.project(x32[q], c.theta[sel], cfg.n_det)) < 1e-5
    rng = np.random.default_rng(9)
    y = np.zeros((2, cfg.n_theta, cfg.n_det))
    y[:, sel] = rng.standard_normal((2, sel.size, cfg.n_det)).astype(np.float32)
    B = host(plan.backproject(dev(y)))
    for q in range(2):
        assert rel_l2(B[q], oradon.backproject(y[q, sel], c.theta[sel], cfg.n)) < 1e-5


def test_large_slice_reconstruction_in_bench_configuration(ops):
    """The benchmark's run (512^2 / 720 / M = 8, autotuned tiles, captured graphs), 20
    iterations: the cost history never rises, and at the returned x_20 (non-zero up to the
    map's border, unlike the phantom) the reported cost, the device cost and the device
    gradient are the oracle's (1e-6, 1e-6, 1e-4 relative)."""
    cfg = configs.SLICE_512
    say("large reconstruction")
    c = synth.make_case(cfg)
    plan = _bench_plan(ops, c)
    iters = 20
    x, rep, hist = plan.reconstruct(dev(c.s_exp), iters=iters, lam=cfg.lam, mu_scale=cfg.mu_scale,
                                    delta_scale=cfg.delta_scale, m=10, cost_hist=True)
    assert rep["rc"] == 0 and rep["iters"] == iters
    h = host(hist)
    assert np.all(np.diff(h) <= 0)
    X = host(x)
    geo = geometry(c, omodel)
    S, gm, gd = omodel.cost_and_grad(X[0], X[1], c.s_exp, geo, cfg.lam_mu, cfg.lam_delta)
    cost, grad = plan.cost_and_grad(x, dev(c.s_exp), cfg.lam_mu, cfg.lam_delta)
    G = host(grad)
    e = (abs(rep["cost"] - S) / S, abs(float(cost.cpu()) - S) / S, rel_l2(G[0], gm), rel_l2(G[1], gd))
    say("reported cost, cost, grad mu, grad delta rel:", e)
    assert e[0] < 1e-6 and e[1] < 1e-6
    assert e[2] < 1e-4 and e[3] < 1e-4


def _variant_case():
    cfg = tiny_cfg(n=130, n_theta=181, n_det=131, n_mask=8)
    return cfg, synth.make_case(cfg)


def test_every_projector_variant(ops):
    """Each compiled projector tile variant (both LDS layouts) on a multi-tile ragged geometry,
    for a dense random map and for a map that is non-zero only on its border rows and columns
    (the window entries that straddle the map's edge: a duplicated entry at column -1 must
    still carry column 0)."""
    from paper_2202_08627_amd import _lib as L
    cfg, c = _variant_case()
    rng = np.random.default_rng(7)
    x = rng.standard_normal((2, cfg.n, cfg.n)).astype(np.float32).astype(np.float64)
    border = np.zeros_like(x)
    for e in (0, -1):
        border[:, e, :] = x[:, e, :]
        border[:, :, e] = x[:, :, e]
    refs = [(xx, np.stack([oradon.project(xx[q], c.theta, cfg.n_det) for q in range(2)]))
            for xx in (x, border)]
    tried = 0
    for v in range(len(ops.variants(0))):
        try:
            plan = ops.Plan(ops.Geometry.from_case(c), proj_variant=v, adj_variant=0)
        except L.EitError as e:
            assert e.code == L.EIT_ERR_SHAPE      # window wider than this variant's pitch
            continue
        say("projector variant", v)
        for xx, ref in refs:
            assert rel_l2(host(plan.project(dev(xx))), ref) < 1e-5, v
        tried += 1
    assert tried >= len(ops.variants(0)) // 2


def test_every_adjoint_variant(ops):
    """Each compiled adjoint tile variant, unsplit and with its angle chunks divided among 3
    blocks per voxel tile and among as many blocks as chunks (uneven ranges, one chunk per
    block). A split result may differ from the unsplit one only by the order of the FP64
    partial sums, and repeated calls must agree bitwise."""
    cfg, c = _variant_case()
    rng = np.random.default_rng(8)
    y = rng.standard_normal((2, cfg.n_theta, cfg.n_det)).astype(np.float32).astype(np.float64)
    ref = np.stack([oradon.backproject(y[q], c.theta, cfg.n) for q in range(2)])
    yd = dev(y)
    for v in range(len(ops.variants(1))):
        base = None
        for g in (1, 3, 64):
            say("adjoint variant", v, "split", g)
            plan = ops.Plan(ops.Geometry.from_case(c), adj_variant=v, adj_splits=g)
            out = plan.backproject(yd)
            assert rel_l2(host(out), ref) < 1e-5, (v, g)
            if base is None:
                base = out
            else:
                assert float((out - base).abs().max()) <= 1e-6 * float(base.abs().max()), (v, g)
            assert torch.equal(plan.backproject(yd), out), (v, g)


def test_split_adjoint_in_cost_and_gradient(ops):
    """The gradient path with the adjoint split over 4 blocks per tile (regulariser added by
    the block that combines the partials) against the oracle."""
    cfg = CASES[1]
    c = synth.make_case(cfg)
    plan = ops.Plan.from_case(c, adj_splits=4)
    geo = geometry(c, omodel)
    rng = np.random.default_rng(5)
    x = c.x_true + 0.3 * np.stack([cfg.mu_scale * rng.standard_normal((cfg.n, cfg.n)),
                                   cfg.delta_scale * rng.standard_normal((cfg.n, cfg.n))])
    x = x.astype(np.float32).astype(np.float64)
    cost, grad = plan.cost_and_grad(dev(x), dev(c.s_exp), cfg.lam_mu, cfg.lam_delta)
    S, gm, gd = omodel.cost_and_grad(x[0], x[1], c.s_exp, geo, cfg.lam_mu, cfg.lam_delta)
    assert float(cost) == pytest.approx(S, rel=1e-5)
    G = host(grad)
    assert rel_l2(G[0], gm) < 1e-4 and rel_l2(G[1], gd) < 1e-4


def test_reconstruct_parity_with_split_adjoint(ops):
    """The plain method with the adjoint split over 3 blocks per tile: the optimiser's update
    then forms each gradient from the partial planes (plus the regulariser) instead of
    reading a finished gradient."""
    cfg = configs.SMALL_64
    say("reconstruct small split adjoint")
    c = synth.make_case(cfg)
    plan = ops.Plan.from_case(c, adj_splits=3)
    assert ops.inspect(plan.geo, adj_splits=3)["adj_splits"] == 3
    x, rep, hist = plan.reconstruct(dev(c.s_exp), iters=cfg.iters, lam=cfg.lam, mu_scale=cfg.mu_scale,
                                    delta_scale=cfg.delta_scale, cost_hist=True)
    xo, st, tr = _oracle_recon(c, cfg, cfg.iters)
    assert rep["rc"] == 0 and rep["iters"] == cfg.iters
    X = host(x)
    assert rel_l2(X[0], xo[0]) < 1e-3
    assert rel_l2(X[1], xo[1]) < 1e-3
    assert np.allclose(host(hist)[1:], tr.cost, rtol=1e-4)


def _mirror_variants(ops):
    return [v for v, t in enumerate(ops.variants(1)) if t[4]]


def test_mirror_adjoint_irregular_angles(ops):
    """The mirror-pair adjoint on an odd map (its middle row is its own mirror) with an odd
    detector count and an angle list that is only partly symmetric: 25 mirrored pairs, 15
    angles without a mirror, 0 with pi, and pi/2 (its own mirror), in shuffled order. Every
    mirror variant, unsplit and split, against the oracle; repeated calls agree bitwise."""
    cfg = tiny_cfg(n=67, n_theta=68, n_det=71, n_mask=4)
    c = synth.make_case(cfg)
    rng = np.random.default_rng(11)
    base = rng.uniform(0, np.pi, 40)
    theta = np.concatenate([base, np.pi - base[:25], [0.0, np.pi / 2, np.pi]])
    theta = theta[rng.permutation(len(theta))]
    assert len(theta) == cfg.n_theta
    geo = ops.Geometry.from_case(c)
    geo.theta = theta
    y = rng.standard_normal((2, cfg.n_theta, cfg.n_det)).astype(np.float32).astype(np.float64)
    ref = np.stack([oradon.backproject(y[q], theta, cfg.n) for q in range(2)])
    yd = dev(y)
    for v in _mirror_variants(ops):
        for g in (1, 2):
            say("mirror adjoint variant", v, "split", g)
            plan = ops.Plan(geo, adj_variant=v, adj_splits=g)
            out = plan.backproject(yd)
            assert rel_l2(host(out), ref) < 1e-5, (v, g)
            assert torch.equal(plan.backproject(yd), out), (v, g)


def test_mirror_adjoint_no_mirrors(ops):
    """An angle list with no mirror pairs at all: every angle reaches its voxel pairs through
    the two windows of its own bins."""
    cfg = tiny_cfg(n=48, n_theta=19, n_det=50, n_mask=4)
    c = synth.make_case(cfg)
    rng = np.random.default_rng(12)
    theta = np.sort(rng.uniform(-np.pi, 2 * np.pi, cfg.n_theta))
    geo = ops.Geometry.from_case(c)
    geo.theta = theta
    y = rng.standard_normal((2, cfg.n_theta, cfg.n_det)).astype(np.float32).astype(np.float64)
    ref = np.stack([oradon.backproject(y[q], theta, cfg.n) for q in range(2)])
    for v in _mirror_variants(ops):
        say("mirror adjoint variant", v, "without mirrors")
        plan = ops.Plan(geo, adj_variant=v)
        assert ops.inspect(geo, adj_variant=v)["n_pairs"] == cfg.n_theta
        assert rel_l2(host(plan.backproject(dev(y))), ref) < 1e-5, v


def test_mirror_adjoint_in_gradient_and_reconstruction(ops):
    """The mirror-pair adjoint inside the cost gradient (split: combine pass) and inside the
    plain method (split: the optimiser's update adds the partial planes) against the oracle."""
    cfg = configs.SMALL_64
    c = synth.make_case(cfg)
    v = _mirror_variants(ops)[0]
    geo = geometry(c, omodel)
    rng = np.random.default_rng(5)
    x = c.x_true + 0.3 * np.stack([cfg.mu_scale * rng.standard_normal((cfg.n, cfg.n)),
                                   cfg.delta_scale * rng.standard_normal((cfg.n, cfg.n))])
    x = x.astype(np.float32).astype(np.float64)
    S, gm, gd = omodel.cost_and_grad(x[0], x[1], c.s_exp, geo, cfg.lam_mu, cfg.lam_delta)
    for g in (1, 2):
        say("mirror adjoint gradient split", g)
        plan = ops.Plan.from_case(c, adj_variant=v, adj_splits=g)
        cost, grad = plan.cost_and_grad(dev(x), dev(c.s_exp), cfg.lam_mu, cfg.lam_delta)
        assert float(cost) == pytest.approx(S, rel=1e-5)
        G = host(grad)
        assert rel_l2(G[0], gm) < 1e-4 and rel_l2(G[1], gd) < 1e-4
    say("mirror adjoint reconstruct")
    plan = ops.Plan.from_case(c, adj_variant=v, adj_splits=2)
    xr, rep, hist = plan.reconstruct(dev(c.s_exp), iters=cfg.iters, lam=cfg.lam,
                                     mu_scale=cfg.mu_scale, delta_scale=cfg.delta_scale,
                                     cost_hist=True)
    xo, st, tr = _oracle_recon(c, cfg, cfg.iters)
    assert rep["rc"] == 0 and rep["iters"] == cfg.iters
    X = host(xr)
    assert rel_l2(X[0], xo[0]) < 1e-3 and rel_l2(X[1], xo[1]) < 1e-3
    assert np.allclose(host(hist)[1:], tr.cost, rtol=1e-4)


def test_mirror_adjoint_degenerate_shapes(ops):
    """The mirror-pair adjoint at the smallest sizes: maps of 2, 3 and 5 voxels (the middle
    row of the odd ones is its own mirror) with one angle, with 0 and pi/2 (both their own
    mirrors) and with one mirrored pair, against the oracle."""
    rng = np.random.default_rng(14)
    for n in (2, 3, 5):
        for theta in (np.array([0.4]), np.array([0.0, np.pi / 2]), np.array([0.3, np.pi - 0.3])):
            cfg = tiny_cfg(n=n, n_theta=len(theta), n_det=n + 1, n_mask=3)
            c = synth.make_case(cfg)
            geo = ops.Geometry.from_case(c)
            geo.theta = theta
            y = rng.standard_normal((2, len(theta), cfg.n_det)).astype(np.float32).astype(np.float64)
            ref = np.stack([oradon.backproject(y[q], theta, n) for q in range(2)])
            for v in _mirror_variants(ops):
                say("mirror adjoint degenerate", n, len(theta), v)
                plan = ops.Plan(geo, adj_variant=v)
                assert rel_l2(host(plan.backproject(dev(y))), ref) < 1e-5, (n, theta, v)
