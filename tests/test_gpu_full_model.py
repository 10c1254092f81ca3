"""The full forward model of eq. 4 on the GPU (h-mode, fitted drift m_o and ring term m_r,
measured flat tables) against the FP64 oracle (oracle/full_model.py) on the same seeded
inputs: cost and gradient for every option and combination, fixed-K reconstruction through
the device-side L-BFGS, and the single-shot retrieval of eq. 3.

Bounds: cost 1e-5 relative; gradient 1e-4 relative L2 over each block of the parameter
vector (maps, drift, ring); x_K 1e-3 relative L2 per block, as for the plain model."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import full_model as fm
from oracle import lbfgs as olbfgs
from oracle import single_shot as oss
from paper_2202_08627_amd import configs, synth
from helpers import rel_l2, tiny_cfg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_08627_amd import ops as _ops
    return _ops


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def say(*a):
    print(*a, flush=True)


# small two-map case with drift and a measured flat; the paper-shaped h-mode case
SMALL_EXT = dataclasses.replace(configs.SMALL_64, flat_scans=20, drift_amp=0.02, sigma_jitter=0.05)
SMALL_H = dataclasses.replace(tiny_cfg(n=48, n_theta=80, n_mask=1, jitter=0.05), angle_span=2.0,
                              mask_list=(0.3,), sigma=0.3, kappa=1.0, gamma_h=5.0, flat_scans=1,
                              drift_amp=0.02, n_ellipses=6)
PAPER = configs.PAPER_220
# h-mode with more than 2048 detector pixels: evaluated as the pair [h, h] by the two-map
# kernels (every other h-mode case runs the single-map kernels)
WIDE_H = dataclasses.replace(tiny_cfg(n=24, n_theta=12, n_mask=1, n_det=2056, jitter=0.05),
                             angle_span=2.0, mask_list=(0.3,), sigma=0.3, kappa=1.0, gamma_h=5.0,
                             flat_scans=1, drift_amp=0.02, n_ellipses=3)


def oracle_setup(c, model):
    cfg = c.cfg
    return fm.Setup(cfg.n, c.theta, cfg.n_det, c.mask_pos, c.flat_amp, c.flat_ctr, c.flat_sigma,
                    cfg.kappa, hmode=model.hmode, gamma=model.gamma, fit_mo=model.fit_drift,
                    fit_mr=model.fit_ring, flat_table=model.flat_table, table_u0=model.table_u0,
                    table_du=model.table_du)


def blocks(st):
    """(name, slice) of the parameter vector's blocks."""
    nn = st.n * st.n
    out = [("maps", slice(0, st.n_maps * nn))]
    off = st.n_maps * nn
    if st.fit_mo:
        out.append(("m_o", slice(off, off + st.theta.size)))
        off += st.theta.size
    if st.fit_mr:
        out.append(("m_r", slice(off, off + st.n_det)))
    return out


def _point(c, st, rng):
    """A point near the phantom, with offsets of the size the drift has."""
    nn = st.n * st.n
    mu = 0.9 * c.mu_true.ravel() + 0.05 * c.cfg.mu_scale * rng.uniform(0, 1, nn)
    parts = [mu] if st.hmode else [mu, 0.9 * c.delta_true.ravel() + 5e-5 * rng.uniform(0, 1, nn)]
    if st.fit_mo:
        parts.append(0.02 * rng.standard_normal(st.theta.size))
    if st.fit_mr:
        parts.append(0.01 * rng.standard_normal(st.n_det))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


OPTIONS = [
    ("hmode", SMALL_H, dict(hmode=True, use_table=False)),
    ("hmode-table", SMALL_H, dict(hmode=True)),
    ("drift", SMALL_EXT, dict(hmode=False, fit_drift=True, use_table=False)),
    ("ring", SMALL_EXT, dict(hmode=False, fit_ring=True, use_table=False)),
    ("table", SMALL_EXT, dict(hmode=False)),
    ("two-map-all", SMALL_EXT, dict(hmode=False, fit_drift=True, fit_ring=True)),
    ("hmode-all", SMALL_H, dict(hmode=True, fit_drift=True, fit_ring=True)),
    ("paper-all", PAPER, dict(hmode=True, fit_drift=True, fit_ring=True)),
    ("hmode-pair-wide", WIDE_H, dict(hmode=True, fit_drift=True)),
]


@pytest.mark.parametrize("name,cfg,kw", OPTIONS, ids=[o[0] for o in OPTIONS])
def test_cost_and_gradient_parity(ops, name, cfg, kw):
    c = synth.make_case(cfg)
    model = ops.Model.from_case(c, **kw)
    plan = ops.Plan(ops.Geometry.from_case(c), model=model)
    st = oracle_setup(c, model)
    assert plan.n_params == st.n_params
    p = _point(c, st, np.random.default_rng(11))
    lam_mu, lam_de = (cfg.lam_mu, 0.0) if st.hmode else (cfg.lam_mu, cfg.lam_delta)
    cost, grad = plan.cost_and_grad(dev(p), dev(c.s_exp), lam_mu, lam_de)
    S, g = fm.cost_and_grad(st, p, c.s_exp, lam_mu, lam_de)
    G = grad.cpu().numpy().astype(np.float64)
    e_c = abs(float(cost) - S) / S
    errs = {b: rel_l2(G[sl], g[sl]) for b, sl in blocks(st)}
    say(f"full model {name}: cost rel {e_c:.2e}, gradient rel-L2 {errs}")
    assert e_c < 1e-5
    for b, e in errs.items():
        assert e < 1e-4, (b, e)
    # the cost-only call gives the same value
    c2, _ = plan.cost_and_grad(dev(p), dev(c.s_exp), lam_mu, lam_de, want_grad=False)
    assert float(c2) == float(cost)


RECON = [
    ("hmode-all", SMALL_H, dict(hmode=True, fit_drift=True, fit_ring=True), 40),
    ("two-map-drift-table", SMALL_EXT, dict(hmode=False, fit_drift=True), 30),
]


@pytest.mark.parametrize("name,cfg,kw,iters", RECON, ids=[r[0] for r in RECON])
def test_fixed_k_reconstruction_parity(ops, name, cfg, kw, iters):
    c = synth.make_case(cfg)
    model = ops.Model.from_case(c, **kw)
    plan = ops.Plan(ops.Geometry.from_case(c), model=model)
    st = oracle_setup(c, model)
    scale = cfg.mu_scale if st.hmode else (cfg.mu_scale, cfg.delta_scale)
    x, rep, hist = plan.reconstruct(dev(c.s_exp), iters=iters, lam=cfg.lam, mu_scale=cfg.mu_scale,
                                    delta_scale=cfg.delta_scale, cost_hist=True)
    prob = fm.ScaledProblem(st, c.s_exp, cfg.lam, scale, model.offset_scale)
    z, ost, tr = olbfgs.minimize(prob, np.zeros(st.n_params), iters)
    xo = prob.to_p(z)
    X = x.cpu().numpy().astype(np.float64)
    errs = {b: rel_l2(X[sl], xo[sl]) for b, sl in blocks(st)}
    h = hist.cpu().numpy()[1:]
    say(f"full model x_{iters} {name}: rel-L2 {errs}; evals GPU {rep['evals']} oracle {ost.evals}")
    assert rep["rc"] == 0 and rep["iters"] == iters
    for b, e in errs.items():
        assert e < 1e-3, (b, e)
    assert np.allclose(h, tr.cost, rtol=1e-4)
    assert np.all(np.diff(hist.cpu().numpy()) <= 0)


@pytest.mark.parametrize("cfg,use_table", [(SMALL_H, False), (SMALL_H, True), (PAPER, True)],
                         ids=["48-gauss", "48-table", "paper-table"])
def test_eq3_single_shot_parity(ops, cfg, use_table):
    c = synth.make_case(cfg)
    model = ops.Model.from_case(c, hmode=True, fit_drift=True, use_table=use_table)
    plan = ops.Plan(ops.Geometry.from_case(c), model=model)
    st = oracle_setup(c, model)
    out = plan.single_shot(dev(c.s_exp)).cpu().numpy().astype(np.float64)
    nn = cfg.n * cfg.n
    f, fp = fm.flat_ic(st, np.broadcast_to(c.mask_pos[0], (1, cfg.n_det)).copy())
    ref = oss.reconstruct_eq3(c.s_exp, c.theta, cfg.n, 0, f[0], fp[0], cfg.kappa * model.gamma)
    e = rel_l2(out[:nn], ref.ravel())
    say(f"eq. 3 single shot {cfg.n}^2 table={use_table}: rel-L2 {e:.2e}")
    assert e < 1e-4
    assert np.all(out[nn:] == 0.0)


def test_model_batch_equals_single_slice_runs(ops):
    """Model plans of different options in one batch (h-mode with drift and ring, h-mode with
    drift, two maps with drift and a table): each slice equals its own run bitwise; a batch
    mixing plain and model plans is refused."""
    cases, _ = synth.make_stack(dataclasses.replace(SMALL_H, n=40, n_det=44), 3, n_granules=4)
    opts = [dict(hmode=True, fit_drift=True, fit_ring=True), dict(hmode=True, fit_drift=True),
            dict(hmode=True, fit_ring=True, use_table=False)]
    plans = [ops.Plan(ops.Geometry.from_case(c), model=ops.Model.from_case(c, **o))
             for c, o in zip(cases, opts)]
    two = synth.make_case(dataclasses.replace(SMALL_EXT, n=36, n_theta=50, n_det=36))
    plans.append(ops.Plan(ops.Geometry.from_case(two), adj_splits=2,
                          model=ops.Model.from_case(two, hmode=False, fit_drift=True)))
    s = [dev(c.s_exp) for c in cases] + [dev(two.s_exp)]
    kw = dict(iters=15, lam=1e-2, mu_scale=SMALL_H.mu_scale, delta_scale=1e-3)
    xs, reps = ops.reconstruct_batch(plans, s, **kw)
    for i, (p, si) in enumerate(zip(plans, s)):
        x1, r1, _ = p.reconstruct(si, **kw)
        assert reps[i]["status"] == 0 and reps[i]["iters"] == 15, (i, reps[i])
        assert r1["evals"] == reps[i]["evals"]
        assert torch.equal(x1, xs[i]), i
    plain = ops.Plan(ops.Geometry.from_case(two))
    from paper_2202_08627_amd import _lib as L
    with pytest.raises(L.EitError) as e:
        ops.reconstruct_batch([plans[0], plain], [s[0], dev(two.s_exp)], iters=2)
    assert e.value.code == L.EIT_ERR_INVALID_ARG
