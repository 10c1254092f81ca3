"""C-ABI checks that need no GPU: every declared symbol is exported, host-side validation
returns the documented error codes before any device call, and the launch geometry the
host tables produce keeps every LDS access of the projector and adjoint kernels in
bounds (emulating the kernels' FP32/FP64 index arithmetic on the host)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2202_08627_amd import _lib as L
from paper_2202_08627_amd import configs, ops, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eitomo.h")

pytestmark = pytest.mark.skipif(not os.path.exists(L.LIB_PATH), reason="library not built")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(eit_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 10
    lib = C.CDLL(L.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


def geo_for(cfg, **over):
    c = synth.make_case(cfg) if cfg.n <= 128 else None
    if c is not None:
        g = ops.Geometry.from_case(c)
    else:
        g = ops.Geometry(cfg.n, cfg.n_theta, cfg.n_det, cfg.n_mask, cfg.kappa,
                         synth.angles(cfg.n_theta), synth.mask_positions(cfg.n_mask),
                         np.ones(cfg.n_det), np.zeros(cfg.n_det), np.full(cfg.n_det, 0.6))
    for k, v in over.items():
        setattr(g, k, v)
    return g


def inspect_rc(g):
    try:
        ops.inspect(g)
        return 0
    except L.EitError as e:
        return e.code


def test_validation_errors():
    g = geo_for(configs.SMALL_64)
    assert inspect_rc(g) == 0
    import copy
    for field, val, code in [("n", 1, L.EIT_ERR_SHAPE), ("n", 5000, L.EIT_ERR_SHAPE),
                             ("n_det", 1, L.EIT_ERR_SHAPE), ("n_mask", 0, L.EIT_ERR_SHAPE),
                             ("n_theta", 0, L.EIT_ERR_SHAPE), ("kappa", float("nan"), L.EIT_ERR_INVALID_ARG)]:
        gg = copy.copy(g)
        setattr(gg, field, val)
        m = max(gg.n_mask, 1)
        gg.mask_pos = np.zeros(m)
        gg.theta = np.zeros(max(gg.n_theta, 1))
        gg.flat_amp = np.ones(max(gg.n_det, 1))
        gg.flat_ctr = np.zeros(max(gg.n_det, 1))
        gg.flat_sigma = np.ones(max(gg.n_det, 1))
        assert inspect_rc(gg) == code, field
    gg = copy.copy(g)
    gg.flat_sigma = np.full(g.n_det, -1.0)
    assert inspect_rc(gg) == L.EIT_ERR_INVALID_ARG
    gg = copy.copy(g)
    gg.theta = np.full(g.n_theta, np.inf)
    assert inspect_rc(gg) == L.EIT_ERR_INVALID_ARG


def test_null_arguments_rejected_without_device():
    lib = L.lib()
    assert lib.eit_project(None, None, None, None, 0, None) == L.EIT_ERR_INVALID_ARG
    assert lib.eit_backproject(None, None, None, None, 0, None) == L.EIT_ERR_INVALID_ARG
    assert lib.eit_cost_and_grad(None, None, None, 0.0, 0.0, None, None, None, 0, None) == L.EIT_ERR_INVALID_ARG
    assert lib.eit_reconstruct(None, None, None, None, None, None, None, 0, None) == L.EIT_ERR_INVALID_ARG
    assert lib.eit_workspace_bytes(None, L.EIT_OP_RECONSTRUCT, 10) == 0
    assert b"NULL" in lib.eit_last_error()
    assert lib.eit_plan_create(None, None, None, None) == L.EIT_ERR_INVALID_ARG


def test_variant_registry():
    pv = ops.variants(0)
    av = ops.variants(1)
    assert len(pv) >= 3 and len(av) >= 3
    for a, w, r, dup in pv:
        assert a * w <= 1024 and w % 64 == 0 and dup in (0, 1)
    for tx, ty, ac, vpt, mir in av:
        assert tx * ty // vpt <= 1024 and (tx * ty // vpt) % 64 == 0 and mir in (0, 1)
    assert {v[4] for v in av} == {0, 1}


def f32(v):
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


def fmaf(a, b, c):
    # float32 fused multiply-add: exact product in FP64 (24x24 bits), one rounding to FP32
    return f32(np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64))


def check_projector_bounds(g, pv):
    """Emulates the projector's per-strip origin (FP64 floor split) and per-row FP32 FMA, and
    checks that the LDS column floor(u) + ioff stays in [0, win_w - 2] with no clamping."""
    try:
        info = ops.inspect(g, proj_variant=pv, tables=True)
    except L.EitError as e:
        assert e.code == L.EIT_ERR_SHAPE      # window wider than this variant's pitch
        return False
    A, W, R = info["proj_a"], info["proj_w"], info["proj_r"]
    assert info["proj_lds_bytes"] <= 64 * 1024
    assert info["win_pitch"] >= info["win_w"]
    pa, groups, wl = info["proj_angles"], info["groups"], info["win_lo"]
    ng, nb, ns = wl.shape
    nd = g.n_det
    a_eff = np.where(groups >= 0, groups, groups[:, :1])                     # [ng, A]
    src = pa[a_eff, 5]
    assert np.all(src == src[:, :1])
    kl = np.array([0, W - 1])
    k = np.arange(nb)[:, None] * W + kl[None, :]                              # [nb, 2]
    k_eff = np.minimum(k, nd - 1)
    t = k_eff - 0.5 * (nd - 1)
    inv = pa[a_eff, 0][:, None, :, None]                                      # [ng,1,A,1]
    base = pa[a_eff, 1][:, None, :, None]
    slope = pa[a_eff, 2][:, None, :, None, None]
    slope_f = pa[a_eff, 3][:, None, :, None, None]
    ut0 = t[None, :, None, :] * inv + base                                   # [ng,nb,A,2]
    p0 = (np.arange(ns) * R).astype(np.float64)
    lo = wl.astype(np.float64)[:, :, None, None, :]                          # [ng,nb,1,1,ns]
    up0 = ut0[..., None] + p0 * slope                                         # [ng,nb,A,2,ns]
    fl0 = np.floor(up0 + np.minimum(0.0, (R - 1) * slope)) - 1.0
    uf = f32(up0 - fl0)
    ioff = fl0 - lo
    assert ioff.min() >= 0
    for r in (0, R - 1):
        u = fmaf(float(r), slope_f, uf)
        assert u.min() >= 0.0, (pv, u.min())           # truncation is the floor
        col = np.trunc(u) + ioff
        assert col.max() <= info["win_w"] - 2, (pv, col.max(), info["win_w"])
    return True


def check_adjoint_bounds(g, av, vpt):
    """Emulates the adjoint's tile origin (FP64) and per-voxel FP32 FMAs (including the
    row offsets of a thread's extra voxels) and checks bins stay in [0, kwin - 2]. The
    mirror-pair kernel evaluates a second coordinate per voxel, in the mirror frame (cos
    negated, offset cd_s), for the tiles of the top half; both are replayed."""
    info = ops.inspect(g, adj_variant=av, tables=True)
    TX, TY, kwin = info["adj_tx"], info["adj_ty"], info["kwin"]
    assert kwin <= info["kwin_pitch_limit"]
    if info["adj_mirror"]:
        assert info["n_ty"] * TY >= (g.n + 1) // 2
        aa = info["adj_angles"]
        _adjoint_frame_bounds(info, vpt, aa[:, 0], aa[:, 1], aa[:, 2], aa[:, 3], aa[:, 4])
        _adjoint_frame_bounds(info, vpt, -aa[:, 0], aa[:, 1], aa[:, 8], -aa[:, 3], aa[:, 4])
        return
    aa = info["adj_angles"]
    _adjoint_frame_bounds(info, vpt, *(aa[:, q] for q in range(5)))


def _adjoint_frame_bounds(info, vpt, cs, sn, cd, csf, snf):
    TX, TY, kwin = info["adj_tx"], info["adj_ty"], info["kwin"]
    JS = TY // vpt
    i0 = (np.arange(info["n_tx"]) * TX).astype(np.float64)
    j0 = (np.arange(info["n_ty"]) * TY).astype(np.float64)
    I0, J0 = np.meshgrid(i0, j0, indexing="xy")
    I0 = I0.ravel()[:, None]
    J0 = J0.ravel()[:, None]
    uc = J0 * sn + (I0 * cs + cd)
    umin = uc + np.minimum(0.0, (TX - 1) * cs) + np.minimum(0.0, (TY - 1) * sn)
    lo = np.floor(umin) - 1
    offs = f32(uc - lo)
    for il in (0, TX - 1):
        for jl in (0, JS - 1):
            u0 = fmaf(float(il), csf, fmaf(float(jl), snf, offs))
            for q in (0, vpt - 1):
                u = u0 if q == 0 else fmaf(float(q * JS), snf, u0)
                assert u.min() >= 0.0, (av, u.min())       # truncation is the floor
                b = np.trunc(u)
                assert b.max() <= kwin - 2, (av, b.max(), kwin)


SHAPES = [configs.SMALL_64, configs.SLICE_512, configs.SLICE_1024,
          configs.SliceConfig(n=256, n_theta=360, n_det=256, n_mask=8),
          configs.SliceConfig(n=768, n_theta=1080, n_det=768, n_mask=8),
          configs.SliceConfig(n=37, n_theta=13, n_det=45, n_mask=3),
          configs.SliceConfig(n=100, n_theta=7, n_det=70, n_mask=1)]


def _all_variants(g):
    ok = [check_projector_bounds(g, pv) for pv in range(len(ops.variants(0)))]
    assert ok[ops.inspect(g)["proj_variant"]]        # the default variant must apply
    for av, (tx, ty, ac, vpt, mir) in enumerate(ops.variants(1)):
        check_adjoint_bounds(g, av, vpt)


@pytest.mark.parametrize("cfg", SHAPES, ids=lambda c: f"{c.n}x{c.n_theta}x{c.n_det}")
def test_lds_indices_in_bounds(cfg):
    _all_variants(geo_for(cfg))


def test_irregular_angles_in_bounds():
    rng = np.random.default_rng(0)
    g = geo_for(configs.SliceConfig(n=96, n_theta=50, n_det=110, n_mask=4))
    g.theta = np.sort(rng.uniform(-np.pi, 2 * np.pi, g.n_theta))
    _all_variants(g)


def test_row_flags_match_oracle_rule():
    """The plan's FP64 row/column decision is the one the oracle's projector uses."""
    from oracle import radon
    g = geo_for(configs.SliceConfig(n=64, n_theta=720, n_det=64, n_mask=5))
    info = ops.inspect(g, tables=True)
    src = info["proj_angles"][:, 5]
    assert np.array_equal(src == 0, radon.row_flags(g.theta))


def _mirror_variant():
    return next(v for v, t in enumerate(ops.variants(1)) if t[4])


def test_mirror_pairs():
    """Angle pairing of the mirror-pair adjoint: for a*pi/N_theta every a in 1 .. N/2 - 1 pairs
    with N - a, while 0 and pi/2 (its own mirror) stay unpaired; for any angle list every pair
    satisfies cos b = -cos a, sin b = sin a, every angle sits in exactly one pair slot, and
    the pair count and chunk split follow."""
    mv = _mirror_variant()
    g = geo_for(configs.SLICE_512)
    info = ops.inspect(g, adj_variant=mv, tables=True)
    mate = info["adj_angles"][:, 9].astype(int)
    nt = g.n_theta
    assert info["adj_mirror"] == 1 and info["n_pairs"] == nt // 2 + 1
    assert mate[0] == -1 and mate[nt // 2] == -1
    assert all(mate[a] == nt - a for a in range(1, nt // 2))
    assert all(mate[a] == -2 for a in range(nt // 2 + 1, nt))
    # the unpaired kernel reports no pairs
    assert ops.inspect(g, adj_variant=3, tables=True)["n_pairs"] == 0
    rng = np.random.default_rng(3)
    base = rng.uniform(0, np.pi, 40)
    for theta in (np.sort(rng.uniform(-np.pi, 2 * np.pi, 50)),       # no mirrors
                  np.concatenate([base, np.pi - base[:25], [0.0, np.pi / 2, np.pi]])):
        gg = geo_for(configs.SliceConfig(n=66, n_theta=len(theta), n_det=70, n_mask=4))
        gg.theta = theta
        inf = ops.inspect(gg, adj_variant=mv, tables=True)
        m = inf["adj_angles"][:, 9].astype(int)
        firsts = [a for a in range(len(theta)) if m[a] != -2]
        assert inf["n_pairs"] == len(firsts)
        seconds = [m[a] for a in firsts if m[a] >= 0]
        assert sorted(firsts + seconds) == list(range(len(theta)))
        for a in firsts:
            if m[a] >= 0:
                assert m[a] > a
                assert abs(np.cos(theta[m[a]]) + np.cos(theta[a])) < 1e-12
                assert abs(np.sin(theta[m[a]]) - np.sin(theta[a])) < 1e-12
    assert inf["n_pairs"] == 40 + 25 - 25 + 2            # 25 mirrored, 0 with pi, pi/2 alone


def test_mirror_pairs_duplicates_and_wrapped_angles():
    """Repeated angles pair one to one in order of appearance; angles given outside
    [0, pi) pair by their cosine and sine (pi + a and -a mirror each other); a lone copy stays
    unpaired."""
    mv = _mirror_variant()
    th = np.array([0.5, 0.5, np.pi - 0.5, np.pi - 0.5, np.pi - 0.5, np.pi + 0.2, -0.2 + 0.0, 1.0])
    g = geo_for(configs.SliceConfig(n=34, n_theta=len(th), n_det=36, n_mask=3))
    g.theta = th
    m = ops.inspect(g, adj_variant=mv, tables=True)["adj_angles"][:, 9].astype(int)
    # pi + 0.2 has cos = -cos(0.2), sin = -sin(0.2) = sin(-0.2) with cos(-0.2) = cos(0.2)
    assert list(m) == [2, 3, -2, -2, -1, 6, -2, -1]


def test_adjoint_split_choice():
    """Adjoint angle split as the plan reports it: automatic (doubled while the launch has
    under 1024 blocks and each part keeps two angle chunks), explicit (clamped to the chunk
    count), rejected above 64; and the kernel's part ranges [g C / G, (g+1) C / G) cover the
    C chunks once each with no empty part."""
    big = geo_for(configs.SLICE_512)
    assert ops.inspect(big)["adj_splits"] == 1                     # 16x16 tiles: 1024 blocks
    info = ops.inspect(big, adj_variant=3)                         # 32x32 tiles: 256 blocks
    assert (info["n_tx"] * info["n_ty"], info["adj_splits"]) == (256, 4)
    small = geo_for(configs.SMALL_64)                              # 90 angles: 3 chunks of 32
    assert ops.inspect(small)["adj_splits"] == 1
    assert ops.inspect(small, adj_splits=2)["adj_splits"] == 2
    assert ops.inspect(small, adj_splits=64)["adj_splits"] == 3
    with pytest.raises(L.EitError) as e:
        ops.inspect(small, adj_splits=65)
    assert e.value.code == L.EIT_ERR_INVALID_ARG
    for C_ in range(1, 40):
        for G in range(1, C_ + 1):
            parts = [(g * C_ // G, (g + 1) * C_ // G) for g in range(G)]
            assert parts[0][0] == 0 and parts[-1][1] == C_
            assert all(a < b for a, b in parts)
            assert all(parts[i][1] == parts[i + 1][0] for i in range(G - 1))
