"""Shared test helpers: tiny seeded problems and error measures (no method arithmetic)."""
import dataclasses

import numpy as np

from paper_2202_08627_amd import configs, synth


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def tiny_cfg(n=16, n_theta=24, n_mask=5, n_ellipses=3, jitter=0.05, **kw):
    return dataclasses.replace(configs.SMALL_64, n=n, n_theta=n_theta, n_det=kw.pop("n_det", n),
                               n_mask=n_mask, n_ellipses=n_ellipses, sigma_jitter=jitter,
                               mu_scale=configs.mu_range_for(n), **kw)


def geometry(case, oracle_model):
    cfg = case.cfg
    return oracle_model.Geometry(cfg.n, case.theta, cfg.n_det, case.mask_pos, case.flat_amp,
                                 case.flat_ctr, case.flat_sigma, cfg.kappa)
