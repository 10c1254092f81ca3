"""Single-shot reconstruction (retrieval + Ram-Lak filtered backprojection) on the GPU against
the FP64 oracle on the same seeded data."""
import numpy as np
import pytest
import torch

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


def _oracle(c):
    cfg = c.cfg
    return oss.reconstruct(c.s_exp, c.theta, cfg.n, c.mask_pos, c.flat_amp, c.flat_ctr, c.flat_sigma,
                           cfg.kappa)


@pytest.mark.parametrize("cfg", [configs.SMALL_64, tiny_cfg(n=37, n_theta=13, n_det=45, n_mask=3),
                                 tiny_cfg(n=96, n_theta=120, n_mask=8)],
                         ids=["64x90", "37x13x45", "96x120"])
def test_single_shot_parity(ops, cfg):
    c = synth.make_case(cfg)
    plan = ops.Plan.from_case(c)
    x = plan.single_shot(torch.as_tensor(c.s_exp, device="cuda")).cpu().numpy().astype(np.float64)
    ref = _oracle(c)
    assert rel_l2(x[0], ref[0]) < 1e-4
    assert rel_l2(x[1], ref[1]) < 1e-4


def test_single_shot_large_slice(ops):
    cfg = configs.SLICE_512
    c = synth.make_case(cfg)
    plan = ops.Plan.from_case(c)
    x = plan.single_shot(torch.as_tensor(c.s_exp, device="cuda")).cpu().numpy().astype(np.float64)
    ref = _oracle(c)
    assert rel_l2(x[0], ref[0]) < 1e-4 and rel_l2(x[1], ref[1]) < 1e-4
    # and it is a sensible starting point: closer to the phantom than zero
    assert np.linalg.norm(x[0] - c.mu_true) < np.linalg.norm(c.mu_true)
