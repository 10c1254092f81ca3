"""Image-quality measures on the device (eq. 6 Fourier ring correlation with its smoothed
cutoff resolution, eq. 7 contrast-to-noise ratio) against the FP64 oracle (oracle/quality.py)
on the same images: random pairs, a noisy phantom pair, odd and even sizes."""
import numpy as np
import pytest
import torch

from oracle import quality as oq
from paper_2202_08627_amd import _lib as L
from paper_2202_08627_amd import configs, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_08627_amd import ops as _ops
    return _ops


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def _pair(n, seed):
    rng = np.random.default_rng(seed)
    base = synth.rasterize(synth.random_ellipses(n, 6, rng), n, 5)
    a = (base + 0.05 * rng.standard_normal((n, n))).astype(np.float32)
    b = (base + 0.05 * rng.standard_normal((n, n))).astype(np.float32)
    return a, b


@pytest.mark.parametrize("n,seed", [(64, 0), (65, 1), (220, 2), (2, 3), (7, 4)])
def test_frc_matches_oracle(ops, n, seed):
    a, b = _pair(n, seed)
    curve, smooth, res, rc = ops.frc(dev(a), dev(b))
    ref = oq.frc_curve(a.astype(np.float64), b.astype(np.float64))
    C = curve.cpu().numpy()
    print(f"FRC n={n}: max |curve - oracle| {np.abs(C - ref).max():.2e}", flush=True)
    assert np.abs(C - ref).max() < 1e-10
    assert np.abs(smooth.cpu().numpy() - oq.smooth(ref)).max() < 1e-10
    r_ref, rc_ref = oq.resolution(ref, n)
    assert rc == pytest.approx(rc_ref, rel=1e-9, abs=1e-12) and res == pytest.approx(r_ref, rel=1e-9)


def test_frc_of_an_image_with_itself_is_one(ops):
    a, _ = _pair(48, 5)
    curve, _, res, rc = ops.frc(dev(a), dev(a))
    assert np.allclose(curve.cpu().numpy(), 1.0, atol=1e-12)
    assert rc == 24.0 and res == 2.0      # never drops below the cutoff: the Nyquist limit


@pytest.mark.parametrize("n", [64, 220])
def test_cnr_matches_oracle(ops, n):
    a, _ = _pair(n, 7)
    for c1, c2, rho in [((0.0, 0.0), (10.0, -5.0), 6.0), ((-n / 2 + 1, 3.0), (4.5, 4.5), 3.3)]:
        v = ops.cnr(dev(a), c1, c2, rho)
        ref = oq.cnr(a.astype(np.float64), c1, c2, rho)
        assert v == pytest.approx(ref, rel=1e-12)


def test_quality_argument_errors(ops):
    a = dev(np.zeros((8, 8)))
    with pytest.raises(L.EitError) as e:
        ops.cnr(a, (100.0, 0.0), (0.0, 0.0), 1.0)
    assert e.value.code == L.EIT_ERR_INVALID_ARG
    assert L.lib().eit_frc_workspace_bytes(2048) == 0
