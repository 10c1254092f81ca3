"""Pins for the oracle's image-quality measures (FRC, eq. 6; CNR, eq. 7): identities, the
statistics of independent noise, the closed form of signal plus noise, and CNR on images
whose disc statistics are exact by construction."""
import numpy as np
import pytest

from oracle import quality as q


def test_frc_of_an_image_with_itself_and_its_negative():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((48, 48))
    c = q.frc_curve(a, a)
    assert np.allclose(c, 1.0, rtol=0, atol=1e-12)
    assert np.allclose(q.frc_curve(a, -a), -1.0, rtol=0, atol=1e-12)
    # invariant to positive scalings of either image
    assert np.allclose(q.frc_curve(3.0 * a, 0.25 * a), 1.0, atol=1e-12)


def test_frc_of_independent_noise_is_near_zero():
    """Two independent white-noise images: each ring's FRC has mean 0 and standard deviation
    about 1/sqrt(pixels in the ring); all rings but the first few must stay within 4 of those."""
    rng = np.random.default_rng(1)
    n = 128
    a, b = rng.standard_normal((2, n, n))
    c = q.frc_curve(a, b)
    k = np.fft.fftfreq(n) * n
    r = np.rint(np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)).astype(int)
    counts = np.array([np.sum(r == i) for i in range(n // 2 + 1)])
    assert np.all(np.abs(c[4:]) < 4.0 / np.sqrt(counts[4:]))


def test_frc_of_signal_plus_noise_matches_closed_form():
    """Image 1 = s + n1, image 2 = s + n2 with white s (variance S) and independent white noise
    (variance N): FRC = S / (S + N) in expectation at every ring."""
    rng = np.random.default_rng(2)
    n = 256
    S, N = 1.0, 0.5
    s = np.sqrt(S) * rng.standard_normal((n, n))
    a = s + np.sqrt(N) * rng.standard_normal((n, n))
    b = s + np.sqrt(N) * rng.standard_normal((n, n))
    c = q.frc_curve(a, b)
    assert abs(np.mean(c[10:]) - S / (S + N)) < 0.01


def test_resolution_crossing():
    """A curve falling linearly from 1 at ring 0 to 0 at ring 40 crosses 0.5 at ring 20 (the
    smoothing of a straight line changes it only at the ends): resolution N / 20."""
    n = 100
    c = np.clip(1.0 - np.arange(n // 2 + 1) / 40.0, 0.0, None)
    res, rc = q.resolution(c, n)
    assert rc == pytest.approx(20.0, abs=1e-9) and res == pytest.approx(5.0, abs=1e-9)


def test_cnr_on_exact_disc_statistics():
    """Discs whose pixels alternate a +- s (exact mean a, population std s whenever the disc has
    an even number of pixels, alternating along the raster order): CNR = |a1 - a2| /
    sqrt(s1^2 + s2^2)."""
    n = 64
    img = np.zeros((n, n))
    spec = [((-12.0, 0.0), 2.0, 0.3), ((13.0, 5.0), 1.2, 0.4)]
    for (x0, y0), a, s in spec:
        m = q.disc_mask(n, x0, y0, 8.0)
        k = int(m.sum())
        assert k % 2 == 0
        img[m] = a + s * np.where(np.arange(k) % 2 == 0, 1.0, -1.0)
    val = q.cnr(img, spec[0][0], spec[1][0], 8.0)
    assert val == pytest.approx(0.8 / np.sqrt(0.3 ** 2 + 0.4 ** 2), rel=1e-12)
