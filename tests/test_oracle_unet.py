"""Pins of the warm-start U-Net oracle (oracle/unet_ref.py) against brute force, finite
differences, closed forms and structural identities."""
import numpy as np
import torch
import torch.nn.functional as F

from oracle import unet_ref as U


def _params(base, seed=0, head_scale=1.0):
    p = U.init_params(base, seed)
    lay, _ = U.offsets(base)
    rng = np.random.default_rng(seed + 1)
    for kind, cin, cout, w, b in lay:
        p[b:b + cout] = 0.05 * rng.standard_normal(cout)      # non-zero biases
        if kind == U.HEAD:
            p[w:b] *= head_scale
    return p


def test_param_count_matches_layer_sizes():
    # base 32: the 4-level network has ~1.9 M parameters
    _, n = U.offsets(32)
    expect = 0
    for kind, cin, cout in U.layer_defs(32):
        expect += cout * {U.CONV: 9, U.UP: 4, U.HEAD: 1}[kind] * cin + cout
    assert n == expect
    assert 1.8e6 < n < 2.0e6


def test_conv_layout_against_loops():
    rng = np.random.default_rng(3)
    ci, co, H, W = 3, 4, 5, 6
    x = rng.standard_normal((ci, H, W))
    Wf = rng.standard_normal(co * 9 * ci)
    b = rng.standard_normal(co)
    ref = U.conv3x3_loops(x, Wf.reshape(co, 9, ci), b)
    Wt = torch.tensor(Wf).reshape(co, 3, 3, ci).permute(0, 3, 1, 2)
    got = F.conv2d(torch.tensor(x)[None], Wt, torch.tensor(b), padding=1)[0].numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
    # the oracle's own weight views use the same permutation
    base = 8
    p = _params(base)
    lay, _ = U.offsets(base)
    kind, cin, cout, w0, b0 = lay[1]
    Wv = U.torch_weights(torch.tensor(p), base)[1][1]
    np.testing.assert_array_equal(Wv.numpy(), torch.tensor(p[w0:b0]).reshape(cout, 3, 3, cin).permute(0, 3, 1, 2).numpy())


def test_upconv_layout_against_loops():
    rng = np.random.default_rng(4)
    ci, co, H, W = 3, 2, 3, 4
    x = rng.standard_normal((ci, H, W))
    Wf = rng.standard_normal(co * 4 * ci)
    b = rng.standard_normal(co)
    ref = U.upconv_loops(x, Wf.reshape(co, 4, ci), b)
    Wt = torch.tensor(Wf).reshape(co, 2, 2, ci).permute(3, 0, 1, 2)
    got = F.conv_transpose2d(torch.tensor(x)[None], Wt, torch.tensor(b), stride=2)[0].numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_zero_head_is_identity():
    base = 8
    p = _params(base, head_scale=0.0)
    lay, _ = U.offsets(base)
    _, _, cout, _, b = lay[-1]
    p[b:b + cout] = 0.0
    x = np.random.default_rng(0).standard_normal((2, 2, 16, 16))
    for emul in (False, True):
        np.testing.assert_array_equal(U.predict(p, x, base, emul), x)


def test_gradient_matches_finite_differences():
    """Central differences of the FP64 loss: within one ReLU/max-pool region the loss is
    quadratic in any single parameter, so the central difference is exact up to rounding."""
    base = 8
    p = _params(base, seed=5, head_scale=10.0)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((2, 2, 16, 16))
    t = x + 0.3 * rng.standard_normal(x.shape)
    _, g = U.loss_and_grad(p, x, t, base)
    lay, _ = U.offsets(base)
    idx = []
    for kind, cin, cout, w, b in lay:          # two weights and one bias from every layer
        idx += list(rng.integers(w, b, 2)) + [int(rng.integers(b, b + cout))]
    h = 1e-5
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (U.loss_and_grad(pp, x, t, base)[0] - U.loss_and_grad(pm, x, t, base)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g).max(), 1e-12) + 1e-5 * abs(g[i]), (i, fd, g[i])


def test_padded_input_channels_get_no_gradient():
    base = 8
    p = _params(base)
    x = np.random.default_rng(2).standard_normal((1, 2, 16, 16))
    _, g = U.loss_and_grad(p, x, x * 0.5, base)
    kind, cin, cout, w, b = U.offsets(base)[0][0]
    W = g[w:b].reshape(cout, 9, cin)
    assert np.all(W[:, :, 2:] == 0.0) and np.any(W[:, :, :2] != 0.0)


def test_batch_items_are_independent():
    base = 8
    p = _params(base, head_scale=5.0)
    x = np.random.default_rng(7).standard_normal((3, 2, 16, 16))
    full = U.predict(p, x, base)
    for i in range(3):
        np.testing.assert_allclose(U.predict(p, x[i:i + 1], base)[0], full[i], rtol=1e-13, atol=1e-13)


def test_transpose_symmetry():
    """Transposing the image and every 3x3 / 2x2 kernel spatially transposes the output:
    pins the (ky, kx) and (dy, dx) tap order."""
    base = 8
    p = _params(base, head_scale=5.0)
    q = p.copy()
    for kind, cin, cout, w, b in U.offsets(base)[0]:
        if kind == U.CONV:
            q[w:b] = p[w:b].reshape(cout, 3, 3, cin).transpose(0, 2, 1, 3).ravel()
        elif kind == U.UP:
            q[w:b] = p[w:b].reshape(cout, 2, 2, cin).transpose(0, 2, 1, 3).ravel()
    x = np.random.default_rng(8).standard_normal((1, 2, 16, 24))
    a = U.predict(p, x, base)
    bt = U.predict(q, x.transpose(0, 1, 3, 2).copy(), base)
    np.testing.assert_allclose(bt, a.transpose(0, 1, 3, 2), rtol=1e-12, atol=1e-12)


def test_bf16_rounding_is_nearest_even():
    one = torch.tensor([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 1.0 + 2.0 ** -9],
                       dtype=torch.float64)
    np.testing.assert_array_equal(U.bf16(one).numpy(), [1.0, 1.0 + 2.0 ** -6, -1.0, 1.0])


def test_bf16_emulation_is_close_but_not_exact():
    base = 8
    p = _params(base, head_scale=5.0)
    x = np.random.default_rng(9).standard_normal((1, 2, 16, 16))
    a, b = U.predict(p, x, base, False) - x, U.predict(p, x, base, True) - x
    rel = np.linalg.norm(a - b) / np.linalg.norm(a)
    assert 1e-5 < rel < 5e-2


def test_maxpool_gradient_goes_to_first_maximum():
    """Tie rule the device follows: the gradient of a 2x2 window goes to its first maximum
    in row-major order."""
    x = torch.tensor([[[[1.0, 2.0], [2.0, 0.5]]]], dtype=torch.float64, requires_grad=True)
    F.max_pool2d(x, 2).sum().backward()
    np.testing.assert_array_equal(x.grad.numpy()[0, 0], [[0, 1], [0, 0]])


def test_adam_closed_form():
    # first step: m = (1-b1) g, v = (1-b2) g^2; bias-corrected update = lr * g / (|g| + eps)
    p, m, v = U.adam(np.array([1.0, -2.0]), np.zeros(2), np.zeros(2), np.array([0.5, -4.0]), 1, 0.01)
    np.testing.assert_allclose(p, [1.0 - 0.01 * 0.5 / (0.5 + 1e-8), -2.0 + 0.01 * 4.0 / (4.0 + 1e-8)], rtol=1e-14)
    np.testing.assert_allclose(m, [0.05, -0.4])
    np.testing.assert_allclose(v, [0.00025, 0.016])
