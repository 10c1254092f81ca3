"""Oracle: the warm-start U-Net (forward, MSE loss, gradient, Adam), on the CPU.

TEST INFRASTRUCTURE ONLY (plain PyTorch CPU ops in FP64; shares no code with the HIP path).

The network is not part of the paper: it is a learned warm start for the iterative
minimisation of eq. 5, mapping the two-channel single-shot reconstruction (mu, delta,
normalised by the caller) to a starting point. Architecture:
    level l = 1..4 has c_l = base * 2^(l-1) channels;
    encoder: two 3x3 convolutions (zero padding) + ReLU per level, 2x2 max pooling between levels;
    decoder: 2x2 stride-2 transposed convolution (c_{l+1} -> c_l), concatenated as [up, skip],
             then two 3x3 convolutions + ReLU;
    head: 1x1 convolution to 2 channels, added to the input (residual).
The input's 2 channels are zero-padded to 8 before the first convolution (the device layout
groups channels by 8); the padded channels' weights receive gradients but never matter.

Parameter vector layout (FP32 on the device, FP64 here), layer by layer, weights then bias:
    3x3 conv   W[cout][ky*3 + kx][cin]
    2x2 up     W[cout][dy*2 + dx][cin]     output pixel (2y + dy, 2x + dx)
    1x1 head   W[2][cin]

BF16 emulation (bf16=True): the device multiplies BF16 operands and accumulates in FP32.
The same values are produced here by rounding, to BF16 with round-to-nearest-even, exactly
the tensors the device stores in BF16: the packed input, the conv and up-conv weights
(straight-through: the gradient goes to the FP32 master weight), every conv / up-conv /
pool output, and the gradient arriving at each of those tensors. The gradient reaching a
skip tensor through the concatenation is rounded on its own before the pooled path's
gradient is added to it and the sum is rounded again (the device stores the first in BF16
and accumulates the second onto it). The head, the loss and all weight gradients stay in
full precision. With bf16=False this is a plain FP64 U-Net. dtype=float32 runs the same
emulation with FP32 accumulation: the gap between the two measures how far any other
accumulation order may drift after BF16 rounding.

Pins (tests/test_oracle_unet.py): autograd gradient vs central finite differences of the
FP64 loss; brute-force loop convolution and transposed convolution with the documented
weight layouts; zero head => output equals input; spatial transposition of image and
kernels transposes the output (tap order); batch items independent; padded input channels
get zero gradient; max-pool gradient to the first maximum; BF16 rounding to nearest even;
the Adam update against its closed form.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

IN_CH = 8          # input channels after zero padding

CONV, UP, HEAD = 0, 1, 2
NAMES = ["a1", "b1", "a2", "b2", "a3", "b3", "a4", "b4", "up3", "d3a", "d3b",
         "up2", "d2a", "d2b", "up1", "d1a", "d1b", "head"]


def layer_defs(base: int):
    """(kind, cin, cout) in parameter order."""
    c = base
    return [(CONV, IN_CH, c), (CONV, c, c), (CONV, c, 2 * c), (CONV, 2 * c, 2 * c),
            (CONV, 2 * c, 4 * c), (CONV, 4 * c, 4 * c), (CONV, 4 * c, 8 * c), (CONV, 8 * c, 8 * c),
            (UP, 8 * c, 4 * c), (CONV, 8 * c, 4 * c), (CONV, 4 * c, 4 * c),
            (UP, 4 * c, 2 * c), (CONV, 4 * c, 2 * c), (CONV, 2 * c, 2 * c),
            (UP, 2 * c, c), (CONV, 2 * c, c), (CONV, c, c),
            (HEAD, c, 2)]


def layer_sizes(kind: int, cin: int, cout: int) -> int:
    taps = {CONV: 9, UP: 4, HEAD: 1}[kind]
    return cout * taps * cin


def offsets(base: int):
    """[(kind, cin, cout, w_off, b_off)] and the total parameter count."""
    out, off = [], 0
    for kind, cin, cout in layer_defs(base):
        nw = layer_sizes(kind, cin, cout)
        out.append((kind, cin, cout, off, off + nw))
        off += nw + cout
    return out, off


def init_params(base: int, seed: int = 0) -> np.ndarray:
    """He-normal weights (fan-in), zero biases; head weights scaled down so that the
    untrained network starts near the identity map."""
    rng = np.random.default_rng(seed)
    lay, n = offsets(base)
    p = np.zeros(n, dtype=np.float64)
    for kind, cin, cout, w, b in lay:
        nw = b - w
        fan_in = cin * {CONV: 9, UP: 1, HEAD: 1}[kind]
        std = np.sqrt(2.0 / fan_in) * (0.1 if kind == HEAD else 1.0)
        p[w:b] = rng.standard_normal(nw) * std
    return p


# --------------------------------------------------------------------------- BF16 rounding
def bf16(t: torch.Tensor) -> torch.Tensor:
    """Round to the nearest BF16 value (ties to even), returned in t's dtype."""
    return t.to(torch.bfloat16).to(t.dtype)


class _RoundBoth(torch.autograd.Function):
    """Value rounded to BF16 on the way forward, gradient rounded on the way back."""

    @staticmethod
    def forward(ctx, x):
        return bf16(x)

    @staticmethod
    def backward(ctx, g):
        return bf16(g)


def _ste(w: torch.Tensor) -> torch.Tensor:
    """BF16 value with the identity gradient (a BF16 copy of an FP32 master weight)."""
    return w + (bf16(w) - w).detach()


# --------------------------------------------------------------------------- layers
def torch_weights(params: torch.Tensor, base: int):
    """Per layer (weight in PyTorch's layout, bias) as views of the flat parameter tensor."""
    lay, _ = offsets(base)
    out = []
    for kind, cin, cout, w, b in lay:
        W = params[w:b]
        if kind == CONV:     # [co][ky*3+kx][ci] -> conv2d weight [co][ci][ky][kx]
            Wt = W.reshape(cout, 3, 3, cin).permute(0, 3, 1, 2)
        elif kind == UP:     # [co][dy*2+dx][ci] -> conv_transpose2d weight [ci][co][dy][dx]
            Wt = W.reshape(cout, 2, 2, cin).permute(3, 0, 1, 2)
        else:                # [o][ci] -> 1x1 conv weight [o][ci][1][1]
            Wt = W.reshape(cout, cin, 1, 1)
        out.append((kind, Wt, params[b:b + cout]))
    return out


def forward(params: torch.Tensor, x: torch.Tensor, base: int, bf16_emul: bool = False) -> torch.Tensor:
    """x: [B][2][H][W] (H, W multiples of 8) -> [B][2][H][W]."""
    q = _RoundBoth.apply if bf16_emul else (lambda t: t)
    qw = _ste if bf16_emul else (lambda t: t)
    layers = torch_weights(params, base)
    it = iter(layers)

    def conv(h):
        _, W, b = next(it)
        return q(F.relu(F.conv2d(h, qw(W), b, padding=1)))

    def up(h):
        _, W, b = next(it)
        return q(F.conv_transpose2d(h, qw(W), b, stride=2))

    B, _, H, Wd = x.shape
    h = torch.cat([x, torch.zeros(B, IN_CH - 2, H, Wd, dtype=x.dtype)], dim=1)
    h = q(h)
    skips = []
    for lvl in range(3):
        h = conv(conv(h))
        skips.append(q(h))          # forward: no-op; backward: rounds the concat-path gradient
        h = q(F.max_pool2d(h, 2))
    h = conv(conv(h))
    for lvl in range(3):
        u = up(h)
        h = torch.cat([u, skips.pop()], dim=1)
        h = conv(conv(h))
    _, Wh, bh = next(it)
    return x + F.conv2d(h, Wh, bh)


def loss_and_grad(params: np.ndarray, x: np.ndarray, target: np.ndarray, base: int,
                  bf16_emul: bool = False, dtype=torch.float64):
    """Mean squared error over all outputs and its gradient with respect to params."""
    p = torch.tensor(np.asarray(params, dtype=np.float64), dtype=dtype, requires_grad=True)
    xt = torch.tensor(np.asarray(x, dtype=np.float64), dtype=dtype)
    tt = torch.tensor(np.asarray(target, dtype=np.float64), dtype=dtype)
    out = forward(p, xt, base, bf16_emul)
    loss = torch.mean((out - tt) ** 2)
    loss.backward()
    return float(loss.detach()), p.grad.double().numpy().copy()


def predict(params: np.ndarray, x: np.ndarray, base: int, bf16_emul: bool = False,
            dtype=torch.float64) -> np.ndarray:
    with torch.no_grad():
        p = torch.tensor(np.asarray(params, dtype=np.float64), dtype=dtype)
        xt = torch.tensor(np.asarray(x, dtype=np.float64), dtype=dtype)
        return forward(p, xt, base, bf16_emul).double().numpy()


def adam(p, m, v, g, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update with bias correction for the given (1-based) step; returns new p, m, v."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# --------------------------------------------------------------------------- brute force (pins)
def conv3x3_loops(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x [ci][H][W], W [co][9][ci] (tap = ky*3 + kx), zero padding; no ReLU."""
    ci, H, Wd = x.shape
    co = W.shape[0]
    y = np.zeros((co, H, Wd))
    for o in range(co):
        for yy in range(H):
            for xx in range(Wd):
                s = b[o]
                for ky in range(3):
                    for kx in range(3):
                        sy, sx = yy + ky - 1, xx + kx - 1
                        if 0 <= sy < H and 0 <= sx < Wd:
                            s += float(np.dot(W[o, ky * 3 + kx], x[:, sy, sx]))
                y[o, yy, xx] = s
    return y


def upconv_loops(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x [ci][H][W], W [co][4][ci] (d = dy*2 + dx) -> [co][2H][2W]."""
    ci, H, Wd = x.shape
    co = W.shape[0]
    y = np.zeros((co, 2 * H, 2 * Wd))
    for o in range(co):
        for yy in range(H):
            for xx in range(Wd):
                for dy in range(2):
                    for dx in range(2):
                        y[o, 2 * yy + dy, 2 * xx + dx] = b[o] + float(np.dot(W[o, dy * 2 + dx], x[:, yy, xx]))
    return y
