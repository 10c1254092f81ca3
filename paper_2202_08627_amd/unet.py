"""Binding of the warm-start U-Net entry points (eit_unet_*): torch tensors provide device
memory and the stream; forward, backward and Adam run in the library's BF16 MFMA kernels.

The network is not part of the paper's method. It maps the two-channel single-shot
reconstruction, each channel divided by its scale (mu_scale, delta_scale), to a start
point for the iterative minimisation of eq. 5 in the same scaled units."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L

KINDS = {0: "conv3x3", 1: "upconv2x2", 2: "head1x1"}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _check_img(t, name, B=None):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
            and t.dim() == 4 and t.shape[1] == 2):
        raise ValueError(f"{name} must be a contiguous CUDA float32 tensor [batch][2][h][w]")
    if B is not None and tuple(t.shape) != tuple(B):
        raise ValueError(f"{name} must have shape {tuple(B)}, got {tuple(t.shape)}")


class UNet:
    """Parameters (FP32, device) and Adam moments of one network."""

    def __init__(self, base: int = 32, params: np.ndarray | torch.Tensor | None = None,
                 device="cuda"):
        h = C.c_void_p()
        L.check(L.lib().eit_unet_create(int(base), C.byref(h)))
        self.handle = h
        self.base = int(base)
        self.n_params = int(L.lib().eit_unet_param_count(h))
        n = L.lib().eit_unet_layers(h, None, 0)
        arr = (L.UNetLayer * n)()
        L.lib().eit_unet_layers(h, arr, n)
        self.layers = [dict(kind=KINDS[a.kind], cin=a.cin, cout=a.cout, w_off=a.w_off, b_off=a.b_off)
                       for a in arr]
        self.device = torch.device(device)
        if params is None:
            self.params = torch.zeros(self.n_params, dtype=torch.float32, device=self.device)
        else:
            self.set_params(params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.step = 0
        self._ws = {}

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                L.lib().eit_unet_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def init_he(self, seed: int = 0, head_scale: float = 0.1):
        """He-normal weights (fan-in; the 2x2 transposed convolution counts one tap per
        output), zero biases, head weights scaled by head_scale so that the residual network
        starts close to the identity map."""
        rng = np.random.default_rng(seed)
        p = np.zeros(self.n_params, dtype=np.float32)
        for l in self.layers:
            taps = {"conv3x3": 9, "upconv2x2": 1, "head1x1": 1}[l["kind"]]
            std = np.sqrt(2.0 / (taps * l["cin"])) * (head_scale if l["kind"] == "head1x1" else 1.0)
            p[l["w_off"]:l["b_off"]] = rng.standard_normal(l["b_off"] - l["w_off"]) * std
        self.set_params(p)
        self.m.zero_()
        self.v.zero_()
        self.step = 0

    def set_params(self, p):
        t = torch.as_tensor(np.asarray(p, dtype=np.float32) if not isinstance(p, torch.Tensor) else p)
        if t.numel() != self.n_params:
            raise ValueError(f"{t.numel()} parameters given, {self.n_params} expected")
        self.params = t.reshape(-1).to(device=self.device, dtype=torch.float32).contiguous().clone()

    def workspace(self, batch, h, w, train):
        key = (batch, h, w, bool(train))
        if key not in self._ws:
            nb = int(L.lib().eit_unet_workspace_bytes(self.handle, batch, h, w, 1 if train else 0))
            if nb == 0:
                L.check(L.EIT_ERR_SHAPE)
            self._ws[key] = torch.empty(nb, dtype=torch.uint8, device=self.device)
        return self._ws[key]

    def forward(self, x, out=None):
        """x [batch][2][h][w] (scaled units) -> [batch][2][h][w]."""
        _check_img(x, "x")
        B, _, H, W = x.shape
        out = torch.empty_like(x) if out is None else out
        _check_img(out, "out", x.shape)
        ws = self.workspace(B, H, W, False)
        L.check(L.lib().eit_unet_forward(self.handle, _p(self.params), _p(x), _p(out), B, H, W,
                                         _p(ws), ws.numel(), _stream()))
        return out

    __call__ = forward

    def train_step(self, x, target, lr: float = 1e-3, apply: bool = True):
        """One MSE step on a batch; returns the loss as a 0-d float64 device tensor. With
        apply=False only self.grad is computed (parameters and moments untouched)."""
        _check_img(x, "x")
        _check_img(target, "target", x.shape)
        B, _, H, W = x.shape
        ws = self.workspace(B, H, W, True)
        loss = torch.empty((), dtype=torch.float64, device=self.device)
        step = self.step + 1 if apply else 0
        L.check(L.lib().eit_unet_train_step(self.handle, _p(self.params), _p(self.m), _p(self.v),
                                            _p(self.grad), step, float(lr), _p(x), _p(target), B, H, W,
                                            _p(loss), _p(ws), ws.numel(), _stream()))
        if apply:
            self.step = step
        return loss

    def state_dict(self):
        return {"base": self.base, "params": self.params.cpu().numpy(), "m": self.m.cpu().numpy(),
                "v": self.v.cpu().numpy(), "step": self.step}

    def load_state_dict(self, d):
        if int(d["base"]) != self.base:
            raise ValueError("base channel count differs")
        self.set_params(d["params"])
        self.m = torch.as_tensor(np.asarray(d["m"], np.float32), device=self.device).contiguous()
        self.v = torch.as_tensor(np.asarray(d["v"], np.float32), device=self.device).contiguous()
        self.grad = torch.zeros_like(self.params)
        self.step = int(d["step"])
