"""bench.py's command-line contract that needs no GPU: more than one GPU is refused with a
message and exit status 2 before any device work, the unet FLOP count matches the layer table,
and the CPU-baseline child prints one JSON record."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2", "--steps", "1", "--warmup", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout.strip() == ""


def test_world_size_above_one_is_refused():
    env = dict(os.environ, WORLD_SIZE="4")
    r = subprocess.run([sys.executable, BENCH], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 2


def test_unet_flops_match_the_layer_table():
    """Forward FLOPs of the 4-level, 32-channel network at 256^2: two 3x3 convolutions per
    level at that level's resolution (encoder, bottleneck, decoder), three 2x2 transposed
    convolutions and the 1x1 head, counted by hand from the architecture."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_2202_08627_amd.unet import UNet
    net = UNet(32, device="cpu")          # the layer table only; no device memory
    h = 256
    px = lambda r: float(r) * r
    conv = lambda r, ci, co: 2.0 * px(r) * 9 * ci * co
    up = lambda r, ci, co: 2.0 * px(r) * 4 * ci * co           # at the coarser input's size
    fwd = (conv(h, 8, 32) + conv(h, 32, 32)
           + conv(h // 2, 32, 64) + conv(h // 2, 64, 64)
           + conv(h // 4, 64, 128) + conv(h // 4, 128, 128)
           + conv(h // 8, 128, 256) + conv(h // 8, 256, 256)
           + up(h // 8, 256, 128) + conv(h // 4, 256, 128) + conv(h // 4, 128, 128)
           + up(h // 4, 128, 64) + conv(h // 2, 128, 64) + conv(h // 2, 64, 64)
           + up(h // 2, 64, 32) + conv(h, 64, 32) + conv(h, 32, 32)
           + 2.0 * px(h) * 32 * 2)
    assert bench.unet_flops(net, h, h, train=False) == pytest.approx(fwd, rel=1e-12)
