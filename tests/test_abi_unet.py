"""Host-only checks of the network's C-ABI (no device needed): layer table and parameter
count against the oracle's documented layout, workspace sizing, argument validation."""
import ctypes as C

from oracle import unet_ref as U
from paper_2202_08627_amd import _lib as L


def test_abi_layer_table_matches_oracle_layout():
    lib = L.lib()
    for base in (8, 16, 32):
        h = C.c_void_p()
        L.check(lib.eit_unet_create(base, C.byref(h)))
        try:
            lay, n = U.offsets(base)
            assert lib.eit_unet_param_count(h) == n
            cnt = lib.eit_unet_layers(h, None, 0)
            arr = (L.UNetLayer * cnt)()
            assert lib.eit_unet_layers(h, arr, cnt) == len(lay)
            for a, (kind, cin, cout, w, b) in zip(arr, lay):
                assert (a.kind, a.cin, a.cout, a.w_off, a.b_off) == (kind, cin, cout, w, b)
            # workspace: 0 for invalid sizes, training needs more than inference
            assert lib.eit_unet_workspace_bytes(h, 1, 12, 16, 0) == 0
            assert lib.eit_unet_workspace_bytes(h, 0, 16, 16, 0) == 0
            wi = lib.eit_unet_workspace_bytes(h, 2, 64, 64, 0)
            wt = lib.eit_unet_workspace_bytes(h, 2, 64, 64, 1)
            assert 0 < wi < wt
        finally:
            lib.eit_unet_destroy(h)


def test_abi_rejects_bad_arguments():
    lib = L.lib()
    h = C.c_void_p()
    assert lib.eit_unet_create(12, C.byref(h)) == L.EIT_ERR_INVALID_ARG
    assert lib.eit_unet_create(4, C.byref(h)) == L.EIT_ERR_INVALID_ARG
    L.check(lib.eit_unet_create(8, C.byref(h)))
    try:
        dummy = C.c_void_p(256)          # never dereferenced: validation fails first
        assert lib.eit_unet_forward(h, dummy, dummy, dummy, 1, 20, 16, dummy, 1 << 30, None) == L.EIT_ERR_SHAPE
        assert lib.eit_unet_forward(h, None, dummy, dummy, 1, 16, 16, dummy, 1 << 30, None) == L.EIT_ERR_INVALID_ARG
        assert lib.eit_unet_forward(h, dummy, dummy, dummy, 1, 16, 16, dummy, 16, None) == L.EIT_ERR_NOMEM
        loss = C.c_void_p(512)
        assert lib.eit_unet_train_step(h, dummy, None, None, dummy, 1, 1e-3, dummy, dummy, 1, 16, 16,
                                       loss, dummy, 1 << 30, None) == L.EIT_ERR_INVALID_ARG
        assert lib.eit_unet_train_step(h, dummy, dummy, dummy, dummy, 1, float("nan"), dummy, dummy, 1,
                                       16, 16, loss, dummy, 1 << 30, None) == L.EIT_ERR_INVALID_ARG
    finally:
        lib.eit_unet_destroy(h)
