"""Host-side validation of the full-model, image-quality and no-allocation entry points, on
the CPU: every invalid option is rejected with the documented code before any device call
(on a machine without a GPU a valid plan request gets as far as the device lookup and
returns EIT_ERR_DEVICE instead)."""
import ctypes as C
import os

import numpy as np
import pytest

from paper_2202_08627_amd import _lib as L
from paper_2202_08627_amd import ops, synth

pytestmark = pytest.mark.skipif(not os.path.exists(L.LIB_PATH), reason="library not built")


def _geo(n=16, n_theta=12, n_mask=1):
    return ops.Geometry(n, n_theta, n, n_mask, 1.0, synth.angles(n_theta, 2.0),
                        np.array([0.3] * n_mask), np.ones(n), np.zeros(n), np.full(n, 0.3))


def _create(geo, model: ops.Model, gaussian=True):
    if not gaussian:
        geo.flat_amp = geo.flat_ctr = geo.flat_sigma = None
    dims, setup, keep = geo.c_args()
    m, tab = model.c_args(geo.n_det)
    til = L.Tiling(-1, -1, 0)
    h = C.c_void_p()
    rc = L.lib().eit_plan_create_model(C.byref(dims), C.byref(setup), C.byref(m), C.byref(til),
                                       C.byref(h))
    del keep, tab
    if rc == L.EIT_OK:
        L.lib().eit_plan_destroy(h)
    return rc


def _table(nd, q=33):
    u = -0.5 + np.arange(q) / (q - 1)
    return np.exp(-u[None, :] ** 2 / 0.18) * np.ones((nd, 1))


def _no_device_ok(rc):
    """A valid request: OK with a GPU, EIT_ERR_DEVICE without one."""
    return rc in (L.EIT_OK, L.EIT_ERR_DEVICE)


def test_valid_model_requests_pass_validation():
    g = _geo()
    assert _no_device_ok(_create(g, ops.Model(hmode=True, gamma=5.0, fit_drift=True, fit_ring=True)))
    assert _no_device_ok(_create(_geo(), ops.Model(hmode=True, flat_table=_table(16)), gaussian=False))
    assert _no_device_ok(_create(_geo(n_mask=3), ops.Model(fit_drift=True, eq3_mask=2)))


@pytest.mark.parametrize("kw,code", [
    (dict(hmode=True, gamma=0.0), L.EIT_ERR_INVALID_ARG),
    (dict(hmode=True, gamma=float("nan")), L.EIT_ERR_INVALID_ARG),
    (dict(offset_scale=-1.0), L.EIT_ERR_INVALID_ARG),
    (dict(eq3_mask=1), L.EIT_ERR_INVALID_ARG),
    (dict(flat_table=np.ones((16, 3))), L.EIT_ERR_SHAPE),
    (dict(flat_table=np.ones((16, 33)), table_du=0.0), L.EIT_ERR_INVALID_ARG),
    (dict(flat_table=np.ones((16, 33)), table_u0=float("inf")), L.EIT_ERR_INVALID_ARG),
], ids=["gamma0", "gamma-nan", "offset-scale", "eq3-mask", "table-short", "table-du", "table-u0"])
def test_invalid_model_options(kw, code):
    assert _create(_geo(), ops.Model(**kw)) == code


def test_table_values_must_be_finite_and_flats_present():
    t = _table(16)
    t[3, 7] = np.nan
    assert _create(_geo(), ops.Model(flat_table=t)) == L.EIT_ERR_INVALID_ARG
    # no Gaussian flats and no table: nothing to model the IC with
    assert _create(_geo(), ops.Model(hmode=True), gaussian=False) == L.EIT_ERR_INVALID_ARG


def test_model_and_quality_null_arguments():
    lib = L.lib()
    g = _geo()
    dims, setup, keep = g.c_args()
    h = C.c_void_p()
    assert lib.eit_plan_create_model(C.byref(dims), C.byref(setup), None, None, C.byref(h)) == L.EIT_ERR_INVALID_ARG
    assert lib.eit_param_count(None) == 0
    assert lib.eit_cost_and_grad_noalloc(None, None, None, 0.0, 0.0, None, None, None) == L.EIT_ERR_INVALID_ARG
    assert lib.eit_frc_workspace_bytes(1) == 0
    assert lib.eit_frc_workspace_bytes(2048) == 0
    assert lib.eit_frc_workspace_bytes(64) == 2 * 64 * 64 * 16 + 3 * 64 * 64 * 8
    assert lib.eit_frc(2048, None, None, None, None, None, 0.5, 1.0, None, 0, None) == L.EIT_ERR_SHAPE
    assert lib.eit_frc(64, None, None, None, None, None, 0.5, 1.0, None, 0, None) == L.EIT_ERR_INVALID_ARG
    assert lib.eit_cnr(64, None, 0.0, 0.0, 1.0, 1.0, 2.0, None, None) == L.EIT_ERR_INVALID_ARG
    # a disc with no pixel centre is refused on the host (the pointers are never used)
    buf = (C.c_float * 4)()
    out = (C.c_double * 1)()
    assert lib.eit_cnr(2, C.cast(buf, C.c_void_p), 50.0, 0.0, 0.0, 0.0, 1.0,
                       C.cast(out, C.c_void_p), None) == L.EIT_ERR_INVALID_ARG
    del keep
