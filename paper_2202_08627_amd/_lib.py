"""ctypes binding of libeitomo.so (include/eitomo.h). Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeitomo.so")

EIT_OK = 0
EIT_ERR_INVALID_ARG = -1
EIT_ERR_SHAPE = -2
EIT_ERR_DEVICE = -3
EIT_ERR_NOMEM = -4
EIT_ERR_NONFINITE = -5
EIT_ERR_LINESEARCH = -6

EIT_OP_PROJECT = 1
EIT_OP_BACKPROJECT = 2
EIT_OP_COST_GRAD = 3
EIT_OP_RECONSTRUCT = 4
EIT_OP_SINGLE_SHOT = 5

ERROR_NAMES = {EIT_ERR_INVALID_ARG: "INVALID_ARG", EIT_ERR_SHAPE: "SHAPE", EIT_ERR_DEVICE: "DEVICE",
               EIT_ERR_NOMEM: "NOMEM", EIT_ERR_NONFINITE: "NONFINITE", EIT_ERR_LINESEARCH: "LINESEARCH"}


class EitError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"EIT_ERR_{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class Dims(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_theta", C.c_int32), ("n_det", C.c_int32),
                ("n_mask", C.c_int32), ("kappa", C.c_double)]


class Setup(C.Structure):
    _fields_ = [("theta", C.POINTER(C.c_double)), ("mask_pos", C.POINTER(C.c_double)),
                ("flat_amp", C.POINTER(C.c_double)), ("flat_ctr", C.POINTER(C.c_double)),
                ("flat_sigma", C.POINTER(C.c_double))]


class Tiling(C.Structure):
    _fields_ = [("proj_variant", C.c_int32), ("adj_variant", C.c_int32),
                ("adj_splits", C.c_int32)]


class Model(C.Structure):
    _fields_ = [("hmode", C.c_int32), ("fit_drift", C.c_int32), ("fit_ring", C.c_int32),
                ("n_table", C.c_int32), ("gamma", C.c_double), ("flat_table", C.POINTER(C.c_double)),
                ("table_u0", C.c_double), ("table_du", C.c_double), ("offset_scale", C.c_double),
                ("eq3_mask", C.c_int32), ("pad", C.c_int32)]


class Opts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("lbfgs_m", C.c_int32), ("max_ls_trials", C.c_int32),
                ("use_graph", C.c_int32), ("lam", C.c_double), ("mu_scale", C.c_double),
                ("delta_scale", C.c_double), ("tol_rel_step", C.c_double), ("c1", C.c_double),
                ("profile", C.c_int32), ("pad", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("evals", C.c_int32),
                ("launches", C.c_int32), ("cost", C.c_double), ("gnorm", C.c_double),
                ("phase_ms", C.c_double * 8), ("phase_steps", C.c_int32), ("pad", C.c_int32)]

PHASES = ["direction", "transpose", "project", "ic", "decide", "backproject", "update", "finalize"]


class PlanInfo(C.Structure):
    _fields_ = [(n, C.c_int32) for n in (
        "proj_variant", "adj_variant", "proj_a", "proj_w", "proj_r", "adj_tx", "adj_ty", "adj_ac",
        "n_groups", "n_dblk", "n_strips", "win_w", "win_pitch", "kwin", "kwin_pitch_limit",
        "n_tx", "n_ty", "adj_splits", "adj_mirror", "n_pairs")] + [("proj_lds_bytes", C.c_int64)]


class UNetLayer(C.Structure):
    _fields_ = [("kind", C.c_int32), ("cin", C.c_int32), ("cout", C.c_int32), ("pad", C.c_int32),
                ("w_off", C.c_int64), ("b_off", C.c_int64)]


_lib = None

VP = C.c_void_p
DP = C.POINTER(C.c_double)
IP = C.POINTER(C.c_int32)

_PROTOS = {
    "eit_plan_create": (C.c_int, [C.POINTER(Dims), C.POINTER(Setup), C.POINTER(Tiling), C.POINTER(VP)]),
    "eit_plan_destroy": (None, [VP]),
    "eit_plan_create_model": (C.c_int, [C.POINTER(Dims), C.POINTER(Setup), C.POINTER(Model),
                                        C.POINTER(Tiling), C.POINTER(VP)]),
    "eit_param_count": (C.c_int64, [VP]),
    "eit_workspace_bytes": (C.c_size_t, [VP, C.c_int32, C.c_int32]),
    "eit_project": (C.c_int, [VP, VP, VP, VP, C.c_size_t, VP]),
    "eit_backproject": (C.c_int, [VP, VP, VP, VP, C.c_size_t, VP]),
    "eit_cost_and_grad": (C.c_int, [VP, VP, VP, C.c_double, C.c_double, VP, VP, VP, C.c_size_t, VP]),
    "eit_reconstruct": (C.c_int, [VP, VP, C.POINTER(Opts), VP, VP, C.POINTER(Report), VP, C.c_size_t, VP]),
    "eit_batch_workspace_bytes": (C.c_size_t, [C.c_int32, C.POINTER(VP), C.c_int32]),
    "eit_reconstruct_batch": (C.c_int, [C.c_int32, C.POINTER(VP), C.POINTER(VP), C.POINTER(VP),
                                        C.POINTER(Opts), C.POINTER(Report), VP, C.c_size_t, VP]),
    "eit_cost_and_grad_noalloc": (C.c_int, [VP, VP, VP, C.c_double, C.c_double, VP, VP, VP]),
    "eit_single_shot": (C.c_int, [VP, VP, VP, VP, C.c_size_t, VP]),
    "eit_frc_workspace_bytes": (C.c_size_t, [C.c_int32]),
    "eit_frc": (C.c_int, [C.c_int32, VP, VP, VP, VP, VP, C.c_double, C.c_double, VP, C.c_size_t, VP]),
    "eit_cnr": (C.c_int, [C.c_int32, VP, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                          VP, VP]),
    "eit_last_error": (C.c_char_p, []),
    "eit_variant_info": (C.c_int, [C.c_int32, C.c_int32, IP, IP, IP, IP]),
    "eit_plan_inspect": (C.c_int, [C.POINTER(Dims), C.POINTER(Setup), C.POINTER(Tiling),
                                   C.POINTER(PlanInfo), DP, IP, IP, DP]),
    "eit_unet_create": (C.c_int, [C.c_int32, C.POINTER(VP)]),
    "eit_unet_destroy": (None, [VP]),
    "eit_unet_param_count": (C.c_int64, [VP]),
    "eit_unet_layers": (C.c_int, [VP, C.POINTER(UNetLayer), C.c_int32]),
    "eit_unet_workspace_bytes": (C.c_size_t, [VP, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "eit_unet_forward": (C.c_int, [VP, VP, VP, VP, C.c_int32, C.c_int32, C.c_int32, VP, C.c_size_t, VP]),
    "eit_unet_train_step": (C.c_int, [VP, VP, VP, VP, VP, C.c_int32, C.c_double, VP, VP, C.c_int32,
                                      C.c_int32, C.c_int32, VP, VP, C.c_size_t, VP]),
}


def lib():
    """Load the library (once). Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not built; run `python -m paper_2202_08627_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc: int):
    if rc != EIT_OK:
        msg = lib().eit_last_error()
        raise EitError(rc, msg.decode() if msg else "")
    return rc


def dptr(a):
    """ctypes double* into a contiguous float64 numpy array (or None)."""
    if a is None:
        return None
    return a.ctypes.data_as(DP)
