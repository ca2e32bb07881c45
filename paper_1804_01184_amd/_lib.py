"""ctypes binding of libfwi2d.so (include/fwi2d.h).

Argument marshalling only: every array operation runs in the HIP library.
There is no fallback: if the library is missing or a call fails, an
exception is raised.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfwi2d.so")

FWI_OK = 0
STATUS = {0: "FWI_OK", -1: "FWI_EINVAL", -2: "FWI_ENOMEM", -3: "FWI_EDEVICE",
          -4: "FWI_EUNSTABLE", -5: "FWI_ENONFINITE", -6: "FWI_ESTATE", -7: "FWI_EWORKSPACE"}

FWI_K_RHO, FWI_VP_RHO, FWI_IP_RHO, FWI_VP_IP, FWI_INVK_INVRHO = 0, 1, 2, 3, 4
FWI_EXEC_BATCHED, FWI_EXEC_PLAIN = 0, 1
FWI_OP_FORWARD, FWI_OP_MISFIT, FWI_OP_GRADIENT = 0, 1, 2

# exported symbols declared in include/fwi2d.h
SYMBOLS = ["fwi_plan_create", "fwi_plan_destroy", "fwi_plan_get_info", "fwi_workspace_bytes",
           "fwi_forward", "fwi_misfit", "fwi_misfit_noalloc", "fwi_misfit_weighted", "fwi_gradient", "fwi_adjoint", "fwi_forward_keep",
           "fwi_adjoint_kept", "fwi_model_convert",
           "fwi_chain_rule", "fwi_contrast_scale", "fwi_descent_direction", "fwi_descent_apply",
           "fwi_descent_norms", "fwi_born_green", "fwi_born_workspace_bytes", "fwi_born_data",
           "fwi_born_misfit", "fwi_born_gradient", "fwi_born_contrasts", "fwi_born_chain",
           "fwi_born_hessian", "fwi_timing_enable", "fwi_timing_read",
           "fwi_sync", "fwi_status_str", "fwi_last_error"]

KERNEL_CLASSES = ["fwd_step", "adj_step", "plain_vel", "plain_pres", "plain_adj_a",
                  "plain_adj_b", "sample", "inject", "other", "fwd_pair", "adj_pair"]


class FwiGrid(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int32), ("nx", ctypes.c_int32), ("npml", ctypes.c_int32),
                ("nt", ctypes.c_int32), ("dz", ctypes.c_double), ("dx", ctypes.c_double),
                ("dt", ctypes.c_double), ("vmax", ctypes.c_double), ("pml_r", ctypes.c_double)]


class FwiAcq(ctypes.Structure):
    _fields_ = [("nshots", ctypes.c_int32), ("nrec", ctypes.c_int32),
                ("wavelet_per_shot", ctypes.c_int32),
                ("src_xz", ctypes.POINTER(ctypes.c_double)),
                ("rec_xz", ctypes.POINTER(ctypes.c_double))]


class FwiExec(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("ckpt_every", ctypes.c_int32),
                ("band_rows", ctypes.c_int32), ("shots_per_group", ctypes.c_int32),
                ("lane_cols", ctypes.c_int32), ("two_step", ctypes.c_int32),
                ("two_step_band_rows", ctypes.c_int32),
                ("two_step_shots_per_group", ctypes.c_int32),
                ("two_step_lane_cols", ctypes.c_int32),
                ("adj_two_step", ctypes.c_int32),
                ("adj_two_step_band_rows", ctypes.c_int32),
                ("adj_two_step_lane_cols", ctypes.c_int32)]


class FwiPlanInfo(ctypes.Structure):
    _fields_ = [("Nz", ctypes.c_int32), ("Nx", ctypes.c_int32), ("ckpt_every", ctypes.c_int32),
                ("segments", ctypes.c_int32), ("band_rows", ctypes.c_int32),
                ("shots_per_group", ctypes.c_int32), ("lane_cols", ctypes.c_int32),
                ("shot_groups", ctypes.c_int32), ("two_step", ctypes.c_int32),
                ("two_step_band_rows", ctypes.c_int32),
                ("two_step_shots_per_group", ctypes.c_int32),
                ("two_step_lane_cols", ctypes.c_int32),
                ("adj_two_step", ctypes.c_int32),
                ("adj_two_step_band_rows", ctypes.c_int32),
                ("adj_two_step_lane_cols", ctypes.c_int32),
                ("mode", ctypes.c_int32),
                ("device", ctypes.c_int32), ("pml_cells", ctypes.c_int64),
                ("cfl", ctypes.c_double)]


class FwiTiming(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 11), ("ms", ctypes.c_double * 11)]


class FwiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Loads libfwi2d.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with "
                          "`python -m paper_1804_01184_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, fp, i32, i64, st = (ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                            ctypes.c_int)
    sz = ctypes.c_size_t
    L.fwi_plan_create.argtypes = [ctypes.POINTER(FwiGrid), ctypes.POINTER(FwiAcq),
                                  ctypes.POINTER(FwiExec), ctypes.POINTER(ctypes.c_void_p)]
    L.fwi_plan_create.restype = st
    L.fwi_plan_destroy.argtypes = [vp]
    L.fwi_plan_destroy.restype = None
    L.fwi_plan_get_info.argtypes = [vp, ctypes.POINTER(FwiPlanInfo)]
    L.fwi_plan_get_info.restype = st
    L.fwi_workspace_bytes.argtypes = [vp, i32]
    L.fwi_workspace_bytes.restype = sz
    L.fwi_forward.argtypes = [vp, i32, fp, fp, fp, fp, vp, sz, vp]
    L.fwi_forward.restype = st
    L.fwi_misfit.argtypes = [vp, fp, fp, fp, fp, vp, sz, vp]
    L.fwi_misfit.restype = st
    L.fwi_misfit_noalloc.argtypes = [vp, fp, fp, fp, fp, vp]
    L.fwi_misfit_noalloc.restype = st
    L.fwi_misfit_weighted.argtypes = [vp, fp, fp, fp, fp, fp, vp, sz, vp]
    L.fwi_misfit_weighted.restype = st
    L.fwi_gradient.argtypes = [vp, i32, fp, fp, fp, fp, fp, fp, fp, fp, vp, sz, vp]
    L.fwi_gradient.restype = st
    L.fwi_adjoint.argtypes = [vp, i32, fp, fp, fp, fp, fp, fp, vp, sz, vp]
    L.fwi_adjoint.restype = st
    L.fwi_forward_keep.argtypes = [vp, i32, fp, fp, fp, fp, vp, sz, vp]
    L.fwi_forward_keep.restype = st
    L.fwi_adjoint_kept.argtypes = [vp, i32, fp, fp, fp, fp, fp, fp, vp, sz, vp]
    L.fwi_adjoint_kept.restype = st
    L.fwi_model_convert.argtypes = [i32, i32, i64, fp, fp, fp, fp, vp]
    L.fwi_model_convert.restype = st
    L.fwi_chain_rule.argtypes = [i32, i64, fp, fp, fp, fp, fp, fp, vp]
    L.fwi_chain_rule.restype = st
    L.fwi_contrast_scale.argtypes = [i64, fp, fp, vp]
    L.fwi_contrast_scale.restype = st
    L.fwi_descent_direction.argtypes = [i64, fp, fp, fp, fp, vp]
    L.fwi_descent_direction.restype = st
    L.fwi_descent_apply.argtypes = [i64, fp, fp, fp, ctypes.c_float, fp, vp]
    L.fwi_descent_apply.restype = st
    L.fwi_descent_norms.argtypes = [i64, fp, fp, fp, vp]
    L.fwi_descent_norms.restype = st
    dbl = ctypes.c_double
    L.fwi_born_green.argtypes = [i32, fp, i32, fp, i32, fp, dbl, dbl, fp, fp, fp, vp]
    L.fwi_born_green.restype = st
    L.fwi_born_workspace_bytes.argtypes = [i32, i32, i32, i32]
    L.fwi_born_workspace_bytes.restype = sz
    L.fwi_born_data.argtypes = [i32, fp, fp, i32, i32, i32, dbl, dbl, dbl, fp, fp,
                                fp, fp, fp, fp, fp, fp, fp, fp, vp, sz, vp]
    L.fwi_born_data.restype = st
    L.fwi_born_misfit.argtypes = [i64, fp, fp, fp, fp, vp, sz, vp]
    L.fwi_born_misfit.restype = st
    L.fwi_born_gradient.argtypes = [i32, fp, fp, i32, i32, i32, dbl, dbl, dbl, fp,
                                    fp, fp, fp, fp, fp, fp, fp, fp, vp, sz, vp]
    L.fwi_born_gradient.restype = st
    L.fwi_born_contrasts.argtypes = [i32, i32, i64, fp, fp, fp, fp, vp]
    L.fwi_born_contrasts.restype = st
    L.fwi_born_chain.argtypes = [i32, i32, i64, fp, fp, fp, fp, fp, fp, vp]
    L.fwi_born_chain.restype = st
    L.fwi_born_hessian.argtypes = [i32, fp, fp, i32, i32, dbl, dbl, fp, fp, fp, fp, fp, fp,
                                   i32, fp, vp]
    L.fwi_born_hessian.restype = st
    L.fwi_timing_enable.argtypes = [vp, i32]
    L.fwi_timing_enable.restype = st
    L.fwi_timing_read.argtypes = [vp, ctypes.POINTER(FwiTiming), i32]
    L.fwi_timing_read.restype = st
    L.fwi_sync.argtypes = [vp]
    L.fwi_sync.restype = st
    L.fwi_status_str.argtypes = [st]
    L.fwi_status_str.restype = ctypes.c_char_p
    L.fwi_last_error.argtypes = []
    L.fwi_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(status):
    if status != FWI_OK:
        msg = lib().fwi_last_error().decode()
        raise FwiError(status, msg)
    return status
