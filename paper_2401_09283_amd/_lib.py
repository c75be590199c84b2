"""ctypes loader and signatures of libgmc.so (the C ABI declared in include/gmc.h).

The HIP library is the only compute path: if it is missing this module raises,
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GMC_LIB", os.path.join(_HERE, "libgmc.so"))

GMC_OK = 0
STATUS = {0: "GMC_OK", -1: "GMC_E_INVALID", -2: "GMC_E_WORKSPACE", -3: "GMC_E_HIP", -4: "GMC_E_GEOMETRY",
          -5: "GMC_E_UNSUPPORTED"}
WEIGHT = {"paper": 0, "fdk": 1}
GRAD = {"paper": 0, "exact": 1}
FLAG_FORCE_GLOBAL = 1
FLAG_FORCE_EDGE = 2
WORK_PREPARED = 1
NOALLOC_SCRATCH_BYTES = 64 << 20   # GMC_NOALLOC_SCRATCH_BYTES

EXPORTS = ["gmc_plan_create", "gmc_plan_destroy", "gmc_workspace_bytes", "gmc_plan_info", "gmc_compose",
           "gmc_backproject", "gmc_backproject_vjp", "gmc_backproject_vjp_noalloc", "gmc_prepare", "gmc_bp_forward", "gmc_bp_vjp",
           "gmc_bp_vjp_finish", "gmc_loss_sumsq_grad", "gmc_loss_entropy_tv",
           "gmc_bspline_theta", "gmc_bspline_grad", "gmc_akima_theta", "gmc_akima_grad", "gmc_forward_project", "gmc_forward_project_parts", "gmc_adam_step", "gmc_gd_step", "gmc_debug_project",
           "gmc_launch_batch", "gmc_check", "gmc_status_string", "gmc_last_error"]


class GmcError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__("%s failed: %s: %s" % (where, STATUS.get(status, status), msg))
        self.status = status


class Geometry(ctypes.Structure):
    _fields_ = [("n_views", ctypes.c_int32), ("det_w", ctypes.c_int32), ("det_h", ctypes.c_int32),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("voxel_mm", ctypes.c_double * 3), ("origin_mm", ctypes.c_double * 3),
                ("weighting", ctypes.c_int32), ("grad_mode", ctypes.c_int32), ("flags", ctypes.c_int32)]


class Work(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("proj", ctypes.c_void_p), ("P", ctypes.c_void_p),
                ("theta", ctypes.c_void_p), ("vol", ctypes.c_void_p), ("grad_vol", ctypes.c_void_p),
                ("grad_theta", ctypes.c_void_p), ("grad_P", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("phase", ctypes.c_int32), ("flags", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libgmc.so not found at %s: build it with `python -m paper_2401_09283_amd.build` "
                          "(there is no non-HIP fallback)" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "gmc_plan_create": ([ctypes.POINTER(Geometry), vp, ctypes.POINTER(vp)], i32),
        "gmc_plan_destroy": ([vp], i32),
        "gmc_workspace_bytes": ([vp], ctypes.c_size_t),
        "gmc_plan_info": ([vp, ctypes.POINTER(i64)], i32),
        "gmc_compose": ([vp, vp, vp, vp, vp, vp], i32),
        "gmc_backproject": ([vp, vp, vp, vp, vp, vp, vp], i32),
        "gmc_backproject_vjp": ([vp, vp, vp, vp, vp, vp, vp, vp, vp], i32),
        "gmc_backproject_vjp_noalloc": ([vp, vp, vp, vp, vp, vp, vp, vp, vp], i32),
        "gmc_prepare": ([vp, vp, vp, i32, vp, vp], i32),
        "gmc_bp_forward": ([vp, vp, vp, vp, vp], i32),
        "gmc_bp_vjp": ([vp, vp, vp, vp, vp], i32),
        "gmc_bp_vjp_finish": ([vp, vp, vp, vp, vp], i32),
        "gmc_loss_sumsq_grad": ([vp, vp, vp, vp, vp, vp], i32),
        "gmc_loss_entropy_tv": ([vp, vp, f64, f64, f64, f64, vp, vp, vp, vp], i32),
        "gmc_bspline_theta": ([i32, i32, vp, vp, vp], i32),
        "gmc_bspline_grad": ([i32, i32, vp, vp, vp], i32),
        "gmc_akima_theta": ([i32, i32, vp, vp, vp], i32),
        "gmc_forward_project": ([vp, vp, vp, vp, vp, vp, vp], i32),
        "gmc_forward_project_parts": ([vp, vp, vp, i32, vp, vp, vp, vp, vp], i32),
        "gmc_akima_grad": ([i32, i32, vp, vp, vp, vp], i32),
        "gmc_adam_step": ([i64, vp, vp, vp, vp, i32, f64, f64, f64, f64, vp], i32),
        "gmc_gd_step": ([i64, vp, vp, i32, f64, f64, vp], i32),
        "gmc_debug_project": ([vp, i64, vp, vp, vp, vp, vp, vp], i32),
        "gmc_launch_batch": ([ctypes.POINTER(Work), i32, vp], i32),
        "gmc_check": ([vp, vp, vp], i32),
        "gmc_status_string": ([i32], ctypes.c_char_p),
        "gmc_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def check(status: int, where: str):
    if status != GMC_OK:
        raise GmcError(status, where, lib().gmc_last_error().decode(errors="replace"))
