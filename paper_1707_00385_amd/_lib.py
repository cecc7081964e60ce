"""ctypes declarations of libqcurv.so's C ABI (include/qcurv.h).

Argument marshalling only.  Loading fails loudly when the library has not been built:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libqcurv.so")

QC_OK = 0
QC_DEPTH_U16, QC_DEPTH_F16, QC_DEPTH_F32 = 0, 1, 2
QC_PREC_MIXED, QC_PREC_FP32, QC_PREC_FP64 = 0, 1, 2
QC_FLAG_VALID, QC_FLAG_FP64, QC_FLAG_ILLCOND = 1, 2, 4
QC_MAX_RADIUS = 18

# Every exported symbol declared in include/qcurv.h.
EXPORTS = ["qc_params_default", "qc_create", "qc_destroy", "qc_fit", "qc_last_refit_count",
           "qc_set_timing", "qc_get_timing", "qc_last_hip_error", "qc_status_string"]


class Intrinsics(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float)]


class Params(ctypes.Structure):
    _fields_ = [("radius", ctypes.c_int32), ("normal_radius", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("k", ctypes.c_float),
                ("reject", ctypes.c_int32), ("depth_scale", ctypes.c_float),
                ("precision", ctypes.c_int32), ("cond_max", ctypes.c_float),
                ("step_max", ctypes.c_float)]


class Frame(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("format", ctypes.c_int32),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("pitch_bytes", ctypes.c_int64), ("K", Intrinsics)]


class Output(ctypes.Structure):
    _fields_ = [("k1", ctypes.c_void_p), ("k2", ctypes.c_void_p), ("normal", ctypes.c_void_p),
                ("residual", ctypes.c_void_p), ("flags", ctypes.c_void_p)]


class Timing(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_uint64), ("fit_ms", ctypes.c_double),
                ("refit_ms", ctypes.c_double)]


_lib = None


class QcError(RuntimeError):
    def __init__(self, status: int, what: str):
        lib = load()
        msg = lib.qc_status_string(status).decode()
        super().__init__(f"{what}: {msg} ({status})")
        self.status = status


def load() -> ctypes.CDLL:
    """Loads libqcurv.so; raises if it is missing (build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first "
                           "(the curvature fit has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.qc_params_default.argtypes = [ctypes.POINTER(Params)]
    lib.qc_params_default.restype = None
    lib.qc_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    lib.qc_create.restype = ctypes.c_int
    lib.qc_destroy.argtypes = [vp]
    lib.qc_destroy.restype = ctypes.c_int
    lib.qc_fit.argtypes = [vp, ctypes.POINTER(Frame), ctypes.POINTER(Params),
                           ctypes.POINTER(Output), vp]
    lib.qc_fit.restype = ctypes.c_int
    lib.qc_last_refit_count.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32)]
    lib.qc_last_refit_count.restype = ctypes.c_int
    lib.qc_set_timing.argtypes = [vp, ctypes.c_int]
    lib.qc_set_timing.restype = ctypes.c_int
    lib.qc_get_timing.argtypes = [vp, ctypes.POINTER(Timing), ctypes.c_int]
    lib.qc_get_timing.restype = ctypes.c_int
    lib.qc_last_hip_error.argtypes = [vp]
    lib.qc_last_hip_error.restype = ctypes.c_int
    lib.qc_status_string.argtypes = [ctypes.c_int]
    lib.qc_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(status: int, what: str) -> None:
    if status != QC_OK:
        raise QcError(status, what)
