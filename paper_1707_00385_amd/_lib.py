"""ctypes declarations of libqcurv.so's C ABI (include/qcurv.h).

Argument marshalling only.  Loading fails loudly when the library has not been built:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# QCURV_LIB may name another build of the same library (e.g. a variant compiled with
# different occupancy settings); by default the in-tree build is used.
LIB_PATH = os.environ.get("QCURV_LIB") or os.path.join(PKG, "libqcurv.so")

QC_OK = 0
QC_ERR_INVALID_ARG = -1
QC_ERR_UNSUPPORTED = -2
QC_DEPTH_U16, QC_DEPTH_F16, QC_DEPTH_F32 = 0, 1, 2
QC_PREC_MIXED, QC_PREC_FP32, QC_PREC_FP64 = 0, 1, 2
QC_FLAG_VALID, QC_FLAG_FP64, QC_FLAG_ILLCOND = 1, 2, 4
QC_MAX_RADIUS = 18

# Every exported symbol declared in include/qcurv.h.
EXPORTS = ["qc_params_default", "qc_create", "qc_destroy", "qc_fit", "qc_fit_batch", "qc_tune",
           "qc_tune_save", "qc_tune_load", "qc_server_create", "qc_server_submit",
           "qc_server_poll", "qc_server_release", "qc_server_get_stats", "qc_server_destroy",
           "qc_last_refit_count", "qc_set_timing", "qc_get_timing", "qc_last_hip_error",
           "qc_status_string", "qc_fit_noalloc"]
QC_ERR_BUSY = -5
QC_ERR_TOO_LARGE = -7
QC_OUT_NORMAL, QC_OUT_RESIDUAL, QC_OUT_FLAGS = 1, 2, 4
QC_MAX_BATCH = 256


class Intrinsics(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float)]


class Params(ctypes.Structure):
    _fields_ = [("radius", ctypes.c_int32), ("normal_radius", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("k", ctypes.c_float),
                ("reject", ctypes.c_int32), ("depth_scale", ctypes.c_float),
                ("precision", ctypes.c_int32), ("cond_max", ctypes.c_float),
                ("step_max", ctypes.c_float), ("tile_width", ctypes.c_int32),
                ("stride", ctypes.c_int32)]


class Frame(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("format", ctypes.c_int32),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("pitch_bytes", ctypes.c_int64), ("K", Intrinsics)]


class Output(ctypes.Structure):
    _fields_ = [("k1", ctypes.c_void_p), ("k2", ctypes.c_void_p), ("normal", ctypes.c_void_p),
                ("residual", ctypes.c_void_p), ("flags", ctypes.c_void_p)]


class BatchItem(ctypes.Structure):
    _fields_ = [("frame", Frame), ("params", Params), ("out", Output)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("memory_budget", ctypes.c_size_t), ("max_batch", ctypes.c_int32),
                ("max_in_flight", ctypes.c_int32), ("outputs", ctypes.c_int32),
                ("staging_budget", ctypes.c_size_t)]


class Request(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("format", ctypes.c_int32),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("pitch_bytes", ctypes.c_int64), ("K", Intrinsics), ("params", Params),
                ("tag", ctypes.c_uint64)]


class Completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("t_submit_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64),
                ("k1", ctypes.c_void_p), ("k2", ctypes.c_void_p), ("normal", ctypes.c_void_p),
                ("residual", ctypes.c_void_p), ("flags", ctypes.c_void_p)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("queued", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("device_bytes_in_use", ctypes.c_size_t)]


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
    lib.qc_fit_noalloc.argtypes = [vp, ctypes.POINTER(Frame), ctypes.POINTER(Params),
                                   ctypes.POINTER(Output), vp]
    lib.qc_fit_noalloc.restype = ctypes.c_int
    lib.qc_fit_batch.argtypes = [vp, ctypes.POINTER(BatchItem), ctypes.c_int32, vp]
    lib.qc_fit_batch.restype = ctypes.c_int
    lib.qc_tune.argtypes = [vp, ctypes.POINTER(Frame), ctypes.POINTER(Params), ctypes.POINTER(Output),
                            ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.qc_tune.restype = ctypes.c_int
    lib.qc_tune_save.argtypes = [vp, ctypes.c_char_p]
    lib.qc_tune_save.restype = ctypes.c_int
    lib.qc_tune_load.argtypes = [vp, ctypes.c_char_p]
    lib.qc_tune_load.restype = ctypes.c_int
    lib.qc_server_create.argtypes = [vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    lib.qc_server_create.restype = ctypes.c_int
    lib.qc_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    lib.qc_server_submit.restype = ctypes.c_int
    lib.qc_server_poll.argtypes = [vp, ctypes.POINTER(Completion), ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32), ctypes.c_int64]
    lib.qc_server_poll.restype = ctypes.c_int
    lib.qc_server_release.argtypes = [vp, ctypes.c_uint64]
    lib.qc_server_release.restype = ctypes.c_int
    lib.qc_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.qc_server_get_stats.restype = ctypes.c_int
    lib.qc_server_destroy.argtypes = [vp]
    lib.qc_server_destroy.restype = ctypes.c_int
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
