"""FP64 CPU oracle of the quadric-patch curvature method -- TEST INFRASTRUCTURE ONLY.

A thin ctypes binding of ``oracle.c``.  Only the tests, the package smoke check and
the benchmark's CPU-baseline leg may import it; the product library never does.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from .build import LIB, build

_lib = None


class OracleParams(ctypes.Structure):
    _fields_ = [("radius", ctypes.c_int32), ("normal_radius", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("reject", ctypes.c_int32),
                ("k", ctypes.c_double), ("stride", ctypes.c_int32)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i64p = ctypes.POINTER(ctypes.c_int64)
        pp = ctypes.POINTER(OracleParams)
        lib.oracle_fit_image.argtypes = [dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double, pp,
                                         dp, dp, dp, dp, u8p, ctypes.c_int32]
        lib.oracle_fit_image.restype = ctypes.c_int
        lib.oracle_fit_pixels.argtypes = [dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double, pp,
                                          i64p, ctypes.c_int64, dp, dp, dp, dp, u8p,
                                          ctypes.c_int32]
        lib.oracle_fit_pixels.restype = ctypes.c_int
        lib.oracle_fit_patch.argtypes = [dp, ctypes.c_int32, ctypes.c_int32, dp, pp, dp, dp, dp,
                                         dp, dp]
        lib.oracle_fit_patch.restype = ctypes.c_int
        lib.oracle_residual_jacobian.argtypes = [dp, ctypes.c_double, ctypes.c_double,
                                                 ctypes.c_double, ctypes.c_double, dp, dp, dp]
        lib.oracle_residual_jacobian.restype = None
        lib.oracle_principal_curvatures.argtypes = [ctypes.c_double] * 3 + [dp, dp]
        lib.oracle_principal_curvatures.restype = None
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray], ctype=ctypes.c_double):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def params(radius: int, iterations: int, k: float, normal_radius: int = 3,
           reject: bool = False, stride: int = 1) -> OracleParams:
    return OracleParams(int(radius), int(normal_radius), int(iterations), int(bool(reject)),
                        float(k), int(stride))


def fit_image(depth_m: np.ndarray, fx: float, fy: float, cx: float, cy: float,
              radius: int, iterations: int, k: float, normal_radius: int = 3,
              reject: bool = False, threads: int = 0, stride: int = 1) -> dict:
    """Fits every pixel.  Returns dict of k1, k2, normal (H,W,3), residual, flags."""
    d = np.ascontiguousarray(depth_m, dtype=np.float64)
    H, W = d.shape
    out = dict(k1=np.empty((H, W)), k2=np.empty((H, W)), normal=np.empty((H, W, 3)),
               residual=np.empty((H, W)), flags=np.empty((H, W), dtype=np.uint8))
    p = params(radius, iterations, k, normal_radius, reject, stride)
    rc = _load().oracle_fit_image(_ptr(d), W, H, fx, fy, cx, cy, ctypes.byref(p),
                                  _ptr(out["k1"]), _ptr(out["k2"]), _ptr(out["normal"]),
                                  _ptr(out["residual"]), _ptr(out["flags"], ctypes.c_uint8),
                                  int(threads))
    if rc != 0:
        raise ValueError("oracle_fit_image rejected its arguments")
    return out


def fit_pixels(depth_m: np.ndarray, pixels: np.ndarray, fx: float, fy: float, cx: float,
               cy: float, radius: int, iterations: int, k: float, normal_radius: int = 3,
               reject: bool = False, threads: int = 0, stride: int = 1) -> dict:
    """Fits only the listed pixels (linear indices v*W+u)."""
    d = np.ascontiguousarray(depth_m, dtype=np.float64)
    H, W = d.shape
    px = np.ascontiguousarray(pixels, dtype=np.int64).ravel()
    n = px.size
    out = dict(k1=np.empty(n), k2=np.empty(n), normal=np.empty((n, 3)), residual=np.empty(n),
               flags=np.empty(n, dtype=np.uint8))
    p = params(radius, iterations, k, normal_radius, reject, stride)
    rc = _load().oracle_fit_pixels(_ptr(d), W, H, fx, fy, cx, cy, ctypes.byref(p),
                                   _ptr(px, ctypes.c_int64), n, _ptr(out["k1"]), _ptr(out["k2"]),
                                   _ptr(out["normal"]), _ptr(out["residual"]),
                                   _ptr(out["flags"], ctypes.c_uint8), int(threads))
    if rc != 0:
        raise ValueError("oracle_fit_pixels rejected its arguments")
    return out


def fit_patch(pts: np.ndarray, centre: int, n0, iterations: int, k: float,
              reject: bool = False) -> dict:
    """Fits one explicit point set; returns k1, k2, normal, residual, state, valid."""
    P = np.ascontiguousarray(pts, dtype=np.float64)
    n0a = np.ascontiguousarray(n0, dtype=np.float64)
    k1 = ctypes.c_double()
    k2 = ctypes.c_double()
    res = ctypes.c_double()
    nrm = np.empty(3)
    st = np.empty(13)
    p = params(1, iterations, k, 1, reject)
    rc = _load().oracle_fit_patch(_ptr(P), P.shape[0], int(centre), _ptr(n0a), ctypes.byref(p),
                                  ctypes.byref(k1), ctypes.byref(k2), _ptr(nrm), ctypes.byref(res),
                                  _ptr(st))
    if rc < 0:
        raise ValueError("oracle_fit_patch rejected its arguments")
    return dict(valid=rc == 1, k1=k1.value, k2=k2.value, normal=nrm, residual=res.value,
                R=st[:9].reshape(3, 3), tz=st[9], A=st[10], B=st[11], C=st[12])


def residual_jacobian(R: np.ndarray, tz: float, A: float, B: float, C: float, p) -> tuple:
    Rm = np.ascontiguousarray(R, dtype=np.float64)
    pa = np.ascontiguousarray(p, dtype=np.float64)
    e = ctypes.c_double()
    J = np.empty(6)
    _load().oracle_residual_jacobian(_ptr(Rm), tz, A, B, C, _ptr(pa), ctypes.byref(e), _ptr(J))
    return e.value, J


def principal_curvatures(A: float, B: float, C: float) -> tuple:
    a = ctypes.c_double()
    b = ctypes.c_double()
    _load().oracle_principal_curvatures(A, B, C, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value
