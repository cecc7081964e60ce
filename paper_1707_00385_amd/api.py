"""Python binding of libqcurv.so.  Argument marshalling only: torch supplies device
memory and streams, every step of the fit runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes
from typing import Dict, Optional, Sequence

import torch

from . import _lib

_FORMATS = {"u16": _lib.QC_DEPTH_U16, "f16": _lib.QC_DEPTH_F16, "f32": _lib.QC_DEPTH_F32}
_PRECISIONS = {"mixed": _lib.QC_PREC_MIXED, "fp32": _lib.QC_PREC_FP32, "fp64": _lib.QC_PREC_FP64}


def default_params() -> _lib.Params:
    p = _lib.Params()
    _lib.load().qc_params_default(ctypes.byref(p))
    return p


def make_params(radius: int = 7, iterations: int = 5, k: float = 1e-5, normal_radius: int = 3,
                depth_scale: float = 1e-3, precision: str = "mixed",
                cond_max: Optional[float] = None, step_max: Optional[float] = None) -> _lib.Params:
    p = default_params()
    p.radius = int(radius)
    p.iterations = int(iterations)
    p.k = float(k)
    p.normal_radius = int(normal_radius)
    p.depth_scale = float(depth_scale)
    p.precision = _PRECISIONS[precision]
    if cond_max is not None:
        p.cond_max = float(cond_max)
    if step_max is not None:
        p.step_max = float(step_max)
    return p


def depth_format(t: torch.Tensor) -> int:
    if t.dtype in (torch.uint16, torch.int16):   # int16 carries u16 bits (torch transfers)
        return _lib.QC_DEPTH_U16
    if t.dtype == torch.float16:
        return _lib.QC_DEPTH_F16
    if t.dtype == torch.float32:
        return _lib.QC_DEPTH_F32
    raise TypeError(f"unsupported depth dtype {t.dtype}")


def upload_depth(depth, fmt: str, device="cuda:0") -> torch.Tensor:
    """Copies a host depth image (numpy) to the GPU in the given sample format: "u16"
    (carried as int16 bits), "f16" or "f32"."""
    import numpy as np
    if fmt == "u16":
        t = torch.from_numpy(np.ascontiguousarray(np.asarray(depth).astype(np.uint16)).view(np.int16))
    elif fmt == "f16":
        t = torch.from_numpy(np.ascontiguousarray(np.asarray(depth).astype(np.float16)))
    elif fmt == "f32":
        t = torch.from_numpy(np.ascontiguousarray(np.asarray(depth).astype(np.float32)))
    else:
        raise ValueError(f"unknown depth format {fmt}")
    return t.to(device)


def make_frame(depth: torch.Tensor, K: Sequence[float]) -> _lib.Frame:
    if depth.dim() != 2 or not depth.is_cuda:
        raise ValueError("depth must be a 2-D tensor on a GPU")
    if depth.stride(1) != 1:
        raise ValueError("depth rows must be contiguous")
    f = _lib.Frame()
    f.depth = depth.data_ptr()
    f.format = depth_format(depth)
    f.height, f.width = depth.shape
    f.pitch_bytes = depth.stride(0) * depth.element_size()
    f.K = _lib.Intrinsics(*[float(x) for x in K])
    return f


def make_outputs(height: int, width: int, device, normal=False, residual=False,
                 flags=True) -> Dict[str, torch.Tensor]:
    o = {"k1": torch.empty((height, width), dtype=torch.float32, device=device),
         "k2": torch.empty((height, width), dtype=torch.float32, device=device)}
    if normal:
        o["normal"] = torch.empty((height, width, 3), dtype=torch.float32, device=device)
    if residual:
        o["residual"] = torch.empty((height, width), dtype=torch.float32, device=device)
    if flags:
        o["flags"] = torch.empty((height, width), dtype=torch.uint8, device=device)
    return o


def output_struct(o: Dict[str, torch.Tensor]) -> _lib.Output:
    s = _lib.Output()
    for name in ("k1", "k2", "normal", "residual", "flags"):
        t = o.get(name)
        if t is not None and not t.is_contiguous():
            raise ValueError(f"output {name} must be contiguous")
        setattr(s, name, t.data_ptr() if t is not None else None)
    return s


class Context:
    """One qc_context (device scratch for the FP64 recomputation list)."""

    def __init__(self, device: int = 0):
        self._lib = _lib.load()
        self._h = ctypes.c_void_p()
        _lib.check(self._lib.qc_create(ctypes.byref(self._h), int(device)), "qc_create")
        self.device = int(device)

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def close(self) -> None:
        if self._h:
            self._lib.qc_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fit(self, depth: torch.Tensor, K: Sequence[float], params: Optional[_lib.Params] = None,
            out: Optional[Dict[str, torch.Tensor]] = None, stream: Optional[torch.cuda.Stream] = None,
            normal: bool = False, residual: bool = False, flags: bool = True,
            **param_kw) -> Dict[str, torch.Tensor]:
        """Fits every pixel of `depth` (H x W on the GPU).  Returns k1, k2 (and normal,
        residual, flags when asked) as GPU tensors; asynchronous on `stream`."""
        if params is None:
            params = make_params(**param_kw)
        frame = make_frame(depth, K)
        if out is None:
            out = make_outputs(frame.height, frame.width, depth.device, normal, residual, flags)
        st = stream if stream is not None else torch.cuda.current_stream(depth.device)
        _lib.check(self._lib.qc_fit(self._h, ctypes.byref(frame), ctypes.byref(params),
                                    ctypes.byref(output_struct(out)),
                                    ctypes.c_void_p(st.cuda_stream)), "qc_fit")
        return out

    def set_timing(self, enable: bool) -> None:
        _lib.check(self._lib.qc_set_timing(self._h, int(bool(enable))), "qc_set_timing")

    def get_timing(self, reset: bool = False) -> dict:
        t = _lib.Timing()
        _lib.check(self._lib.qc_get_timing(self._h, ctypes.byref(t), int(bool(reset))),
                   "qc_get_timing")
        return {"calls": int(t.calls), "fit_ms": float(t.fit_ms), "refit_ms": float(t.refit_ms)}

    def last_refit_count(self) -> int:
        n = ctypes.c_uint32()
        _lib.check(self._lib.qc_last_refit_count(self._h, ctypes.byref(n)), "qc_last_refit_count")
        return int(n.value)
