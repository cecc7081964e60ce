"""Python binding of libqcurv.so.  Argument marshalling only: torch supplies device
memory and streams, every step of the fit runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Sequence

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
                cond_max: Optional[float] = None, step_max: Optional[float] = None,
                tile_width: int = 0, reject: int = 0, stride: int = 1) -> _lib.Params:
    p = default_params()
    p.reject = int(reject)
    p.stride = int(stride)
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
    p.tile_width = int(tile_width)
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

    def fit_noalloc(self, depth: torch.Tensor, K: Sequence[float], out: Dict[str, torch.Tensor],
                    params: Optional[_lib.Params] = None, stream: Optional[torch.cuda.Stream] = None,
                    **param_kw) -> Dict[str, torch.Tensor]:
        """qc_fit_noalloc: as fit(), into caller-allocated outputs `out` (make_outputs),
        with the recomputation list in the library's fixed device scratch."""
        if params is None:
            params = make_params(**param_kw)
        frame = make_frame(depth, K)
        st = stream if stream is not None else torch.cuda.current_stream(depth.device)
        _lib.check(self._lib.qc_fit_noalloc(self._h, ctypes.byref(frame), ctypes.byref(params),
                                            ctypes.byref(output_struct(out)),
                                            ctypes.c_void_p(st.cuda_stream)), "qc_fit_noalloc")
        return out

    def fit_batch(self, jobs: Sequence[tuple], stream: Optional[torch.cuda.Stream] = None
                  ) -> List[Dict[str, torch.Tensor]]:
        """Fits several frames in one batched launch.  `jobs` holds (depth, K, params,
        out) tuples (out may be None: k1, k2 and flags are allocated).  Returns the
        output dicts in job order; asynchronous on `stream`."""
        if len(jobs) > _lib.QC_MAX_BATCH:
            raise ValueError(f"at most {_lib.QC_MAX_BATCH} frames per batch")
        items = (_lib.BatchItem * max(len(jobs), 1))()
        outs = []
        for i, (depth, K, params, out) in enumerate(jobs):
            frame = make_frame(depth, K)
            if out is None:
                out = make_outputs(frame.height, frame.width, depth.device)
            items[i].frame = frame
            items[i].params = params
            items[i].out = output_struct(out)
            outs.append(out)
        dev = jobs[0][0].device if jobs else torch.device("cuda", self.device)
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        _lib.check(self._lib.qc_fit_batch(self._h, items, len(jobs), ctypes.c_void_p(st.cuda_stream)),
                   "qc_fit_batch")
        return outs

    def tune(self, depth: torch.Tensor, K: Sequence[float], params: _lib.Params, reps: int = 5,
             stream: Optional[torch.cuda.Stream] = None, with_schedule: bool = False):
        """qc_tune: times the FP32 tile shapes (and, for MIXED, FP64 throughout) on this
        frame and records the fastest; returns the tile width, or (tile width, schedule)."""
        frame = make_frame(depth, K)
        out = make_outputs(frame.height, frame.width, depth.device)
        st = stream if stream is not None else torch.cuda.current_stream(depth.device)
        tw, sched = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(self._lib.qc_tune(self._h, ctypes.byref(frame), ctypes.byref(params),
                                     ctypes.byref(output_struct(out)), int(reps),
                                     ctypes.c_void_p(st.cuda_stream), ctypes.byref(tw),
                                     ctypes.byref(sched)), "qc_tune")
        return (int(tw.value), int(sched.value)) if with_schedule else int(tw.value)

    def tune_save(self, path: str) -> None:
        _lib.check(self._lib.qc_tune_save(self._h, path.encode()), "qc_tune_save")

    def tune_load(self, path: str) -> None:
        _lib.check(self._lib.qc_tune_load(self._h, path.encode()), "qc_tune_load")

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


_SAMPLE_FORMAT = {"u16": _lib.QC_DEPTH_U16, "f16": _lib.QC_DEPTH_F16, "f32": _lib.QC_DEPTH_F32}


class Server:
    """A qc_server: frames submitted from host memory are admitted by device memory,
    uploaded and fitted in continuously formed batches; results stay on the device until
    released.  The server owns `ctx` until close()."""

    def __init__(self, ctx: Context, memory_budget: int = 1 << 30, max_batch: int = 64,
                 max_in_flight: int = 2, outputs: int = 0, staging_budget: int = 256 << 20):
        self._lib = ctx._lib
        self.ctx = ctx
        cfg = _lib.ServerConfig(int(memory_budget), int(max_batch), int(max_in_flight),
                                int(outputs), int(staging_budget))
        self._h = ctypes.c_void_p()
        _lib.check(self._lib.qc_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(self._h)),
                   "qc_server_create")

    def submit(self, depth, fmt: str, K: Sequence[float], params: _lib.Params, tag: int = 0):
        """Queues a host frame (numpy, row-major).  Returns the ticket, or None when the
        pinned staging is full right now (QC_ERR_BUSY)."""
        import numpy as np
        a = np.ascontiguousarray(depth)
        r = _lib.Request()
        r.depth = a.ctypes.data
        r.format = _SAMPLE_FORMAT[fmt]
        r.height, r.width = a.shape
        r.pitch_bytes = a.strides[0]
        r.K = _lib.Intrinsics(*[float(x) for x in K])
        r.params = params
        r.tag = int(tag)
        t = ctypes.c_uint64()
        st = self._lib.qc_server_submit(self._h, ctypes.byref(r), ctypes.byref(t))
        if st == _lib.QC_ERR_BUSY:
            return None
        _lib.check(st, "qc_server_submit")
        return int(t.value)

    def poll(self, max_n: int = 64, wait_us: int = 0) -> list:
        buf = (_lib.Completion * max(int(max_n), 1))()
        n = ctypes.c_int32()
        _lib.check(self._lib.qc_server_poll(self._h, buf, int(max_n), ctypes.byref(n), int(wait_us)),
                   "qc_server_poll")
        return [buf[i] for i in range(n.value)]

    def release(self, ticket: int) -> None:
        _lib.check(self._lib.qc_server_release(self._h, int(ticket)), "qc_server_release")

    def stats(self) -> dict:
        s = _lib.ServerStats()
        _lib.check(self._lib.qc_server_get_stats(self._h, ctypes.byref(s)), "qc_server_get_stats")
        return {f: int(getattr(s, f)) for f, _ in _lib.ServerStats._fields_}

    def close(self) -> None:
        if self._h:
            self._lib.qc_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_view(ptr: int, shape: Sequence[int], dtype, device=0) -> torch.Tensor:
    """Copies `prod(shape)` elements at device address `ptr` into a new tensor."""
    import numpy as np
    n = int(np.prod(shape))
    itemsize = torch.tensor([], dtype=dtype).element_size()
    out = torch.empty(n, dtype=dtype, device=torch.device("cuda", device))
    hip = _hip_runtime()
    rc = hip.hipMemcpy(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(int(ptr)),
                       ctypes.c_size_t(n * itemsize), ctypes.c_int(3))   # device to device
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")
    return out.reshape(tuple(shape))


_HIP = None


def _hip_runtime():
    global _HIP
    if _HIP is None:
        _HIP = ctypes.CDLL("libamdhip64.so")
        _HIP.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _HIP.hipMemcpy.restype = ctypes.c_int
    return _HIP
