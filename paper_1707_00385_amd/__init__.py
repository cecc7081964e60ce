"""MI355X-native principal curvatures from range images by robust quadric-patch fitting.

The per-pixel fit runs in hand-written HIP kernels for gfx950 behind the C ABI of
``libqcurv.so`` (declared in ``include/qcurv.h``).  This package is a thin binding:
argument marshalling only.  Importing it does not load the library; the first call
does, and fails loudly if the library has not been built.
"""
__all__ = ["scenes"]
