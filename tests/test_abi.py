"""The C ABI library loads on any machine and exports what include/qcurv.h declares.
No compute call is made here (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1707_00385_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "qcurv.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qc_[a-z_]+)\s*\(", text)))


def test_header_declarations_match_binding():
    assert _declared_functions() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _declared_functions():
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_defaults_and_status_strings():
    lib = _lib.load()
    p = _lib.Params()
    lib.qc_params_default(ctypes.byref(p))
    assert (p.radius, p.normal_radius, p.iterations) == (7, 3, 5)
    assert p.k == pytest.approx(1e-5) and p.depth_scale == pytest.approx(1e-3)
    assert p.precision == _lib.QC_PREC_MIXED and p.reject == 0
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.qc_status_string(code)
    assert lib.qc_status_string(12345) == b"unknown status"


def test_null_arguments_rejected_without_a_device():
    lib = _lib.load()
    assert lib.qc_fit(None, None, None, None, None) == -1
    assert lib.qc_create(None, 0) == -1
    assert lib.qc_destroy(None) == 0
    assert lib.qc_last_hip_error(None) == 0
    assert lib.qc_last_refit_count(None, None) == -1
