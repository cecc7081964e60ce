"""The C ABI library loads on any machine and exports what include/qcurv.h declares.
No compute call is made here (no GPU needed)."""
import ctypes
import os
import re
import subprocess

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
    assert p.precision == _lib.QC_PREC_MIXED and p.reject == 0 and p.stride == 1
    assert p.cond_max == pytest.approx(15.0) and p.step_max == pytest.approx(0.1)
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert lib.qc_status_string(code)
    assert lib.qc_status_string(12345) == b"unknown status"


def test_null_arguments_rejected_without_a_device():
    lib = _lib.load()
    assert lib.qc_fit(None, None, None, None, None) == -1
    assert lib.qc_fit_noalloc(None, None, None, None, None) == -1
    assert lib.qc_create(None, 0) == -1
    assert lib.qc_destroy(None) == 0
    assert lib.qc_last_hip_error(None) == 0
    assert lib.qc_last_refit_count(None, None) == -1


# struct name in the header -> ctypes class in the binding
_STRUCTS = {"qc_intrinsics": "Intrinsics", "qc_params": "Params", "qc_frame": "Frame",
            "qc_output": "Output", "qc_batch_item": "BatchItem", "qc_server_config": "ServerConfig",
            "qc_request": "Request", "qc_completion": "Completion", "qc_server_stats": "ServerStats",
            "qc_timing": "Timing"}


def test_struct_layouts_match_header(tmp_path):
    """Every struct the binding marshals has the header's size and field offsets (a C
    program compiled against include/qcurv.h prints them)."""
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "qcurv.h"', 'int main(void) {']
    for c_name, py_name in _STRUCTS.items():
        cls = getattr(_lib, py_name)
        lines.append(f'printf("{c_name} size %zu\\n", sizeof({c_name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{c_name} {field} %zu\\n", offsetof({c_name}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        struct, field, value = line.split()
        got[(struct, field)] = int(value)
    for c_name, py_name in _STRUCTS.items():
        cls = getattr(_lib, py_name)
        assert got[(c_name, "size")] == ctypes.sizeof(cls), c_name
        for field, _ in cls._fields_:
            assert got[(c_name, field)] == getattr(cls, field).offset, (c_name, field)
