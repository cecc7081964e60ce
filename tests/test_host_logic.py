"""Host-side logic of the library that runs without a GPU."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_range_allocator_first_fit_and_coalescing(tmp_path):
    """The serving loop's device-memory admission uses this allocator: random sequences
    are checked against a brute-force occupancy map (first fit, no overlap, exact
    accounting, full coalescing)."""
    exe = tmp_path / "test_range_alloc"
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall",
                    "-I", os.path.join(ROOT, "paper_1707_00385_amd", "csrc"),
                    os.path.join(ROOT, "tests", "cpp", "test_range_alloc.cpp"), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    assert out.strip() == "OK"
