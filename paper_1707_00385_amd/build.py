"""Builds libqcurv.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libqcurv.so")

# Kernel translation units (compiled in parallel: the per-frame kernels for each of
# default / rejection / strided / strided + rejection, and the batched kernels, each
# instantiate every window size) and the host side.
SOURCES = ["fit_frame.hip", "fit_frame_reject.hip", "fit_frame_strided.hip",
           "fit_frame_strided_reject.hip", "fit_batch.hip", "qcurv_api.cpp", "serve.cpp"]

# Packed FP32 instructions are disabled: the compiler would otherwise form them from
# scalar float code.  fp-contract is off so that every fused multiply-add is the one
# written in the source, which keeps results independent of tile shape and batching.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-ffp-contract=off", "-Wall", "-Wno-unused-function"]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, extra: list | None = None) -> str:
    build_dir = os.path.join(PKG, "_build")
    os.makedirs(build_dir, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        cmds.append([hipcc()] + HIP_FLAGS + (extra or []) + ["-I", INCLUDE, "-I", CSRC] +
                    ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", "0")) or os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(jobs) as pool:
        procs = list(pool.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
    for cmd, proc in zip(cmds, procs):
        if verbose or proc.returncode != 0:
            print(" ".join(cmd), flush=True)
            sys.stderr.write(proc.stderr)
        if proc.returncode != 0:
            raise subprocess.CalledProcessError(proc.returncode, cmd)
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
