"""Build step for the HIP library ``libccl.so`` (gfx950).

``python -m paper_1712_09789_amd.build`` compiles the kernels and the C-ABI
host code with hipcc and links them in-tree, next to this file.
The host-sanitized variant for the CPU tests is built by
``build_sanitized.py``.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libccl.so")
ARCH = "gfx950"

# Packed-FP32 instructions are kept out of every HIP object.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


# Tile heights the kernels are compiled for (one object each; ccl_kernels.h
# lists the same heights).
TILE_ROWS = (32, 64, 128)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    common = ["-O3", "-std=c++17", "-fPIC", "-Wall", f"-I{INCLUDE}", f"-I{CSRC}"]
    objs = []
    for rows in TILE_ROWS:
        k_obj = os.path.join(BUILD, f"ccl_kernels_r{rows}.o")
        _run([hipcc, *common, f"-DCCL_TILE_ROWS={rows}", f"-DCCL_SHAPE_NS=r{rows}",
              f"--offload-arch={ARCH}", *DEVICE_FLAGS, "-c",
              os.path.join(CSRC, "ccl_kernels.hip"), "-o", k_obj], verbose)
        objs.append(k_obj)
    a_obj = os.path.join(BUILD, "ccl_api.o")
    _run([hipcc, *common, "-x", "hip", f"--offload-arch={ARCH}", *DEVICE_FLAGS, "-c",
          os.path.join(CSRC, "ccl_api.cpp"), "-o", a_obj], verbose)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs, a_obj],
         verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)
