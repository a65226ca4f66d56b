"""Host-sanitized build of the library for the CPU tests of the C ABI.

``python -m paper_1712_09789_amd.build_sanitized`` links
``_build/libccl_san.so`` from the kernel objects of the last regular build
and the host code compiled under AddressSanitizer and
UndefinedBehaviorSanitizer, with the C++ library's bounds assertions on.
Only the host pass is instrumented (every sanitizer flag is given to it
alone); the device code is the regular build's.  The library is linked
without a sanitizer runtime: a process that loads it preloads the
compiler's shared one (asan_runtime()), which also holds the undefined-
behaviour handlers.
"""
from __future__ import annotations

import glob
import os
import sys

from paper_1712_09789_amd.build import ARCH, BUILD, CSRC, DEVICE_FLAGS, INCLUDE, TILE_ROWS, _run

SAN_LIB = os.path.join(BUILD, "libccl_san.so")
HOST_SANITIZE = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
                 "-Xarch_host -fno-sanitize-recover=undefined "
                 "-Xarch_host -fno-omit-frame-pointer -D_GLIBCXX_ASSERTIONS").split()


def asan_runtime() -> str | None:
    """The compiler's shared AddressSanitizer runtime, or None."""
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def build_sanitized(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = [os.path.join(BUILD, f"ccl_kernels_r{rows}.o") for rows in TILE_ROWS]
    missing = [o for o in objs if not os.path.exists(o)]
    if missing:
        raise FileNotFoundError(f"kernel objects missing ({missing[0]}); "
                                "run `python -m paper_1712_09789_amd.build` first")
    a_obj = os.path.join(BUILD, "ccl_api_san.o")
    _run([hipcc, "-O1", "-g", "-std=c++17", "-fPIC", "-Wall", f"-I{INCLUDE}", f"-I{CSRC}",
          *HOST_SANITIZE, "-x", "hip", f"--offload-arch={ARCH}", *DEVICE_FLAGS, "-c",
          os.path.join(CSRC, "ccl_api.cpp"), "-o", a_obj], verbose)
    tmp = SAN_LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs, a_obj],
         verbose)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    print(build_sanitized(verbose=True))
    sys.exit(0)
