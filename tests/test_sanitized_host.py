"""The host side of the C ABI under AddressSanitizer and
UndefinedBehaviorSanitizer: the CPU tests of the ABI (argument validation,
launch-policy tables and their loader, workspace sizing, the error paths)
run again in a child process against libccl_san.so, the library built with
the host code instrumented and the C++ library's bounds assertions on
(paper_1712_09789_amd/build_sanitized.py).  Any sanitizer report
fails the test; the device code is not instrumented."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sanitized():
    b = pytest.importorskip("paper_1712_09789_amd.build_sanitized")
    rt = b.asan_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime in this toolchain")
    if not os.path.exists(b.SAN_LIB):
        b.build_sanitized()
    return b.SAN_LIB, rt


def test_library_is_instrumented(sanitized):
    lib, _ = sanitized
    out = subprocess.run(["nm", "-D", lib], capture_output=True, text=True, check=True).stdout
    assert "__asan_report_load" in out and "__ubsan_handle" in out


def test_abi_tests_are_clean_under_the_sanitizers(sanitized):
    lib, rt = sanitized
    env = dict(os.environ, LD_PRELOAD=rt, CCL_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", "tests/test_abi.py", "tests/test_binding_cpu.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    log = r.stdout + r.stderr
    assert "AddressSanitizer" not in log and "runtime error:" not in log, log[-4000:]
    assert r.returncode == 0, log[-4000:]
    assert " passed" in log
