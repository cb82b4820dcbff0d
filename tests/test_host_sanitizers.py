"""CPU: the library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds a host-only instrumented copy of the library (tests/sanitizer/build_host_san.py)
and runs the C driver tests/sanitizer/host_abi_check.c against it: default schedules
for every edge up to 4096, the autotuner cache reader on malformed and hostile
files, descriptor validation of plans, batches and particle objects, and the
resource hooks.  A sanitizer finding aborts the driver, which fails the test."""

import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc"))
                    or not os.path.exists("/opt/rocm/llvm/bin/clang"), reason="needs hipcc and clang")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, os.path.join(HERE, "sanitizer"))
    try:
        import build_host_san
    finally:
        sys.path.pop(0)
    drv = build_host_san.build(str(tmp_path / "build"))
    run = tmp_path / "run"
    run.mkdir()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([drv, str(run)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-6000:]
    assert "host ABI checks passed" in r.stdout
