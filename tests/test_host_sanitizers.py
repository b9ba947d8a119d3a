"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two small programs in tests/sanitize/ are built with gcc/g++ and
-fsanitize=address,undefined (no recovery: the first report aborts):
  * host_check.cpp with the library's pure host translation units
    (csrc/tables.cpp: Gauss-Legendre and the packed tables; csrc/stepper.cpp:
    the BDF(1,2) flow stepper behind frg_flow_solve);
  * oracle_check.c with the oracle (oracle/frg_oracle.c), every entry point on
    small and edge-case inputs.
A run passes when the program exits 0 and prints its "... checks ok" line.  The
flow server's threads need a HIP device and are covered by the GPU tests'
bitwise alone-versus-batched checks instead of ThreadSanitizer.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2607_24908_amd", "csrc")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _build_and_run(cmd, exe, expect):
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    if b.returncode != 0 and "asan" in (b.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + b.stderr[-300:])
    assert b.returncode == 0, b.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert expect in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_host_tables_and_stepper_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_check")
    cmd = ["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(HERE, "sanitize", "host_check.cpp"), os.path.join(CSRC, "tables.cpp"),
           os.path.join(CSRC, "stepper.cpp"), "-o", exe]
    _build_and_run(cmd, exe, "host checks ok")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_check")
    cmd = ["gcc", "-std=gnu11", *SAN, "-Wno-unknown-pragmas",
           os.path.join(HERE, "sanitize", "oracle_check.c"),
           os.path.join(ROOT, "oracle", "frg_oracle.c"), "-lm", "-o", exe]
    _build_and_run(cmd, exe, "oracle checks ok")
