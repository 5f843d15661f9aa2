"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The library's host side (``api.cpp``: argument checks, camera and ROI set-up,
  frame tables and their pinned staging, batch building, tuning and handle
  bookkeeping) built with g++ sanitizers and linked against a host-memory
  stand-in for the HIP runtime and the kernel launchers
  (``tests/sanitize/fake_hip.cpp``), driven through valid and rejected calls
  (``tests/sanitize/api_driver.cpp``).
* The tetrahedral location tables (``tet_build.cpp``) checked point by point
  against brute force (``tests/sanitize/tet_driver.cpp``).
* The oracle's C code built with gcc sanitizers and run on small inputs and
  edge cases (``tests/sanitize/oracle_driver.c``).

Each run must exit 0 with no sanitizer report; leak detection is on.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined"]


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, timeout=600, env=ENV)
    return r.returncode, r.stdout + r.stderr


def _check(rc, log):
    assert rc == 0, log[-4000:]
    assert "AddressSanitizer" not in log and "runtime error" not in log and "LeakSanitizer" not in log, log[-4000:]


def test_api_host_code_under_sanitizers(tmp_path):
    if shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include/hip"):
        pytest.skip("g++ or the HIP headers are missing")
    inc = ["-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2501_01628_amd", "csrc")]
    exe = str(tmp_path / "api_driver")
    rc, log = _run(["g++", *inc, *FLAGS, "-ffp-contract=off", os.path.join(SAN, "api_driver.cpp"),
                    os.path.join(ROOT, "paper_2501_01628_amd", "csrc", "api.cpp"),
                    os.path.join(ROOT, "paper_2501_01628_amd", "csrc", "tet_build.cpp"),
                    os.path.join(SAN, "fake_hip.cpp"), "-o", exe], str(tmp_path))
    assert rc == 0, log[-4000:]
    rc, log = _run([exe], str(tmp_path))
    _check(rc, log)
    assert "OK: 0 failed expectations" in log


def test_tet_location_tables_under_sanitizers(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ is missing")
    exe = str(tmp_path / "tet_driver")
    rc, log = _run(["g++", "-std=c++17", *FLAGS, "-ffp-contract=off", "-I",
                    os.path.join(ROOT, "paper_2501_01628_amd", "csrc"), os.path.join(SAN, "tet_driver.cpp"),
                    os.path.join(ROOT, "paper_2501_01628_amd", "csrc", "tet_build.cpp"), "-o", exe], str(tmp_path))
    assert rc == 0, log[-4000:]
    rc, log = _run([exe], str(tmp_path))
    _check(rc, log)
    assert "OK: 0 failed expectations" in log


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is missing")
    exe = str(tmp_path / "oracle_driver")
    rc, log = _run(["gcc", "-std=gnu11", *FLAGS, "-ffp-contract=off", "-Wno-unknown-pragmas",
                    os.path.join(SAN, "oracle_driver.c"), "-o", exe, "-lm"], str(tmp_path))
    assert rc == 0, log[-4000:]
    rc, log = _run([exe], str(tmp_path))
    _check(rc, log)
    assert "OK: 0 failed checks" in log
