"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

- The oracle (oracle/oracle.c) with tests/sanitize/oracle_main.c: searches
  of several shapes in both evaluation orders, forced prefixes, sampled
  scores, degenerate and non-finite inputs, argument errors.
- The library's host runtime (csrc/driver.cpp: argument checks, workspace
  sizing and carving, the iteration loop, batch scheduling, the graph cache,
  result copies) built with g++ against tests/sanitize/fake_hip.cpp, a host
  stand-in of the HIP runtime and of the kernel launchers, driven by
  tests/sanitize/driver_main.cpp through every entry point, undersized
  workspaces and failed allocations.

Both programs abort on the first sanitizer report; leaks are checked too
(the batch graph cache, which lives until the process ends, is suppressed).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2109_13993_amd", "csrc")
FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0"
    env["LSAN_OPTIONS"] = "suppressions=%s:print_suppressions=0" % os.path.join(SAN, "lsan.supp")
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "4"
    return env


def _build(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower() and "cannot find" in r.stderr:
        pytest.skip("sanitizer runtime not installed")
    assert r.returncode == 0, r.stderr[-4000:]


def _run(exe, tag):
    r = subprocess.run([exe], capture_output=True, text=True, env=_env(), timeout=600)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out and "ERROR: LeakSanitizer" not in out, out[-4000:]
    assert "runtime error" not in out, out[-4000:]
    assert r.returncode == 0 and ("%s host checks passed" % tag) in r.stdout, out[-4000:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _build(["gcc", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off"] + FLAGS +
           [os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(SAN, "oracle_main.c"), "-o", exe, "-lm"])
    _run(exe, "oracle")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include/hip"),
                    reason="g++ or the HIP headers not found")
def test_driver_host_code_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "driver_san")
    _build(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC] + FLAGS +
           [os.path.join(CSRC, "driver.cpp"), os.path.join(SAN, "fake_hip.cpp"),
            os.path.join(SAN, "driver_main.cpp"), "-o", exe])
    _run(exe, "driver")
