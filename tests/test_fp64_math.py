"""Host check of the FP64 path's logarithm (log1p_unit in csrc/fp64_math.h).

The FP64 pair and entropy kernels form log cosh(u) + ln 2 as
|u| + log(1 + e^{-2|u|}) with a binary64 log(1 + y) written for 0 <= y <= 1.
The header compiles for the host as well; with contraction off (the function
spells out its fused multiply-adds) the host build performs the same
binary64 operations in the same order as the device build, and its accuracy
is pinned here against a long double reference.  The FP64 parity tests pin
the device build through the kernels' results.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2109_13993_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_log1p_unit_within_two_ulp(tmp_path):
    exe = str(tmp_path / "fp64_math_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-I", CSRC,
                    os.path.join(HERE, "fp64_math_check.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    max_ulp, worst, bad = float(out[0]), float(out[1]), int(out[2])
    assert bad == 0
    assert max_ulp < 2.0, (max_ulp, worst)
