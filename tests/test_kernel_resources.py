"""Static checks of the gfx950 code object: every kernel runs without
private (scratch) memory, and the mixed-mode pair kernel fits the register
budget that lets a compute unit hold four of its work-groups.

Compiles csrc/kernels.hip to AMD assembly with the library's own flags (no
GPU needed) and reads the kernel descriptors' metadata.
"""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def kernel_meta(tmp_path_factory):
    if shutil.which("hipcc") is None:
        pytest.skip("needs hipcc")
    from paper_2109_13993_amd import build as lib_build
    out = str(tmp_path_factory.mktemp("asm") / "kernels.s")
    cmd = ["hipcc", "-x", "hip", "-S", "--cuda-device-only", os.path.join(lib_build.CSRC, "kernels.hip"),
           "-o", out] + [f for f in lib_build.COMMON if f not in ("-fPIC",)]
    subprocess.run(cmd, check=True, capture_output=True)
    text = open(out).read()
    meta = {}
    for m in re.finditer(r"\.name:\s+(\S+)\n(.*?)\.vgpr_count:\s+(\d+)", text, re.S):
        scratch = re.search(r"\.private_segment_fixed_size:\s+(\d+)", m.group(2))
        meta[m.group(1)] = {"vgpr": int(m.group(3)), "scratch": int(scratch.group(1)) if scratch else -1}
    assert meta, "no kernel metadata found"
    return meta


def test_no_kernel_uses_scratch(kernel_meta):
    bad = {k: v for k, v in kernel_meta.items() if v["scratch"] != 0}
    assert not bad, bad


def test_mixed_pair_kernel_register_budget(kernel_meta):
    # 256-thread groups, four per compute unit: 4 waves per SIMD, 128 VGPRs each
    pair = [v for k, v in kernel_meta.items() if "k_pair_bandILb1E" in k]
    assert pair and all(v["vgpr"] <= 128 for v in pair), pair
