"""The hardware binary32 exp2 / log2 behind the mixed-precision rounding
bounds (lingam_check_terms): over every binary32 argument of the ranges the
per-sample terms use, their largest error must lie within the constants the
worst-case bound T_err_bound assumes, and their largest mean error within a
binade within the constants the probable bound T_err_prob assumes
(include/lingam.h: LINGAM_EXP2_ERR, LINGAM_LOG2_ERR, LINGAM_EXP2_BIAS,
LINGAM_LOG2_BIAS)."""
import os
import re

import pytest

import paper_2109_13993_amd as lg

pytestmark = pytest.mark.gpu

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lingam.h")


def _constant(name):
    m = re.search(r"#define\s+%s\s+([0-9.eE+-]+)" % name, open(HEADER).read())
    return float(m.group(1))


def test_hardware_exp2_log2_within_the_bound_constants():
    r = lg.check_terms()
    print("v_exp_f32 on [-126, 0]: max %.3f u32, mean %.4f u32, largest binade mean %.4f u32; "
          "v_log_f32 on [1, 2]: max %.3f u32, mean %.4f u32" % (
              r["exp2_max_rel"], r["exp2_mean_rel"], r["exp2_max_binade_mean"], r["log2_max_abs"],
              r["log2_mean_abs"]), flush=True)
    assert r["exp2_count"] == 0x42FC0000 + 1 and r["log2_count"] == (1 << 23) + 1
    assert r["exp2_max_rel"] <= _constant("LINGAM_EXP2_ERR")
    assert r["log2_max_abs"] <= _constant("LINGAM_LOG2_ERR")
    assert r["exp2_max_binade_mean"] <= _constant("LINGAM_EXP2_BIAS")
    assert abs(r["log2_mean_abs"]) <= _constant("LINGAM_LOG2_BIAS")
