"""Host-side checks of the C ABI (no GPU needed, no device work issued):
the library loads, exports every function include/lingam.h declares, the
ctypes mirrors of the structs match the C layout, and invalid arguments are
rejected before any device call."""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

import paper_2109_13993_amd as lg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lingam.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lingam_[A-Za-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lg.LIB_PATH):
        pytest.fail("liblingam.so is not built (run __graft_entry__.build())")
    return lg.load_library()


def test_library_exports_every_declared_function(lib):
    declared = _declared_functions()
    assert set(declared) == set(lg.SYMBOLS)
    for name in declared:
        assert hasattr(lib, name), name
    nm = subprocess.run(["nm", "-D", "--defined-only", lg.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (lingam_\w+)", nm))
    assert set(declared) <= exported


def _c_layout():
    src = r"""
#include <stddef.h>
#include <stdio.h>
#include "lingam.h"
#define F(T, f) printf(#T " " #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("lingam_opts size %zu\n", sizeof(lingam_opts));
  printf("lingam_result size %zu\n", sizeof(lingam_result));
  printf("lingam_dataset size %zu\n", sizeof(lingam_dataset));
FIELDS
  return 0;
}
"""
    fields = []
    for T, cls in (("lingam_opts", lg.LingamOpts), ("lingam_result", lg.LingamResult),
                   ("lingam_dataset", lg.LingamDataset)):
        for f, _ in cls._fields_:
            fields.append("  F(%s, %s)" % (T, f))
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(src.replace("FIELDS", "\n".join(fields), 1))
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    res = {}
    for line in out.splitlines():
        a, b, v = line.split()
        res[(a, b)] = int(v)
    return res


def test_struct_layout_matches_header():
    lay = _c_layout()
    for T, cls in (("lingam_opts", lg.LingamOpts), ("lingam_result", lg.LingamResult),
                   ("lingam_dataset", lg.LingamDataset)):
        assert lay[(T, "size")] == ctypes.sizeof(cls), T
        for f, _ in cls._fields_:
            assert lay[(T, f)] == getattr(cls, f).offset, (T, f)


def test_defaults_and_status_strings(lib):
    o = lg.default_opts()
    assert o.struct_size == ctypes.sizeof(lg.LingamOpts)
    assert o.use_threshold == 1 and o.precision == 0 and o.cov_refresh_every == -1
    assert o.gamma0 == 0.0 and o.gamma_mult == 4.0
    for s in range(7):
        assert len(lg.status_string(s)) > 0
    assert lg.workspace_size(20000, 500) > 2 * 500 * 20000 * 8
    assert lg.workspace_size(1, 5) == 0


def _call(X, n, p, opts=None, order=True, M=None):
    lib = lg.load_library()
    o = opts if opts is not None else lg.default_opts()
    res = lg.LingamResult()
    buf = np.zeros(max(p, 1), dtype=np.int32)
    if order:
        res.order = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    if M is not None:
        res.M = M.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    ptr = ctypes.c_void_p(X.ctypes.data) if X is not None else None
    return lib.lingam_fit_order(ptr, n, p, ctypes.byref(o), ctypes.byref(res)), lib.lingam_last_error().decode()


def test_invalid_arguments_rejected_before_device_work(lib):
    X = np.zeros((4, 10))
    assert _call(None, 10, 4)[0] == lg.E_INVALID
    assert _call(X, 10, 4, order=False)[0] == lg.E_INVALID
    assert _call(X, 1, 4)[0] == lg.E_INVALID
    assert _call(X, 10, 0)[0] == lg.E_INVALID
    o = lg.default_opts(); o.struct_size = 3
    st, msg = _call(X, 10, 4, o)
    assert st == lg.E_INVALID and "struct_size" in msg
    o = lg.default_opts(); o.precision = 7
    assert _call(X, 10, 4, o)[0] == lg.E_INVALID
    o = lg.default_opts(); o.chunk_samples = 100
    assert _call(X, 10, 4, o)[0] == lg.E_INVALID
    o = lg.default_opts(); o.record_M_iters = 1
    assert _call(X, 10, 4, o)[0] == lg.E_INVALID  # no M buffer
    for forced in ([0, 0], [5], [-1]):
        o, keep = lg._make_opts(forced_order=forced)
        st, msg = _call(X, 10, 4, o)
        assert st == lg.E_INVALID and "forced" in msg


def test_baseline_pair_strategies_validated_before_device_work(lib):
    # the paper's baseline mappings (ablation variants) evaluate every ordered
    # pair in FP64: the threshold, messaging and the binary32 modes are refused
    X = np.zeros((4, 10))
    for strategy in (1, 2, 3):
        o = lg.default_opts(); o.pair_strategy = strategy
        st, msg = _call(X, 10, 4, o)                         # threshold and messaging on
        assert st == lg.E_INVALID and "pair_strategy" in msg
        o.use_threshold = 0
        assert _call(X, 10, 4, o)[0] == lg.E_INVALID       # messaging still on
        o.messaging = 0; o.precision = lg.PREC["mixed"]
        assert _call(X, 10, 4, o)[0] == lg.E_INVALID
    for bad in (-1, 4):
        o = lg.default_opts(); o.pair_strategy = bad
        st, msg = _call(X, 10, 4, o)
        assert st == lg.E_INVALID and "pair_strategy" in msg


def test_batch_entry_point_reports_status(lib):
    res = (lg.LingamResult * 1)()
    st = lib.lingam_fit_order_batch(0, None, None, res)
    assert st == lg.E_INVALID


def _batch_call(lib, sets_py, opts=None):
    """Call lingam_fit_order_batch on host arrays (validation only: every call
    here is rejected before any device work)."""
    count = len(sets_py)
    sets = (lg.LingamDataset * count)()
    outs = (lg.LingamResult * count)()
    orders = []
    for k, (X, idx) in enumerate(sets_py):
        sets[k].X = ctypes.c_void_p(X.ctypes.data) if X is not None else None
        sets[k].p, sets[k].n = X.shape if X is not None else (3, 10)
        if idx is not None:
            sets[k].sample_idx = idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            sets[k].n_idx = idx.size
        orders.append(np.zeros(sets[k].p, dtype=np.int32))
        outs[k].order = orders[-1].ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    o = opts if opts is not None else lg.default_opts()
    return lib.lingam_fit_order_batch(count, sets, ctypes.byref(o), outs)


def test_batch_validation(lib):
    X = np.zeros((3, 10))
    assert _batch_call(lib, [(None, None)]) == lg.E_INVALID                       # NULL X
    assert _batch_call(lib, [(X, np.array([0, 10], dtype=np.int64))]) == lg.E_INVALID   # index >= n
    assert _batch_call(lib, [(X, np.array([-1, 2], dtype=np.int64))]) == lg.E_INVALID   # index < 0
    assert _batch_call(lib, [(X, np.array([1], dtype=np.int64))]) == lg.E_INVALID       # n_idx < 2
    o = lg.default_opts()
    o.x_dtype = 1
    assert _batch_call(lib, [(X, np.array([0, 1, 2], dtype=np.int64))], o) == lg.E_UNSUPPORTED
    o = lg.default_opts()
    o.record_M_iters = 1
    assert _batch_call(lib, [(X, None)], o) == lg.E_UNSUPPORTED
    keep = np.array([0, 1], dtype=np.int32)
    o = lg.default_opts()
    o.forced_order = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    o.forced_len = 2
    assert _batch_call(lib, [(X, None)], o) == lg.E_UNSUPPORTED


def test_workspace_size_is_consistent(lib):
    # the size comes from the same layout code as the call itself: a batch of
    # one data set needs what the single call needs plus the work queue's
    # list of sets, and the size grows with the options that add buffers
    X = np.zeros((30, 5000))
    o = lg.default_opts()
    single = lib.lingam_workspace_size(5000, 30, ctypes.byref(o))
    sets = (lg.LingamDataset * 1)()
    sets[0].X = ctypes.c_void_p(X.ctypes.data)
    sets[0].p, sets[0].n = X.shape
    batch1 = lib.lingam_workspace_size_batch(1, sets, ctypes.byref(o))
    assert single < batch1 <= single + 512
    o.x_on_device = 1
    dev = lib.lingam_workspace_size(5000, 30, ctypes.byref(o))
    assert dev < single and single - dev >= 30 * 5000 * 8
    o.record_M_iters = 3
    assert lib.lingam_workspace_size(5000, 30, ctypes.byref(o)) >= dev + 3 * 30 * 30 * 8
    assert lib.lingam_workspace_size_batch(0, sets, ctypes.byref(o)) == 0


def test_too_small_workspace_rejected_before_device_work(lib):
    # the workspace is checked on the host: a pointer that is never
    # dereferenced (no device work is issued) gives NOMEM or INVALID
    X = np.zeros((4, 300))
    need = lib.lingam_workspace_size(300, 4, None)
    o = lg.default_opts()
    o.workspace = ctypes.c_void_p(1 << 40)
    o.workspace_bytes = need - 1
    st, msg = _call(X, 300, 4, o)
    assert st == lg.E_NOMEM and str(need) in msg
    o.workspace = ctypes.c_void_p((1 << 40) + 64)     # not 256-byte aligned
    o.workspace_bytes = need
    st, msg = _call(X, 300, 4, o)
    assert st == lg.E_INVALID and "aligned" in msg
    o = lg.default_opts()
    o.workspace = ctypes.c_void_p(1 << 40)
    o.workspace_bytes = 16
    assert _batch_call(lib, [(np.zeros((3, 10)), None)], o) == lg.E_NOMEM
