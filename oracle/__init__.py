"""FP64 CPU oracle for the DirectLiNGAM causal-order search (ParaLiNGAM,
arXiv 2109.13993, Alg. 1-2, Eq. (Itest) and Eq. (HApp)).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and
the CPU-baseline leg of the benchmark.  The GPU library never imports it.
All functions take and return numpy float64 arrays; row i of X holds the n
samples of variable i (the paper's p x n data layout).
"""
import ctypes
import os

import numpy as np

from . import build as _build

OK, E_INVALID, E_NONFINITE, E_DEGENERATE, E_NOMEM = 0, 1, 2, 3, 4
STATUS_NAMES = {0: "ok", 1: "invalid", 2: "nonfinite", 3: "degenerate", 4: "nomem"}

_lib = None


class OracleError(RuntimeError):
    def __init__(self, status, bad_i=-1, bad_j=-1):
        super().__init__("oracle status %s (bad_i=%d bad_j=%d)" %
                         (STATUS_NAMES.get(status, status), bad_i, bad_j))
        self.status, self.bad_i, self.bad_j = status, bad_i, bad_j


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = _build.LIB
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
        _build.build(force=True)
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    i64, i32 = ctypes.c_int64, ctypes.c_int32
    lib.oracle_entropy.restype = ctypes.c_double
    lib.oracle_entropy.argtypes = [dp, i64]
    lib.oracle_entropy_moments.restype = None
    lib.oracle_entropy_moments.argtypes = [dp, i64, dp, dp]
    lib.oracle_standardize.restype = ctypes.c_int
    lib.oracle_standardize.argtypes = [dp, i64, dp]
    lib.oracle_compare.restype = ctypes.c_int
    lib.oracle_compare.argtypes = [dp, dp, i64, dp]
    lib.oracle_fit_order.restype = ctypes.c_int
    lib.oracle_fit_order.argtypes = [dp, i64, i64, i32, ip, i32, i32, ip, dp, dp, dp, dp, i32, ip, ip, i32]
    lib.oracle_sampled_at.restype = ctypes.c_int
    lib.oracle_sampled_at.argtypes = [dp, i64, i64, ip, i32, ip, i32, dp, ip, ip, i32, dp, dp, i32]
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def entropy(u):
    """Eq. (HApp) of a (standardized) sample."""
    u = _f64(u)
    return _load().oracle_entropy(_dp(u), u.size)


def entropy_moments(u):
    """(E[log cosh u], E[u exp(-u^2/2)]) of a sample, the two moments of Eq. (HApp)."""
    u = _f64(u)
    e1, e2 = ctypes.c_double(), ctypes.c_double()
    _load().oracle_entropy_moments(_dp(u), u.size, ctypes.byref(e1), ctypes.byref(e2))
    return e1.value, e2.value


def standardize(x):
    """Row normalisation: subtract the mean, divide by the (n-1) standard deviation."""
    x = _f64(x)
    z = np.empty_like(x)
    st = _load().oracle_standardize(_dp(x), x.size, _dp(z))
    if st != OK:
        raise OracleError(st)
    return z


def compare(xi, xj):
    """The likelihood-ratio test I(x_i, x_j, r_i^(j), r_j^(i)) of Eq. (Itest)."""
    xi, xj = _f64(xi), _f64(xj)
    assert xi.shape == xj.shape and xi.ndim == 1
    out = ctypes.c_double()
    st = _load().oracle_compare(_dp(xi), _dp(xj), xi.size, ctypes.byref(out))
    if st != OK:
        raise OracleError(st)
    return out.value


def fit_order(X, max_roots=0, forced_order=None, nthreads=0, M_iters=0, want_T=True, pair_once=False):
    """Plain DirectLiNGAM causal-order search (Alg. 1 without the estimate of B, Alg. 2).

    Returns dict(order=int32[p] (-1 past the last root), T=float64[p,p] or None
    (T[t, v] = -S_v at iteration t, NaN if v is not in U_t), H=float64[p,p] or None
    (H[t, v] = entropy estimate of normalised x_v at iteration t),
    M=float64[M_iters,p,p] or None, B=float64[M_iters,p,p] or None: the correlation of
    each normalised pair, i.e. its regression coefficient).  Raises OracleError on
    invalid/degenerate input.  pair_once=True evaluates each unordered pair once
    and takes the reverse test as its exact negation (messaging, Sec. 3.1):
    bitwise the same outputs in half the time, for the large fixtures.
    """
    X = _f64(X)
    p, n = X.shape
    order = np.full(p, -1, dtype=np.int32)
    T = np.full((p, p), np.nan) if want_T else None
    H = np.full((p, p), np.nan) if want_T else None
    M = np.full((M_iters, p, p), np.nan) if M_iters > 0 else None
    B = np.full((M_iters, p, p), np.nan) if M_iters > 0 else None
    fo = np.ascontiguousarray(forced_order if forced_order is not None else [], dtype=np.int32)
    bi, bj = ctypes.c_int32(-1), ctypes.c_int32(-1)
    st = _load().oracle_fit_order(
        _dp(X), n, p, int(max_roots), _ip(fo) if fo.size else None, int(fo.size), int(nthreads),
        _ip(order), _dp(T) if T is not None else None, _dp(H) if H is not None else None,
        _dp(M) if M is not None else None, _dp(B) if B is not None else None,
        int(M_iters), ctypes.byref(bi), ctypes.byref(bj), int(bool(pair_once)))
    if st != OK:
        raise OracleError(st, bi.value, bj.value)
    return {"order": order, "T": T, "H": H, "M": M, "B": B}


def sampled_at(X, prefix, t, vars=(), pairs=(), nthreads=0, with_corr=False):
    """Scores and tests at iteration t after following the root prefix[:t].

    Returns (T for each v in vars, I for each ordered pair in pairs); with
    with_corr=True also the correlation of each pair.
    """
    X = _f64(X)
    p, n = X.shape
    pre = np.ascontiguousarray(list(prefix)[:t], dtype=np.int32)
    va = np.ascontiguousarray(list(vars), dtype=np.int32)
    pr = np.asarray(list(pairs), dtype=np.int32).reshape(-1, 2)
    pi, pj = np.ascontiguousarray(pr[:, 0]), np.ascontiguousarray(pr[:, 1])
    T = np.full(va.size, np.nan)
    M = np.full(pi.size, np.nan)
    Bc = np.full(pi.size, np.nan)
    st = _load().oracle_sampled_at(
        _dp(X), n, p, _ip(pre) if pre.size else None, int(t), _ip(va) if va.size else None,
        int(va.size), _dp(T), _ip(pi) if pi.size else None, _ip(pj) if pj.size else None,
        int(pi.size), _dp(M), _dp(Bc), int(nthreads))
    if st != OK:
        raise OracleError(st)
    return (T, M, Bc) if with_corr else (T, M)


def estimate_B(X, order):
    """Alg. 1, last step: the causal strengths B from a causal order K, by
    plain least squares -- each variable regressed (with an intercept) on all
    variables before it in K (Sec. 2.3: covariance-based regression along the
    recovered order).  Returns B (p x p, float64) with B[i, j] the
    coefficient of x_j in the regression of x_i, zero where x_j does not
    precede x_i.  numpy's least-squares solver serves as the regression."""
    X = _f64(X)
    p, n = X.shape
    order = [int(v) for v in order]
    assert sorted(order) == list(range(p)), "order must be a permutation"
    B = np.zeros((p, p))
    ones = np.ones((n, 1))
    for t in range(1, p):
        i, pred = order[t], order[:t]
        A = np.hstack([X[pred].T, ones])
        coef, *_ = np.linalg.lstsq(A, X[i], rcond=None)
        B[i, pred] = coef[:-1]
    return B
