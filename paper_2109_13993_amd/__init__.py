"""MI355X (gfx950) DirectLiNGAM causal-order search.

Thin ctypes binding over the C ABI declared in include/lingam.h; every step of
the search runs in the HIP library liblingam.so.  This module only marshals
arguments.  There is no CPU fallback: if the library is not built, calls
raise RuntimeError.

    from paper_2109_13993_amd import fit_order
    res = fit_order(X)            # X: p x n numpy array or torch tensor (row = variable)
    res.order                     # causal order, roots first
"""
import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblingam.so")

OK, E_INVALID, E_NONFINITE, E_DEGENERATE, E_NOMEM, E_DEVICE, E_UNSUPPORTED = range(7)
PREC = {"fp64": 0, "mixed": 1, "fp32": 1, "fp32_storage": 2}
LAYOUT = {"var_major": 0, "sample_major": 1}
PAIR_STRATEGY = {"default": 0, "block_worker": 1, "thread_worker": 2, "block_compare": 3}

# Exported symbols of the C ABI (kept in sync with include/lingam.h).
SYMBOLS = ("lingam_opts_default", "lingam_fit_order", "lingam_fit_order_noalloc", "lingam_fit_order_batch",
           "lingam_workspace_size", "lingam_workspace_size_batch", "lingam_estimate_B", "lingam_check_terms",
           "lingam_status_string", "lingam_last_error")


class LingamOpts(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("precision", ctypes.c_int32),
        ("layout", ctypes.c_int32),
        ("x_dtype", ctypes.c_int32),
        ("x_on_device", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("use_threshold", ctypes.c_int32),
        ("gamma0", ctypes.c_double),
        ("gamma_mult", ctypes.c_double),
        ("cov_refresh_every", ctypes.c_int32),
        ("max_roots", ctypes.c_int32),
        ("forced_order", ctypes.POINTER(ctypes.c_int32)),
        ("forced_len", ctypes.c_int32),
        ("record_M_iters", ctypes.c_int32),
        ("band_blocks", ctypes.c_int32),
        ("chunk_samples", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("profile", ctypes.c_int32),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_uint64),
        ("estimate_B", ctypes.c_int32),
        ("batch_queue", ctypes.c_int32),
        ("graph", ctypes.c_int32),
        ("band_target", ctypes.c_double),
        ("first_band_blocks", ctypes.c_int32),
        ("messaging", ctypes.c_int32),
        ("pair_strategy", ctypes.c_int32),
    ]


class LingamResult(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.POINTER(ctypes.c_int32)),
        ("T", ctypes.POINTER(ctypes.c_double)),
        ("T_state", ctypes.POINTER(ctypes.c_uint8)),
        ("H", ctypes.POINTER(ctypes.c_double)),
        ("M", ctypes.POINTER(ctypes.c_double)),
        ("T_err_bound", ctypes.POINTER(ctypes.c_double)),
        ("B", ctypes.POINTER(ctypes.c_double)),
        ("T_err_prob", ctypes.POINTER(ctypes.c_double)),
        ("pairs_evaluated", ctypes.c_uint64),
        ("pair_samples", ctypes.c_uint64),
        ("pairs_computed", ctypes.c_uint64),
        ("threshold_rounds", ctypes.c_uint64),
        ("bands", ctypes.c_uint64),
        ("seconds_total", ctypes.c_double),
        ("seconds_device", ctypes.c_double),
        ("seconds_pair_kernel", ctypes.c_double),
        ("pair_kernel_launches", ctypes.c_uint64),
        ("iterations", ctypes.c_int32),
        ("bad_i", ctypes.c_int32),
        ("bad_j", ctypes.c_int32),
        ("status", ctypes.c_int32),
    ]


class LingamDataset(ctypes.Structure):
    _fields_ = [
        ("X", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("p", ctypes.c_int64),
        ("sample_idx", ctypes.POINTER(ctypes.c_int64)),
        ("n_idx", ctypes.c_int64),
    ]


class LingamTermCheck(ctypes.Structure):
    _fields_ = [
        ("exp2_max_rel", ctypes.c_double),
        ("exp2_mean_rel", ctypes.c_double),
        ("exp2_max_binade_mean", ctypes.c_double),
        ("log2_max_abs", ctypes.c_double),
        ("log2_mean_abs", ctypes.c_double),
        ("exp2_count", ctypes.c_uint64),
        ("log2_count", ctypes.c_uint64),
    ]


class LingamError(RuntimeError):
    def __init__(self, status, message, bad_i=-1, bad_j=-1):
        super().__init__("lingam status %d: %s" % (status, message))
        self.status, self.bad_i, self.bad_j = status, bad_i, bad_j


_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblingam.so (raises RuntimeError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("liblingam.so not found at %s; build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'` or "
                           "`python paper_2109_13993_amd/build.py`" % path)
    lib = ctypes.CDLL(path)
    lib.lingam_opts_default.restype = None
    lib.lingam_opts_default.argtypes = [ctypes.POINTER(LingamOpts)]
    lib.lingam_fit_order.restype = ctypes.c_int
    lib.lingam_fit_order.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.POINTER(LingamOpts), ctypes.POINTER(LingamResult)]
    lib.lingam_fit_order_noalloc.restype = ctypes.c_int
    lib.lingam_fit_order_noalloc.argtypes = lib.lingam_fit_order.argtypes
    lib.lingam_fit_order_batch.restype = ctypes.c_int
    lib.lingam_fit_order_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(LingamDataset),
                                           ctypes.POINTER(LingamOpts), ctypes.POINTER(LingamResult)]
    lib.lingam_workspace_size.restype = ctypes.c_uint64
    lib.lingam_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(LingamOpts)]
    lib.lingam_workspace_size_batch.restype = ctypes.c_uint64
    lib.lingam_workspace_size_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(LingamDataset),
                                                ctypes.POINTER(LingamOpts)]
    lib.lingam_estimate_B.restype = ctypes.c_int
    lib.lingam_estimate_B.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(LingamOpts),
                                      ctypes.POINTER(ctypes.c_double)]
    lib.lingam_check_terms.restype = ctypes.c_int
    lib.lingam_check_terms.argtypes = [ctypes.c_int32, ctypes.POINTER(LingamTermCheck)]
    lib.lingam_status_string.restype = ctypes.c_char_p
    lib.lingam_status_string.argtypes = [ctypes.c_int]
    lib.lingam_last_error.restype = ctypes.c_char_p
    lib.lingam_last_error.argtypes = []
    _lib = lib
    return lib


@dataclass
class FitResult:
    order: np.ndarray                 # [p] int32, -1 past the last root
    T: Optional[np.ndarray] = None    # [p, p] float64, T[t, v] = -S_v at iteration t
    T_state: Optional[np.ndarray] = None  # [p, p] uint8 (0 absent, 1 complete, 2 pruned)
    H: Optional[np.ndarray] = None    # [p, p] entropy of v at iteration t
    M: Optional[np.ndarray] = None    # [k, p, p] test matrices of the first k iterations
    T_err: Optional[np.ndarray] = None  # [p, p] rounding bound of T (mixed; 0 in FP64 mode)
    B: Optional[np.ndarray] = None    # [p, p] causal strengths (estimate_B), B[i, j] = effect of x_j on x_i
    T_err_prob: Optional[np.ndarray] = None  # [p, p] probable rounding bound of T (mixed modes)
    pairs_evaluated: int = 0
    pair_samples: int = 0
    pairs_computed: int = 0
    threshold_rounds: int = 0
    bands: int = 0
    seconds_total: float = 0.0
    seconds_device: float = 0.0
    seconds_pair_kernel: float = 0.0
    pair_kernel_launches: int = 0
    iterations: int = 0
    extra: dict = field(default_factory=dict)


def default_opts() -> LingamOpts:
    o = LingamOpts()
    load_library().lingam_opts_default(ctypes.byref(o))
    return o


def _make_opts(precision="fp64", use_threshold=True, gamma0=0.0, gamma_mult=0.0,
               cov_refresh_every=None, max_roots=0, forced_order=None, record_M_iters=0,
               band_blocks=0, chunk_samples=0, layout="var_major", device=-1, profile=False):
    o = default_opts()
    o.precision = PREC[precision]
    o.layout = LAYOUT[layout]
    o.use_threshold = 1 if use_threshold else 0
    o.gamma0 = float(gamma0)
    o.gamma_mult = float(gamma_mult)
    if cov_refresh_every is not None:
        o.cov_refresh_every = int(cov_refresh_every)
    o.max_roots = int(max_roots)
    o.record_M_iters = int(record_M_iters)
    o.band_blocks = int(band_blocks)
    o.chunk_samples = int(chunk_samples)
    o.device = int(device)
    o.profile = 1 if profile else 0
    keep = None
    if forced_order is not None and len(forced_order) > 0:
        keep = np.ascontiguousarray(forced_order, dtype=np.int32)
        o.forced_order = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        o.forced_len = keep.size
    return o, keep


def _apply_tuned(o, kind, precision, p, n, queue=None, graph=None):
    """Fill the launch parameters the caller left at their defaults from the
    autotuner's entry for this device and problem bucket, if any."""
    from . import autotune
    t = autotune.lookup(kind, precision, p, n)
    if not t:
        return
    if o.chunk_samples == 0 and "chunk_samples" in t:
        o.chunk_samples = int(t["chunk_samples"])
    if o.band_blocks == 0 and o.first_band_blocks == 0 and "first_band_blocks" in t:
        o.first_band_blocks = int(t["first_band_blocks"])
    if o.band_target == 0.0 and "band_target" in t:
        o.band_target = float(t["band_target"])
    if o.gamma_mult == 0.0 and "gamma_mult" in t:
        o.gamma_mult = float(t["gamma_mult"])
    if queue is None and "batch_queue" in t:
        o.batch_queue = int(t["batch_queue"])
    if graph is None and "graph" in t and o.workspace:
        o.graph = int(t["graph"])


def fit_order(X, precision: str = "fp64", use_threshold: bool = True, gamma0: float = 0.0,
              gamma_mult: float = 0.0, cov_refresh_every=None, max_roots: int = 0,
              forced_order=None, record_M_iters: int = 0, want_T: bool = True,
              want_H: bool = True, band_blocks: int = 0, chunk_samples: int = 0,
              layout: str = "var_major", stream=None, profile: bool = False,
              workspace=None, noalloc: bool = False, estimate_B: bool = False,
              band_target: float = 0.0, first_band_blocks: int = 0, tune: bool = True,
              messaging: bool = True, pair_strategy: str = "default") -> FitResult:
    """Causal order of the variables of X (lingam_fit_order).

    X is a p x n array (row i = samples of variable i; layout="sample_major"
    for n x p) of float64 or float32: a numpy array (copied to the device by the
    library) or a torch tensor (a CUDA/HIP tensor is used in place on its
    device and on `stream`, default the current torch stream).
    workspace: optional device tensor (e.g. torch.empty(nbytes, dtype=torch.uint8,
    device="cuda")) that the call carves its device buffers from
    (workspace_size() bytes at least).
    noalloc: call lingam_fit_order_noalloc, which carves every buffer from the
    library's fixed per-GPU device array and allocates nothing.
    estimate_B: also estimate the causal strengths B from the order (result.B).
    pair_strategy: "default", or one of the paper's baseline mappings of the
    tests (Sec. 5.3) kept as ablations -- "block_worker", "thread_worker",
    "block_compare" -- which need precision="fp64", use_threshold=False and
    messaging=False.
    band_target / chunk_samples / band_blocks: launch tuning (never changes a
    result); left at 0 they take the autotuner's entry for this device and
    problem bucket when there is one (tune=True), else the library defaults.
    """
    lib = load_library()
    o, keep = _make_opts(precision, use_threshold, gamma0, gamma_mult, cov_refresh_every,
                         max_roots, forced_order, record_M_iters, band_blocks, chunk_samples, layout,
                         profile=profile)
    if workspace is not None:
        o.workspace = ctypes.c_void_p(workspace.data_ptr())
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    o.estimate_B = 1 if estimate_B else 0
    is_torch = type(X).__module__.startswith("torch")
    if is_torch:
        import torch
        if X.dtype not in (torch.float64, torch.float32):
            raise TypeError("X must be float64 or float32")
        X = X.contiguous()
        ptr = X.data_ptr()
        o.x_dtype = 0 if X.dtype == torch.float64 else 1
        if X.is_cuda:
            o.x_on_device = 1
            o.device = X.device.index if X.device.index is not None else torch.cuda.current_device()
            s = stream if stream is not None else torch.cuda.current_stream(X.device)
            o.stream = ctypes.c_void_p(s.cuda_stream if hasattr(s, "cuda_stream") else int(s))
        shape = tuple(X.shape)
        host_ref = X
    else:
        arr = np.asarray(X)
        if arr.dtype not in (np.float64, np.float32):
            arr = arr.astype(np.float64)
        arr = np.ascontiguousarray(arr)
        o.x_dtype = 0 if arr.dtype == np.float64 else 1
        ptr = arr.ctypes.data
        shape = arr.shape
        host_ref = arr
        if stream is not None:
            o.stream = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    if len(shape) != 2:
        raise ValueError("X must be 2-D")
    p, n = (shape[0], shape[1]) if layout == "var_major" else (shape[1], shape[0])
    o.band_target = float(band_target)
    o.first_band_blocks = int(first_band_blocks)
    o.messaging = 1 if messaging else 0
    o.pair_strategy = PAIR_STRATEGY[pair_strategy]
    if tune:
        _apply_tuned(o, "single", precision, p, n)
    order = np.full(p, -1, dtype=np.int32)
    T = np.full((p, p), np.nan) if want_T else None
    Ts = np.zeros((p, p), dtype=np.uint8) if want_T else None
    H = np.full((p, p), np.nan) if want_H else None
    Terr = np.full((p, p), np.nan) if want_T else None
    Terrp = np.full((p, p), np.nan) if want_T else None
    M = np.full((record_M_iters, p, p), np.nan) if record_M_iters > 0 else None
    Bm = np.full((p, p), np.nan) if estimate_B else None
    res = LingamResult()
    res.order = order.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    if T is not None:
        res.T = T.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        res.T_state = Ts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    if H is not None:
        res.H = H.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if Terr is not None:
        res.T_err_bound = Terr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        res.T_err_prob = Terrp.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if M is not None:
        res.M = M.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if Bm is not None:
        res.B = Bm.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    entry = lib.lingam_fit_order_noalloc if noalloc else lib.lingam_fit_order
    st = entry(ctypes.c_void_p(ptr), n, p, ctypes.byref(o), ctypes.byref(res))
    del host_ref, keep
    if st != OK:
        raise LingamError(st, lib.lingam_last_error().decode(), res.bad_i, res.bad_j)
    return FitResult(order=order, T=T, T_state=Ts, H=H, M=M, T_err=Terr, B=Bm, T_err_prob=Terrp,
                     pairs_evaluated=res.pairs_evaluated, pair_samples=res.pair_samples,
                     pairs_computed=res.pairs_computed, threshold_rounds=res.threshold_rounds,
                     bands=res.bands, seconds_total=res.seconds_total,
                     seconds_device=res.seconds_device, seconds_pair_kernel=res.seconds_pair_kernel,
                     pair_kernel_launches=res.pair_kernel_launches, iterations=res.iterations)


def fit_order_batch(datasets, precision: str = "fp64", use_threshold: bool = True, gamma0: float = 0.0,
                    gamma_mult: float = 0.0, cov_refresh_every=None, max_roots: int = 0,
                    band_blocks: int = 0, chunk_samples: int = 0, want_T: bool = True,
                    want_H: bool = False, profile: bool = False, stream=None, queue=None,
                    workspace=None, graph=None, band_target: float = 0.0, first_band_blocks: int = 0,
                    tune: bool = True):
    """Causal orders of many data sets in one batched search (lingam_fit_order_batch).

    `datasets` is a list whose items are either a p x n array (numpy, float64
    or float32; all of one dtype) or a tuple (base, sample_idx): a bootstrap
    resample of the columns of the float64 p x n array `base` (the same base
    object may be shared by many items; it is uploaded once).  Returns a list
    of FitResult; a data set that failed has extra["status"] != 0.
    """
    lib = load_library()
    o, _ = _make_opts(precision, use_threshold, gamma0, gamma_mult, cov_refresh_every, max_roots,
                      None, 0, band_blocks, chunk_samples, profile=profile)
    o.band_target = float(band_target)
    o.first_band_blocks = int(first_band_blocks)
    if workspace is not None:
        o.workspace = ctypes.c_void_p(workspace.data_ptr())
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    if tune:
        from . import autotune
        _apply_tuned(o, "batch", precision, *autotune.batch_shape(datasets), queue=queue, graph=graph)
    if queue is not None:
        o.batch_queue = 1 if queue else 0
    if graph is not None:
        o.graph = 1 if graph else 0
    if stream is not None:
        o.stream = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    count = len(datasets)
    sets = (LingamDataset * count)()
    outs = (LingamResult * count)()
    keep, results = [], []
    dtype = None
    for k, item in enumerate(datasets):
        if isinstance(item, tuple):
            base, idx = item
            base = np.ascontiguousarray(base, dtype=np.float64)
            idx = np.ascontiguousarray(idx, dtype=np.int64)
            keep += [base, idx]
            sets[k].X = ctypes.c_void_p(base.ctypes.data)
            sets[k].p, sets[k].n = base.shape
            sets[k].sample_idx = idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            sets[k].n_idx = idx.size
            p = base.shape[0]
        else:
            arr = np.asarray(item)
            if arr.dtype not in (np.float64, np.float32):
                arr = arr.astype(np.float64)
            arr = np.ascontiguousarray(arr)
            if dtype is None:
                dtype = arr.dtype
            elif arr.dtype != dtype:
                raise TypeError("all data sets of a batch must have one dtype")
            keep.append(arr)
            sets[k].X = ctypes.c_void_p(arr.ctypes.data)
            sets[k].p, sets[k].n = arr.shape
            p = arr.shape[0]
        r = dict(order=np.full(p, -1, dtype=np.int32),
                 T=np.full((p, p), np.nan) if want_T else None,
                 T_state=np.zeros((p, p), dtype=np.uint8) if want_T else None,
                 H=np.full((p, p), np.nan) if want_H else None,
                 T_err=np.full((p, p), np.nan) if want_T else None,
                 T_err_prob=np.full((p, p), np.nan) if want_T else None)
        outs[k].order = r["order"].ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        if want_T:
            outs[k].T = r["T"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            outs[k].T_state = r["T_state"].ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
            outs[k].T_err_bound = r["T_err"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            outs[k].T_err_prob = r["T_err_prob"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if want_H:
            outs[k].H = r["H"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        results.append(r)
    o.x_dtype = 1 if dtype == np.float32 else 0
    st = lib.lingam_fit_order_batch(count, sets, ctypes.byref(o), outs)
    if st != OK and all(outs[k].status == OK for k in range(count)):
        raise LingamError(st, lib.lingam_last_error().decode())
    del keep
    res = []
    for k, r in enumerate(results):
        out = outs[k]
        res.append(FitResult(order=r["order"], T=r["T"], T_state=r["T_state"], H=r["H"], T_err=r["T_err"],
                             T_err_prob=r["T_err_prob"],
                             pairs_evaluated=out.pairs_evaluated, pair_samples=out.pair_samples,
                             pairs_computed=out.pairs_computed, threshold_rounds=out.threshold_rounds,
                             bands=out.bands, seconds_total=out.seconds_total,
                             seconds_device=out.seconds_device,
                             seconds_pair_kernel=out.seconds_pair_kernel,
                             pair_kernel_launches=out.pair_kernel_launches, iterations=out.iterations,
                             extra={"status": out.status, "bad_i": out.bad_i, "bad_j": out.bad_j}))
    return res


def estimate_B(X, order, precision: str = "fp64", layout: str = "var_major", stream=None) -> np.ndarray:
    """Causal strengths B of X along a causal order (lingam_estimate_B): each
    variable regressed by least squares on every variable before it in
    `order`.  Returns B (p x p float64), B[i, j] = coefficient of x_j for x_i."""
    lib = load_library()
    o, _ = _make_opts(precision, layout=layout)
    is_torch = type(X).__module__.startswith("torch")
    if is_torch:
        import torch
        X = X.contiguous()
        o.x_dtype = 0 if X.dtype == torch.float64 else 1
        ptr, shape, keep = X.data_ptr(), tuple(X.shape), X
        if X.is_cuda:
            o.x_on_device = 1
            o.device = X.device.index if X.device.index is not None else torch.cuda.current_device()
            s = stream if stream is not None else torch.cuda.current_stream(X.device)
            o.stream = ctypes.c_void_p(s.cuda_stream if hasattr(s, "cuda_stream") else int(s))
    else:
        keep = np.ascontiguousarray(X if np.asarray(X).dtype in (np.float64, np.float32)
                                    else np.asarray(X, dtype=np.float64))
        o.x_dtype = 0 if keep.dtype == np.float64 else 1
        ptr, shape = keep.ctypes.data, keep.shape
    p, n = (shape[0], shape[1]) if layout == "var_major" else (shape[1], shape[0])
    K = np.ascontiguousarray(order, dtype=np.int32)
    B = np.full((p, p), np.nan)
    st = lib.lingam_estimate_B(ctypes.c_void_p(ptr), n, p, K.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               ctypes.byref(o), B.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    del keep
    if st != OK:
        raise LingamError(st, lib.lingam_last_error().decode())
    return B


def check_terms(device: int = -1) -> dict:
    """Measured error of the hardware binary32 exp2 / log2 over the argument
    ranges of the per-sample terms, in units of 2^-24 (lingam_check_terms)."""
    lib = load_library()
    r = LingamTermCheck()
    st = lib.lingam_check_terms(int(device), ctypes.byref(r))
    if st != OK:
        raise LingamError(st, lib.lingam_last_error().decode())
    return {f: getattr(r, f) for f, _ in LingamTermCheck._fields_}


def status_string(status: int) -> str:
    return load_library().lingam_status_string(int(status)).decode()


def batch_workspace_size(datasets, precision: str = "fp64", chunk_samples: int = 0) -> int:
    """Device bytes of one fit_order_batch call over `datasets` (host inputs,
    as fit_order_batch takes them): lingam_workspace_size_batch."""
    o, _ = _make_opts(precision, chunk_samples=chunk_samples)
    count = len(datasets)
    sets = (LingamDataset * count)()
    keep = []
    for k, item in enumerate(datasets):
        if isinstance(item, tuple):
            base, idx = item
            base = np.ascontiguousarray(base, dtype=np.float64)
            idx = np.ascontiguousarray(idx, dtype=np.int64)
            keep += [base, idx]
            sets[k].X = ctypes.c_void_p(base.ctypes.data)
            sets[k].p, sets[k].n = base.shape
            sets[k].sample_idx = idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            sets[k].n_idx = idx.size
        else:
            arr = np.ascontiguousarray(item)
            keep.append(arr)
            o.x_dtype = 1 if arr.dtype == np.float32 else 0
            sets[k].X = ctypes.c_void_p(arr.ctypes.data)
            sets[k].p, sets[k].n = arr.shape
    return int(load_library().lingam_workspace_size_batch(count, sets, ctypes.byref(o)))


def workspace_size(n: int, p: int, precision: str = "fp64", x_on_device: bool = False,
                   x_dtype: str = "float64", record_M_iters: int = 0) -> int:
    """Device bytes of one fit_order call (lingam_workspace_size)."""
    o, _ = _make_opts(precision, record_M_iters=record_M_iters)
    o.x_on_device = 1 if x_on_device else 0
    o.x_dtype = 1 if x_dtype == "float32" else 0
    return int(load_library().lingam_workspace_size(n, p, ctypes.byref(o)))
