"""Write the FP64 oracle's expected results for the full-size workloads into
tests/golden/ (test infrastructure).

Every value written here comes from the plain CPU oracle (this package) run on
inputs from the seeded generator (paper_2109_13993_amd.synth, which holds no
part of the search); nothing is read from the GPU library.  The oracle runs
with pair_once=True (each unordered pair evaluated once, the reverse test its
exact negation), which the oracle pins show gives bitwise the outputs of the
ordered evaluation in half the time.

Fixtures (JSON, floats written with repr so they read back bit for bit):
  workload3.json  p=500, n=20000, Laplace noise: the full causal order; per
                  iteration the root and the runner-up with their complete
                  scores T and FP64 score tolerances; full score rows at a
                  spread of iterations.
  workload5.json  p=1000, n=50000, uniform noise, binary32 input: the first 5
                  roots and the full score row of each of those iterations.
  workload4.json  32 of the 256 bootstrap resamples (every 8th) of the
                  p=100, n=5000 base set, and 8 of the 64 uneven data sets
                  (every 9th): full orders, root and runner-up per iteration.

The score tolerance stored next to each T is the FP64 parity tolerance of the
GPU tests: a test I_ij may differ by 1e-9 |I_ij| + 1e-14 max(1, 1/(1 - b_ij^2))
(b_ij the pair's correlation), and a score S_i = sum_j min(0, I_ij)^2 by
1e-9 |T_i| + sum_j (2 |min(0, I_ij)| lim_ij + lim_ij^2).

Usage: python -m oracle.make_fixtures {3,5,4,all} [--threads N]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2109_13993_amd import synth  # noqa: E402

GOLDEN = os.path.join(ROOT, "tests", "golden")
REL, M_ABS = 1e-9, 1e-14

# iterations of workload 3 whose whole score row is stored
ROW_ITERS_3 = (0, 1, 2, 5, 10, 25, 50, 100, 200, 300, 400, 450, 490, 495, 498)


def score_limits(T, M, B):
    """FP64 score tolerance of every entry of T[t, v] from the oracle's own
    tests M[t, v, :] and correlations B[t, v, :] (NaN where undefined)."""
    lim = REL * np.abs(M) + M_ABS * np.maximum(1.0, 1.0 / (1.0 - B * B))
    neg = np.abs(np.minimum(M, 0.0))
    extra = np.nansum(2.0 * neg * lim + lim * lim, axis=-1)
    return REL * np.abs(T) + extra


def run_search(X, threads, max_roots=0):
    p = X.shape[0]
    iters = p if max_roots == 0 else max_roots
    t0 = time.time()
    o = oracle.fit_order(X, max_roots=max_roots, M_iters=iters, nthreads=threads, pair_once=True)
    dt = time.time() - t0
    lim = score_limits(o["T"][:iters], o["M"], o["B"])
    return o, lim, dt


def top_two(o, lim, t):
    """[root, T_root, tol_root, runner-up, T_runner, tol_runner] of iteration t
    (the runner-up entries are absent when one variable is left)."""
    row = o["T"][t]
    live = np.flatnonzero(np.isfinite(row))
    root = int(o["order"][t])
    rec = [root, float(row[root]), float(lim[t, root])]
    rest = live[live != root]
    if rest.size:
        k = int(rest[np.argmax(row[rest])])
        rec += [k, float(row[k]), float(lim[t, k])]
    return rec


def score_row(o, lim, t):
    row = o["T"][t]
    live = np.flatnonzero(np.isfinite(row))
    return {"vars": live.tolist(), "T": [float(v) for v in row[live]],
            "tol": [float(v) for v in lim[t, live]]}


def write(name, obj):
    os.makedirs(GOLDEN, exist_ok=True)
    path = os.path.join(GOLDEN, name)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(obj, f, separators=(",", ":"))
        f.write("\n")
    os.replace(tmp, path)
    print("wrote %s (%d bytes)" % (path, os.path.getsize(path)), flush=True)


def workload3(threads):
    ds = synth.config_dataset(3)
    p, n = ds.X.shape
    o, lim, dt = run_search(ds.X, threads)
    print("workload 3: oracle %.0f s" % dt, flush=True)
    write("workload3.json", {
        "workload": "p=500 n=20000 edge prob 0.02 Laplace noise, synth.config_dataset(3)",
        "p": p, "n": n, "oracle_seconds": dt,
        "order": [int(v) for v in o["order"]],
        "top_two": [top_two(o, lim, t) for t in range(p - 1)],
        "rows": {str(t): score_row(o, lim, t) for t in ROW_ITERS_3 if t < p - 1},
    })


def workload5(threads):
    ds = synth.config_dataset(5, dtype=np.float32)
    X = ds.X.astype(np.float64)   # the binary32 input, exactly
    p, n = X.shape
    o, lim, dt = run_search(X, threads, max_roots=5)
    print("workload 5: oracle %.0f s" % dt, flush=True)
    write("workload5.json", {
        "workload": "p=1000 n=50000 edge prob 0.01 uniform noise, binary32 input, "
                    "synth.config_dataset(5, dtype=float32); first 5 roots",
        "p": p, "n": n, "oracle_seconds": dt,
        "order": [int(v) for v in o["order"][:5]],
        "top_two": [top_two(o, lim, t) for t in range(5)],
        "rows": {str(t): score_row(o, lim, t) for t in range(5)},
    })


def workload4(threads):
    base = synth.config_dataset(4).X
    idx = synth.bootstrap_indices(base.shape[1], 256, synth.rng_for(4, 1))
    uneven = synth.uneven_datasets(64, synth.rng_for(4, 2))
    boot, t_all = [], 0.0
    for k in range(0, 256, 8):
        X = np.ascontiguousarray(base[:, idx[k]])
        o, lim, dt = run_search(X, threads)
        t_all += dt
        boot.append({"resample": k, "order": [int(v) for v in o["order"]],
                     "top_two": [top_two(o, lim, t) for t in range(X.shape[0] - 1)]})
        print("workload 4 resample %d: %.1f s" % (k, dt), flush=True)
    sets = []
    for k in range(0, 64, 9):
        X = uneven[k].X
        o, lim, dt = run_search(X, threads)
        t_all += dt
        sets.append({"set": k, "p": X.shape[0], "n": X.shape[1], "order": [int(v) for v in o["order"]],
                     "top_two": [top_two(o, lim, t) for t in range(X.shape[0] - 1)]})
        print("workload 4 uneven set %d (p=%d n=%d): %.1f s" % (k, X.shape[0], X.shape[1], dt), flush=True)
    write("workload4.json", {
        "workload": "bootstrap: synth.bootstrap_indices(5000, 256, synth.rng_for(4, 1)) of "
                    "synth.config_dataset(4); uneven: synth.uneven_datasets(64, synth.rng_for(4, 2))",
        "oracle_seconds": t_all, "bootstrap": boot, "uneven": sets,
    })


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("which", choices=["3", "5", "4", "all"])
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    todo = ["3", "5", "4"] if a.which == "all" else [a.which]
    for w in todo:
        {"3": workload3, "5": workload5, "4": workload4}[w](a.threads)


if __name__ == "__main__":
    main()
