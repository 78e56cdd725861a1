"""Experiments of the paper's evaluation, re-run on this library (one GPU).

  scalability  Sec. 5.4 (Fig. 4): the paper's synthetic workload
               (synth.paper_scalability_dataset: sparse or dense parents,
               weights +-U[0.5, 0.95], noise sign(g)|g|^e) for p in
               {100, 200, 500, 1000} and n in {1024, 2048, 4096, 8192}: the
               order time of each precision and the share of pairs the
               threshold evaluates.
  ablation     the claims of Sec. 1 and Sec. 3.1-3.2: pairs evaluated and time
               with the threshold off, without messaging (every direction
               evaluated by its own variable), and over the multiplier c and
               the initial threshold gamma0.  Every variant must give the
               same order (the paper's exactness claim), which is checked.
  flux         Sec. 5.2 (Table 1): stand-ins of the metabolic-flux data sets
               (synth.flux_like_dataset, rows near the null space of a sparse
               stoichiometric-like matrix) at the real sets' p and n = 10000,
               and the exactly collinear case, which must end DEGENERATE.
  baselines    Sec. 5.3 (Fig. 3): the paper's baseline mappings of the tests
               (block worker, thread worker, block compare; FP64, every
               ordered pair) against this library's FP64 search, on the
               flux-like stand-ins: the full order time of each, the speedup
               of the library over each, and the same pair kernel without the
               threshold and messaging (which separates the mapping from the
               pairs the paper's method avoids).  A baseline whose time,
               extrapolated as p^3 from the previous stand-in, would exceed
               `max_seconds` is skipped and reported as such.  Names are
               those of the flux data sets, or p<k> for a stand-in of k
               variables.

Each prints JSON lines on stdout (one per measurement); times are wall
times of lingam_fit_order on device-resident input, median of `reps`.

    python -m paper_2109_13993_amd.experiments ablation --p 500 --n 4096
"""
import argparse
import json
import sys
import time

import numpy as np


def _timed(fn, reps):
    import torch
    r = fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2], r


def _emit(rec):
    print(json.dumps(rec), flush=True)


def scalability(ps=(100, 200, 500, 1000), ns=(1024, 2048, 4096, 8192), precisions=("mixed", "fp64"), reps=3):
    import torch
    import paper_2109_13993_amd as lg
    from paper_2109_13993_amd import synth
    for dense in (False, True):
        for p in ps:
            for n in ns:
                ds = synth.paper_scalability_dataset(p, n, dense, np.random.default_rng([5, 4, p, n, int(dense)]))
                X = torch.from_numpy(ds.X).to("cuda:0")
                for prec in precisions:
                    t, r = _timed(lambda: lg.fit_order(X, precision=prec, want_H=False), reps)
                    unpruned = (p + 1) * p * (p - 1) // 6
                    _emit({"experiment": "scalability", "graph": "dense" if dense else "sparse", "p": p, "n": n,
                           "precision": prec, "ms": t * 1e3, "pairs_evaluated": r.pairs_evaluated,
                           "pairs_unpruned": unpruned, "evaluated_share": r.pairs_evaluated / unpruned,
                           "order_respects_graph": synth.order_respects_graph(r.order, ds.B)})


def ablation(p=500, n=4096, precision="mixed", reps=3, dense=False):
    import torch
    import paper_2109_13993_amd as lg
    from paper_2109_13993_amd import synth
    ds = synth.paper_scalability_dataset(p, n, dense, np.random.default_rng([5, 5, p, n, int(dense)]))
    X = torch.from_numpy(ds.X).to("cuda:0")
    unpruned = (p + 1) * p * (p - 1) // 6
    variants = [("paper defaults (threshold, messaging)", {}),
                ("threshold off", {"use_threshold": False}),
                ("messaging off", {"messaging": False}),
                ("threshold and messaging off", {"use_threshold": False, "messaging": False})]
    variants += [("c = %g" % c, {"gamma_mult": c}) for c in (1.5, 2.0, 4.0, 8.0, 16.0)]
    variants += [("gamma0 = %g" % g, {"gamma0": g}) for g in (1e-8, 1e-6, 1e-4)]
    ref = None
    for name, kw in variants:
        t, r = _timed(lambda: lg.fit_order(X, precision=precision, want_H=False, **kw), reps)
        if ref is None:
            ref = r.order.copy()
        _emit({"experiment": "ablation", "variant": name, "p": p, "n": n, "precision": precision,
               "graph": "dense" if dense else "sparse", "ms": t * 1e3, "pairs_evaluated": r.pairs_evaluated,
               "evaluated_share_of_unpruned": r.pairs_evaluated / unpruned,
               "threshold_rounds": r.threshold_rounds, "order_equals_defaults": bool(np.array_equal(r.order, ref))})


def flux(names=None, n=10000, precisions=("mixed",), reps=1):
    import torch
    import paper_2109_13993_amd as lg
    from paper_2109_13993_amd import synth
    names = names or list(synth.FLUX_P)
    for name in names:
        p = synth.FLUX_P[name]
        ds = synth.flux_like_dataset(p, n, np.random.default_rng([5, 6, p]))
        X = torch.from_numpy(ds.X).to("cuda:0")
        for prec in precisions:
            rec = {"experiment": "flux", "stand_in_for": name, "p": p, "n": n, "precision": prec}
            try:
                t, r = _timed(lambda: lg.fit_order(X, precision=prec, want_T=False, want_H=False), reps)
                unpruned = (p + 1) * p * (p - 1) // 6
                rec.update(status="ok", seconds=t, pairs_evaluated=r.pairs_evaluated,
                           evaluated_share_of_unpruned=r.pairs_evaluated / unpruned)
            except lg.LingamError as e:
                # near-collinear stand-ins can hold pairs with 1 - corr^2 <= 1e-12
                rec.update(status="degenerate" if e.status == lg.E_DEGENERATE else str(e.status), error=str(e))
            _emit(rec)
    # exactly collinear: the search must stop with DEGENERATE
    ds = synth.flux_like_dataset(85, 2000, np.random.default_rng([5, 7]), noise=0.0)
    try:
        lg.fit_order(ds.X, precision="fp64")
        status = "ok"
    except lg.LingamError as e:
        status = {lg.E_DEGENERATE: "degenerate"}.get(e.status, str(e.status))
    _emit({"experiment": "flux", "stand_in_for": "ecoli_core, exactly collinear", "p": 85, "n": 2000,
           "status": status})


def baselines(names=("ecoli_core", "iJR904"), n=10000, reps=1, max_seconds=120.0):
    import torch
    import paper_2109_13993_amd as lg
    from paper_2109_13993_amd import synth
    last = {}
    for name in names:
        # a named data set's size, or "p<k>" for a flux-like stand-in of k variables
        p = synth.FLUX_P[name] if name in synth.FLUX_P else int(name.lstrip("p"))
        ds = synth.flux_like_dataset(p, n, np.random.default_rng([5, 6, p]))
        X = torch.from_numpy(ds.X).to("cuda:0")
        base_kw = dict(precision="fp64", want_T=False, want_H=False)
        t_lib, r_lib = _timed(lambda: lg.fit_order(X, **base_kw), reps)
        runs = [("library (threshold, messaging)", t_lib, r_lib)]
        flat = dict(base_kw, use_threshold=False, messaging=False)
        t_flat, r_flat = _timed(lambda: lg.fit_order(X, **flat), reps)
        runs.append(("library pair kernel, every ordered pair", t_flat, r_flat))
        for s in ("block_worker", "thread_worker", "block_compare"):
            if s in last:
                p0, t0 = last[s]
                if t0 * (p / p0) ** 3 > max_seconds:
                    _emit({"experiment": "baselines", "stand_in_for": name, "p": p, "n": n, "strategy": s,
                           "status": "skipped", "extrapolated_seconds": t0 * (p / p0) ** 3})
                    continue
            t, r = _timed(lambda: lg.fit_order(X, pair_strategy=s, **flat), reps)
            last[s] = (p, t)
            runs.append((s, t, r))
        for label, t, r in runs:
            _emit({"experiment": "baselines", "stand_in_for": name, "p": p, "n": n, "strategy": label,
                   "status": "ok", "seconds": t, "pairs_evaluated": r.pairs_evaluated,
                   "library_speedup": t / t_lib, "order_equals_library": bool(np.array_equal(r.order, r_lib.order))})


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("which", choices=["scalability", "ablation", "flux", "baselines"])
    ap.add_argument("--p", type=int, default=500)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed", "fp32_storage"])
    ap.add_argument("--dense", action="store_true")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--names", default=None, help="flux, baselines: comma-separated data-set names")
    ap.add_argument("--max-seconds", type=float, default=120.0, help="baselines: skip longer extrapolated runs")
    a = ap.parse_args()
    if a.which == "scalability":
        scalability(reps=a.reps)
    elif a.which == "ablation":
        ablation(a.p, a.n, a.precision, a.reps, a.dense)
    elif a.which == "flux":
        flux(a.names.split(",") if a.names else None, reps=max(1, a.reps // 3))
    else:
        baselines(tuple(a.names.split(",")) if a.names else ("ecoli_core", "iJR904"), reps=max(1, a.reps // 3),
                  max_seconds=a.max_seconds)


if __name__ == "__main__":
    sys.exit(main())
