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


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("which", choices=["scalability", "ablation", "flux"])
    ap.add_argument("--p", type=int, default=500)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed", "fp32_storage"])
    ap.add_argument("--dense", action="store_true")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--names", default=None, help="flux: comma-separated data-set names")
    a = ap.parse_args()
    if a.which == "scalability":
        scalability(reps=a.reps)
    elif a.which == "ablation":
        ablation(a.p, a.n, a.precision, a.reps, a.dense)
    else:
        flux(a.names.split(",") if a.names else None, reps=max(1, a.reps // 3))


if __name__ == "__main__":
    sys.exit(main())
