#!/usr/bin/env python3
"""Benchmark of the causal-order search on one MI355X.

Workload: p = 500 variables, n = 20000 samples, random DAG with edge
probability 0.02, weights +-U[0.5, 2], Laplace noise, rows permuted (seeded,
synthetic).  One step = one full causal-order search (normalise, covariance,
all p iterations of entropies + threshold rounds of the pair kernel + root
selection + rank-1 update) on the input already resident in device memory.

Reported: evaluated pair-samples per second of the mixed-precision path
(binary32 per-sample terms) and its order wall time, the same for the FP64
path, the pair kernel's VALU roofline fraction (pair-kernel time measured with
HIP events attached to each pair-kernel launch on the library's stream), and
the FP64 CPU oracle's rate on a
bounded sample of the same workload.  Prints one JSON line on stdout.
"""
import argparse
import json
import os
import sys
import time

# VALU issue model of gfx950 used for the pair kernel's roofline:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13 lane-slots/s (binary32
# FMA/add/mul, binary64 FMA and conversions issue one lane-slot each;
# v_exp_f32 / v_log_f32 take two).  One mixed-precision pair-sample needs
# 2 binary64 FMAs + 2 conversions (the two residuals) + 2 x 7 binary32 ops and
# 2 x 3 transcendentals (log cosh and u exp(-u^2/2) of each residual):
# 18 + 6 x 2 = 30 lane-slots.
PEAK_LANE_SLOTS = 256 * 4 * 16 * 2.4e9
SLOTS_PER_PAIR_SAMPLE_MIXED = 2 + 2 + 2 * 7 + 6 * 2


ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pair_kernel_p500_n20000.traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("kernels.hip", "lingam_internal.h", "fp64_math.h")


def kernel_source_digest():
    """sha256 over the code of the device sources, in a fixed order: comments
    are dropped and white space collapsed, so only a change of the code
    itself invalidates the recorded traffic."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        text = open(os.path.join(ROOT, "paper_2109_13993_amd", "csrc", name)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per pair-kernel launch from the committed rocprofv3 counter
    summary, or None if the device sources changed since it was taken."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
        digest = kernel_source_digest()
    except OSError:
        return None
    if digest != rec.get("kernel_sources_sha256"):
        return None
    return rec.get("traffic_bytes_per_launch")


def timed_runs(lg, X, precision, steps, warmup, **kw):
    """Wall time per search over `steps` searches (after `warmup`), then the
    same number of searches again with a pair of HIP events attached to every
    pair-kernel launch on the library's stream, which take the launch's own
    start and end (timed launches slow the search as a whole, so those
    searches give the kernel durations, not the wall time)."""
    import torch
    for _ in range(warmup):
        lg.fit_order(X, precision=precision, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [lg.fit_order(X, precision=precision, **kw) for _ in range(steps)]
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    prof = [lg.fit_order(X, precision=precision, profile=True, **kw) for _ in range(steps)]
    torch.cuda.synchronize()
    t_prof = (time.perf_counter() - t0) / steps
    return t_plain, res, t_prof, prof


def mixed_error_report(rm, r64, p):
    """Score error of the mixed run against the FP64 run over the iterations
    both share (same prefix of the order), the a-priori bounds, and the gap
    rule: iterations whose top score is separated from every other by the
    bounds, and how many of those disagree with FP64 (must be 0).  A pruned
    variable enters with its partial score, an upper bound on its T, so with
    the threshold on the rule can only certify iterations whose pruned
    variables sit far below the root."""
    import numpy as np
    diff = np.flatnonzero(rm.order != r64.order)
    upto = int(diff[0]) + 1 if diff.size else p - 1
    upto = min(upto, p - 1)
    both = (rm.T_state[:upto] == 1) & (r64.T_state[:upto] == 1)
    dT = np.abs(rm.T[:upto][both] - r64.T[:upto][both])
    certified = violations = 0
    for t in range(upto):
        row, err = rm.T[t], rm.T_err[t]
        live = np.isfinite(row)
        comp = live & (rm.T_state[t] == 1)
        top = int(np.flatnonzero(comp)[np.argmax(row[comp])])
        others = live.copy()
        others[top] = False
        if not others.any() or row[top] - err[top] > np.max(row[others] + err[others]):
            certified += 1
            violations += int(top != r64.order[t])
    return {"iterations_compared": upto, "max_abs_dT": float(dT.max()) if dT.size else 0.0,
            "max_T_err_bound": float(np.nanmax(rm.T_err[:upto][both])) if dT.size else 0.0,
            "max_dT_over_bound": float(np.max(dT / (rm.T_err[:upto][both] + 1e-12))) if dT.size else 0.0,
            "gap_rule_certified_iterations": certified, "gap_rule_violations": violations}


def batch_report(lg, synth, sequential_sample=8):
    """Batched searches (lingam_fit_order_batch), mixed precision: 256
    bootstrap resamples of one p=100, n=5000 data set, and 64 data sets of
    uneven shape (p in [20, 200], n in [1000, 20000]).  Makespan (median of
    three calls), aggregate
    evaluated pair-samples/s, and the same sets run one lingam_fit_order call
    at a time (a sample of them, timed and scaled to all sets)."""
    import numpy as np
    import torch
    out = {}
    base = synth.config_dataset(4).X
    boot = [(base, idx) for idx in synth.bootstrap_indices(base.shape[1], 256, synth.rng_for(4, 1))]
    uneven = [d.X for d in synth.uneven_datasets(64, synth.rng_for(4, 2))]
    for name, sets in (("bootstrap_256_p100_n5000", boot), ("uneven_64_p20-200_n1000-20000", uneven)):
        lg.fit_order_batch(sets[:8], precision="mixed", want_T=False)   # warm-up
        torch.cuda.synchronize()
        times = []
        for _ in range(3):   # the median of three batch calls
            t0 = time.perf_counter()
            res = lg.fit_order_batch(sets, precision="mixed", want_T=False)
            times.append(time.perf_counter() - t0)
        dt = sorted(times)[1]
        ps = sum(r.pair_samples for r in res)
        ok = all(r.extra["status"] == 0 for r in res)
        # one call per data set, on an evenly spaced sample of the sets (host
        # inputs, as in the batch), timed and scaled to all sets
        pick = np.linspace(0, len(sets) - 1, sequential_sample).astype(int)
        singles = []
        for k in pick:
            item = sets[k]
            singles.append(np.ascontiguousarray(item[0][:, item[1]]) if isinstance(item, tuple) else item)
        t0 = time.perf_counter()
        same = True
        for k, X in zip(pick, singles):
            r1 = lg.fit_order(X, precision="mixed", want_T=False, want_H=False)
            same &= bool(np.array_equal(r1.order, res[k].order))
        dt_seq = (time.perf_counter() - t0) / len(pick) * len(sets)
        out[name] = {"sets": len(sets), "makespan_ms": dt * 1e3, "pair_samples_per_s": ps / dt,
                     "all_ok": ok, "one_call_per_set_ms_estimate": dt_seq * 1e3,
                     "speedup_vs_one_call_per_set": dt_seq / dt,
                     "orders_equal_single_calls": same}
        log("batch %s: %d sets in %.1f ms, %.3e pair-samples/s (one call per set: about %.1f ms, x%.1f)" % (
            name, len(sets), dt * 1e3, ps / dt, dt_seq * 1e3, dt_seq / dt))
    return out


def cpu_baseline(X, nvars):
    import oracle
    p, n = X.shape
    nvars = min(nvars, p)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    oracle.sampled_at(X, [], 0, vars=list(range(nvars)), nthreads=cores)
    dt = time.perf_counter() - t0
    pair_samples = nvars * (p - 1) * n
    return {"value": pair_samples / dt, "unit": "pair-samples/s", "cores": cores, "kind": "oracle",
            "sample": "iteration-0 scores of %d of the %d variables (%d tests x %d samples, "
                      "FP64 plain DirectLiNGAM), %.1f s" % (nvars, p, nvars * (p - 1), n, dt)}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=None, help="timed FP64 searches (default: --steps)")
    ap.add_argument("--cpu-vars", type=int, default=160, help="variables in the CPU-oracle sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU path")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-search workloads")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; this build has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes, "copies": 5}))
        return

    import paper_2109_13993_amd as lg
    from paper_2109_13993_amd import synth

    ds = synth.config_dataset(3)
    p, n = ds.X.shape
    X = torch.from_numpy(ds.X).to("cuda:0")
    torch.cuda.synchronize()
    log("workload p=%d n=%d on %s" % (p, n, torch.cuda.get_device_name(0)))

    t_mix, res_mix, t_mix_prof, prof_mix = timed_runs(lg, X, "mixed", args.steps, args.warmup)
    pairs = res_mix[-1].pair_samples
    value = pairs / t_mix
    kern_s = sum(r.seconds_pair_kernel for r in prof_mix) / len(prof_mix)
    launches = prof_mix[-1].pair_kernel_launches
    achieved = pairs * SLOTS_PER_PAIR_SAMPLE_MIXED / kern_s
    log("mixed: %.1f ms/search, %.3e pair-samples/s, pair kernel %.1f ms in %d launches "
        "(%.1f us avg), pairs %d evaluated / %d computed" % (
            t_mix * 1e3, value, kern_s * 1e3, launches, kern_s / max(launches, 1) * 1e6,
            res_mix[-1].pairs_evaluated, res_mix[-1].pairs_computed))

    # the same search with X in host memory (the copy to the device inside the call)
    t0 = time.perf_counter()
    rh = lg.fit_order(ds.X, precision="mixed")
    t_host = time.perf_counter() - t0
    log("mixed, host input: %.1f ms/search" % (t_host * 1e3))

    out = {
        "metric": "pair-sample evals/s + causal-order wall time, p=500 n=20k, FP32 vs FP64",
        "value": value,
        "unit": "pair-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mix * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "DirectLiNGAM causal order, p=500 n=20000, edge prob 0.02, "
                               "Laplace noise, seeded", "p": p, "n": n, "precision": "mixed",
                   "threshold": True},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_SLOTS / 1e12,
                     "unit": "Tlane-slot/s", "frac": achieved / PEAK_LANE_SLOTS, "traffic": measured_traffic(),
                     "kernel": "k_pair_band<mixed>", "slots_per_pair_sample": SLOTS_PER_PAIR_SAMPLE_MIXED,
                     "pair_kernel_ms_per_step": kern_s * 1e3, "launches_per_step": launches,
                     "avg_launch_us": kern_s / max(launches, 1) * 1e6,
                     "ms_per_step_with_events": t_mix_prof * 1e3},
        "pairs_evaluated": res_mix[-1].pairs_evaluated,
        "pairs_computed": res_mix[-1].pairs_computed,
        "effective_pair_samples_per_s": (p + 1) * p * (p - 1) // 6 * n / t_mix,
        "threshold_rounds": res_mix[-1].threshold_rounds,
        "host_input": {"ms_per_step": t_host * 1e3, "pair_samples_per_s": rh.pair_samples / t_host},
    }
    if not args.no_fp64:
        steps64 = args.fp64_steps if args.fp64_steps is not None else min(args.steps, 3)
        t64, res64, _, prof64 = timed_runs(lg, X, "fp64", steps64, min(args.warmup, 1))
        v64 = res64[-1].pair_samples / t64
        k64 = sum(r.seconds_pair_kernel for r in prof64) / len(prof64)
        same = bool(np.array_equal(res64[-1].order, res_mix[-1].order))
        first_diff = int(np.argmax(res64[-1].order != res_mix[-1].order)) if not same else -1
        out["mixed_error"] = mixed_error_report(res_mix[-1], res64[-1], p)
        # the gap rule on complete scores: one mixed search without the
        # threshold, so that no competitor is known only by a partial score
        rfull = lg.fit_order(X, precision="mixed", use_threshold=False)
        full = mixed_error_report(rfull, res64[-1], p)
        out["mixed_error"]["unpruned_search"] = {
            "order_equals_threshold_search": bool(np.array_equal(rfull.order, res_mix[-1].order)),
            "gap_rule_certified_iterations": full["gap_rule_certified_iterations"],
            "gap_rule_violations": full["gap_rule_violations"],
            "max_abs_dT": full["max_abs_dT"], "max_T_err_bound": full["max_T_err_bound"]}
        log("mixed error: gap rule certifies %d iterations (threshold search), %d (unpruned search); "
            "violations %d / %d" % (out["mixed_error"]["gap_rule_certified_iterations"],
                                    full["gap_rule_certified_iterations"],
                                    out["mixed_error"]["gap_rule_violations"], full["gap_rule_violations"]))
        out["fp64"] = {"value": v64, "ms_per_step": t64 * 1e3, "pair_kernel_ms_per_step": k64 * 1e3,
                       "pairs_evaluated": res64[-1].pairs_evaluated}
        out["speedup_fp32_vs_fp64"] = t64 / t_mix
        out["order_fp32_equals_fp64"] = same
        out["order_first_difference"] = first_diff
        log("fp64: %.1f ms/search, %.3e pair-samples/s, pair kernel %.1f ms; orders equal: %s" % (
            t64 * 1e3, v64, k64 * 1e3, same))
    if not args.no_batch:
        out["batch"] = batch_report(lg, synth)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(ds.X, args.cpu_vars)
        log("cpu oracle: %.3e pair-samples/s on %d threads" % (
            out["cpu_baseline"]["value"], out["cpu_baseline"]["cores"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
