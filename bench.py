#!/usr/bin/env python3
"""Benchmark of the causal-order search on one MI355X.

Headline workload: p = 500 variables, n = 20000 samples, random DAG with edge
probability 0.02, weights +-U[0.5, 2], Laplace noise, rows permuted (seeded,
synthetic).  One step = one full causal-order search (normalise, covariance,
all p iterations of entropies + threshold rounds of the pair kernel + root
selection + rank-1 update) on the input already resident in device memory.

Reported (one JSON line on stdout):
  value / ms_per_step   evaluated pair-samples per second and order wall time
                        of the mixed-precision path (binary32 per-sample terms)
  fp64, fp32_storage    the same search in the other two precisions
  roofline              the mixed pair kernel's achieved VALU lane-slot rate
                        (kernel time from HIP events attached to each pair-kernel
                        launch on the library's stream) against the issue peak;
                        roofline_fp64 the same for the binary64 pair kernel
  oracle                the orders against the FP64 oracle's stored orders
                        (tests/golden), and the rounding-bound gap rule
  workloads             the other workloads: p=10/n=1000, p=100/n=10000, and
                        p=1000/n=50000 with binary32 storage
  batch                 256 bootstrap resamples and 64 uneven data sets
  cpu_baseline          the FP64 oracle on the host cores, bounded sample
"""
import argparse
import json
import os
import sys
import time

# VALU issue model of gfx950 used for the pair kernels' rooflines:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13 lane-slots/s (binary32
# FMA/add/mul, binary64 FMA and conversions issue one lane-slot each;
# v_exp_f32 / v_log_f32 take two).  One mixed-precision pair-sample needs
# 2 binary64 FMAs + 2 conversions (the two residuals) + 2 x 7 binary32 ops and
# 2 x 3 transcendentals (log cosh and u exp(-u^2/2) of each residual):
# 18 + 6 x 2 = 30 lane-slots.  With binary32 rows the residuals are two
# binary32 FMAs: 16 + 6 x 2 = 28.
PEAK_LANE_SLOTS = 256 * 4 * 16 * 2.4e9
SLOTS_PER_PAIR_SAMPLE_MIXED = 2 + 2 + 2 * 7 + 6 * 2
SLOTS_PER_PAIR_SAMPLE_FP32S = 2 + 2 * 7 + 6 * 2

ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pair_kernel_p500_n20000.traffic.json")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "pair_kernel_p500_n20000.counters.json")
GOLDEN = os.path.join(ROOT, "tests", "golden")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("paper_2109_13993_amd/csrc/kernels.hip", "paper_2109_13993_amd/csrc/lingam_internal.h",
                  "paper_2109_13993_amd/csrc/fp64_math.h", "include/lingam.h")


def kernel_source_digest():
    """sha256 over the code of the device sources, in a fixed order: comments
    are dropped and white space collapsed, so only a change of the code
    itself invalidates a recorded counter value."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        text = open(os.path.join(ROOT, name)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def _record(path):
    """A committed counter record, or None if the device sources changed since."""
    try:
        rec = json.load(open(path))
        if kernel_source_digest() != rec.get("kernel_sources_sha256"):
            return None
        return rec
    except (OSError, ValueError):
        return None


def measured_traffic():
    rec = _record(TRAFFIC_FILE)
    return rec.get("traffic_bytes_per_launch") if rec else None


def fixture(name):
    try:
        return json.load(open(os.path.join(GOLDEN, name)))
    except (OSError, ValueError):
        return None


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
    prof = [lg.fit_order(X, precision=precision, profile=True, **kw) for _ in range(steps)]
    torch.cuda.synchronize()
    return t_plain, res, prof


def kernel_stats(prof):
    kern_s = sum(r.seconds_pair_kernel for r in prof) / len(prof)
    launches = prof[-1].pair_kernel_launches
    return kern_s, launches


def median_time(fn, reps=3):
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2], r


def gap_rule(r, ref_order, upto, probable=False):
    """Iterations [0, upto) of a mixed run whose top score the rounding bounds
    (worst-case T_err, or the probable T_err_prob) separate from every other
    (certified), and how many of those have a root other than ref_order's
    (violations, must be 0).  A pruned variable enters with its partial
    score, an upper bound on its T."""
    import numpy as np
    certified = violations = 0
    E = r.T_err_prob if probable else r.T_err
    for t in range(upto):
        row, err = r.T[t], E[t]
        live = np.isfinite(row)
        comp = live & (r.T_state[t] == 1)
        top = int(np.flatnonzero(comp)[np.argmax(row[comp])])
        others = live.copy()
        others[top] = False
        if not others.any() or row[top] - err[top] > np.max(row[others] + err[others]):
            certified += 1
            violations += int(top != ref_order[t])
    return certified, violations


def mixed_error_report(rm, r64, p):
    """Score error of a mixed run against the FP64 run over the iterations
    both share (same prefix of the order), the a-priori bounds, and the gap
    rule against the FP64 order."""
    import numpy as np
    diff = np.flatnonzero(rm.order != r64.order)
    upto = min(int(diff[0]) + 1 if diff.size else p - 1, p - 1)
    both = (rm.T_state[:upto] == 1) & (r64.T_state[:upto] == 1)
    dT = np.abs(rm.T[:upto][both] - r64.T[:upto][both])
    cert, viol = gap_rule(rm, r64.order, upto)
    cert_p, viol_p = gap_rule(rm, r64.order, upto, probable=True)
    return {"iterations_compared": upto, "max_abs_dT": float(dT.max()) if dT.size else 0.0,
            "max_T_err_bound": float(np.nanmax(rm.T_err[:upto][both])) if dT.size else 0.0,
            "max_dT_over_bound": float(np.max(dT / (rm.T_err[:upto][both] + 1e-12))) if dT.size else 0.0,
            "max_dT_over_probable_bound": float(np.max(dT / (rm.T_err_prob[:upto][both] + 1e-12)))
            if dT.size else 0.0,
            "gap_rule_certified_iterations": cert, "gap_rule_violations": viol,
            "probable_bound_certified_iterations": cert_p, "probable_bound_violations": viol_p}


def order_vs_fixture(order, fx, k=None):
    import numpy as np
    if fx is None:
        return None
    ref = np.array(fx["order"])
    got = np.asarray(order)[:len(ref) if k is None else k]
    ref = ref[:got.size]
    diff = np.flatnonzero(got != ref)
    return {"equal": bool(diff.size == 0), "first_difference": int(diff[0]) if diff.size else -1,
            "compared": int(ref.size)}


def workload_legs(lg, synth):
    """The other workloads, device-resident input, median of three calls."""
    import numpy as np
    import oracle
    import torch
    out = {}
    ds1 = synth.config_dataset(1)
    X1 = torch.from_numpy(ds1.X).to("cuda:0")
    o1 = oracle.fit_order(ds1.X)["order"]
    leg = {"workload": "p=10 n=1000 edge prob 0.3 uniform noise"}
    for prec in ("fp64", "mixed"):
        t, r = median_time(lambda: lg.fit_order(X1, precision=prec))
        leg[prec] = {"ms": t * 1e3, "order_equals_oracle": bool(np.array_equal(r.order, o1))}
    out["p10_n1000"] = leg
    ds2 = synth.config_dataset(2)
    X2 = torch.from_numpy(ds2.X).to("cuda:0")
    leg = {"workload": "p=100 n=10000 edge prob 0.1, noise law per variable"}
    for prec in ("fp64", "mixed", "fp32_storage"):
        t, r = median_time(lambda: lg.fit_order(X2, precision=prec))
        leg[prec] = {"ms": t * 1e3, "pair_samples_per_s": r.pair_samples / t, "pairs_evaluated": r.pairs_evaluated}
    orders = {prec: lg.fit_order(X2, precision=prec).order for prec in ("fp64", "mixed", "fp32_storage")}
    leg["orders_equal_across_precisions"] = bool(all(np.array_equal(orders["fp64"], v) for v in orders.values()))
    out["p100_n10000"] = leg
    log("workload p=100: %s" % {k: round(v["ms"], 2) for k, v in leg.items() if isinstance(v, dict)})
    ds5 = synth.config_dataset(5, dtype=np.float32)
    X5 = torch.from_numpy(ds5.X).to("cuda:0")
    fx5 = fixture("workload5.json")
    leg = {"workload": "p=1000 n=50000 edge prob 0.01 uniform noise, binary32 input"}
    for prec in ("fp32_storage", "mixed"):
        lg.fit_order(X5, precision=prec, max_roots=2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = lg.fit_order(X5, precision=prec, want_H=False)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        leg[prec] = {"full_order_ms": t * 1e3, "pair_samples_per_s": r.pair_samples / t,
                     "pairs_evaluated": r.pairs_evaluated,
                     "first5_vs_oracle": order_vs_fixture(r.order, fx5, 5)}
    t0 = time.perf_counter()
    r = lg.fit_order(X5, precision="fp64", max_roots=5)
    torch.cuda.synchronize()
    leg["fp64_first5"] = {"ms": (time.perf_counter() - t0) * 1e3, "vs_oracle": order_vs_fixture(r.order, fx5, 5)}
    out["p1000_n50000"] = leg
    log("workload p=1000: fp32 storage %.0f ms, mixed %.0f ms" % (leg["fp32_storage"]["full_order_ms"],
                                                                 leg["mixed"]["full_order_ms"]))
    return out


def batch_report(lg, synth, sequential_sample=8):
    """Batched searches (lingam_fit_order_batch), mixed precision: 256
    bootstrap resamples of one p=100, n=5000 data set, and 64 data sets of
    uneven shape (p in [20, 200], n in [1000, 20000]).  Makespan (median of
    three calls, on a workspace allocated once, tuned launch parameters),
    aggregate evaluated pair-samples/s, the orders against the oracle's on
    the stored subset, and the same sets run one lingam_fit_order call at a
    time (a sample of them, timed and scaled to all sets)."""
    import numpy as np
    import torch
    out = {}
    base = synth.config_dataset(4).X
    boot = [(base, idx) for idx in synth.bootstrap_indices(base.shape[1], 256, synth.rng_for(4, 1))]
    uneven = [d.X for d in synth.uneven_datasets(64, synth.rng_for(4, 2))]
    fx = fixture("workload4.json")
    for name, sets, key, fxl in (("bootstrap_256_p100_n5000", boot, "resample", fx and fx["bootstrap"]),
                                 ("uneven_64_p20-200_n1000-20000", uneven, "set", fx and fx["uneven"])):
        ws = torch.empty(lg.batch_workspace_size(sets, "mixed") + 4096, dtype=torch.uint8, device="cuda:0")
        lg.fit_order_batch(sets, precision="mixed", want_T=False, workspace=ws)   # warm-up (and graph capture)
        torch.cuda.synchronize()
        times = []
        for _ in range(3):   # the median of three batch calls
            t0 = time.perf_counter()
            res = lg.fit_order_batch(sets, precision="mixed", want_T=False, workspace=ws)
            times.append(time.perf_counter() - t0)
        dt = sorted(times)[1]
        ps = sum(r.pair_samples for r in res)
        ok = all(r.extra["status"] == 0 for r in res)
        vs = None
        if fxl:
            vs = {"sets_compared": len(fxl),
                  "orders_equal": int(sum(np.array_equal(res[e[key]].order, e["order"]) for e in fxl))}
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
        from paper_2109_13993_amd import autotune
        out[name] = {"sets": len(sets), "makespan_ms": dt * 1e3, "pair_samples_per_s": ps / dt,
                     "all_ok": ok, "one_call_per_set_ms_estimate": dt_seq * 1e3,
                     "speedup_vs_one_call_per_set": dt_seq / dt, "orders_equal_single_calls": same,
                     "vs_oracle": vs,
                     "tuned_params": autotune.lookup("batch", "mixed", *autotune.batch_shape(sets)),
                     "valu_frac_wall": ps * SLOTS_PER_PAIR_SAMPLE_MIXED / dt / PEAK_LANE_SLOTS}
        log("batch %s: %d sets in %.1f ms, %.3e pair-samples/s (one call per set: about %.1f ms, x%.1f); "
            "vs oracle %s" % (name, len(sets), dt * 1e3, ps / dt, dt_seq * 1e3, dt_seq / dt, vs))
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(X, nvars):
    """The FP64 oracle as it is (ordered pairs: each test computes both
    residual entropies, and every unordered pair is evaluated twice, once
    per direction), timed on the host cores on the iteration-0 scores of
    `nvars` variables.  In the GPU's unit (one unordered pair and sample,
    both residuals) the oracle's rate is half its ordered-test rate."""
    import oracle
    from paper_2109_13993_amd import synth
    p, n = X.shape
    nvars = min(nvars, p)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    oracle.sampled_at(X, [], 0, vars=list(range(nvars)), nthreads=cores)
    dt = time.perf_counter() - t0
    ordered = nvars * (p - 1) * n
    out = {"value": ordered / 2.0 / dt, "unit": "pair-samples/s", "cores": cores, "kind": "oracle",
           "sample": "iteration-0 scores of %d of the %d variables of the p=500 n=20000 workload: %d ordered "
                     "tests x %d samples in %.1f s (FP64 plain DirectLiNGAM); GPU unit = ordered tests / 2"
                     % (nvars, p, nvars * (p - 1), n, dt),
           "ordered_test_samples_per_s": ordered / dt, "cpu_model": cpu_model()}
    # single-thread legs (the paper's serial baseline is one core)
    ds1 = synth.config_dataset(1)
    t0 = time.perf_counter()
    oracle.fit_order(ds1.X, nthreads=1)
    t1 = time.perf_counter() - t0
    p1, n1 = ds1.X.shape
    ord1 = (p1 + 1) * p1 * (p1 - 1) // 3 * n1   # ordered tests of all iterations x n
    ds2 = synth.config_dataset(2)
    t0 = time.perf_counter()
    oracle.sampled_at(ds2.X, [], 0, vars=list(range(10)), nthreads=1)
    t2 = time.perf_counter() - t0
    out["single_thread"] = {
        "p10_n1000_full_search_s": t1, "p10_n1000_pair_samples_per_s": ord1 / 2.0 / t1,
        "p100_n10000_sample": "iteration-0 scores of 10 variables, %.2f s" % t2,
        "p100_n10000_pair_samples_per_s": 10 * 99 * ds2.X.shape[1] / 2.0 / t2}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=None, help="timed FP64 searches (default: min(steps, 3))")
    ap.add_argument("--cpu-vars", type=int, default=450, help="variables in the CPU-oracle sample (about 12 s on 16 threads)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 and binary32-storage searches")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-search workloads")
    ap.add_argument("--no-workloads", action="store_true", help="skip the other workloads")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; the library has no multi-GPU path (got --gpus %d)" % args.gpus,
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
    fx3 = fixture("workload3.json")

    t_mix, res_mix, prof_mix = timed_runs(lg, X, "mixed", args.steps, args.warmup)
    pairs = res_mix[-1].pair_samples
    value = pairs / t_mix
    kern_s, launches = kernel_stats(prof_mix)
    achieved = pairs * SLOTS_PER_PAIR_SAMPLE_MIXED / kern_s
    log("mixed: %.1f ms/search, %.3e pair-samples/s, pair kernel %.1f ms in %d launches "
        "(%.1f us avg), pairs %d evaluated / %d computed" % (
            t_mix * 1e3, value, kern_s * 1e3, launches, kern_s / max(launches, 1) * 1e6,
            res_mix[-1].pairs_evaluated, res_mix[-1].pairs_computed))

    # the same search with X in host memory (the copy to the device inside the call)
    t0 = time.perf_counter()
    rh = lg.fit_order(ds.X, precision="mixed")
    t_host = time.perf_counter() - t0

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
                     "avg_launch_us": kern_s / max(launches, 1) * 1e6},
        "pairs_evaluated": res_mix[-1].pairs_evaluated,
        "pairs_computed": res_mix[-1].pairs_computed,
        "effective_pair_samples_per_s": (p + 1) * p * (p - 1) // 6 * n / t_mix,
        "threshold_rounds": res_mix[-1].threshold_rounds,
        "host_input": {"ms_per_step": t_host * 1e3, "pair_samples_per_s": rh.pair_samples / t_host},
        "oracle": {"mixed_order": order_vs_fixture(res_mix[-1].order, fx3)},
    }
    if fx3 is not None:
        cert, viol = gap_rule(res_mix[-1], fx3["order"], p - 1)
        cert_p, viol_p = gap_rule(res_mix[-1], fx3["order"], p - 1, probable=True)
        out["oracle"]["mixed_gap_rule"] = {"certified": cert, "violations": viol,
                                           "probable_certified": cert_p, "probable_violations": viol_p}
    counters = _record(COUNTERS_FILE)
    if not args.no_fp64:
        steps64 = args.fp64_steps if args.fp64_steps is not None else min(args.steps, 3)
        t64, res64, prof64 = timed_runs(lg, X, "fp64", steps64, min(args.warmup, 1))
        v64 = res64[-1].pair_samples / t64
        k64, l64 = kernel_stats(prof64)
        same = bool(np.array_equal(res64[-1].order, res_mix[-1].order))
        out["mixed_error"] = mixed_error_report(res_mix[-1], res64[-1], p)
        # the gap rule on complete scores: one mixed search without the
        # threshold, so that no competitor is known only by a partial score
        rfull = lg.fit_order(X, precision="mixed", use_threshold=False)
        full = mixed_error_report(rfull, res64[-1], p)
        out["mixed_error"]["unpruned_search"] = {
            "order_equals_threshold_search": bool(np.array_equal(rfull.order, res_mix[-1].order)),
            "gap_rule_certified_iterations": full["gap_rule_certified_iterations"],
            "gap_rule_violations": full["gap_rule_violations"],
            "probable_bound_certified_iterations": full["probable_bound_certified_iterations"],
            "probable_bound_violations": full["probable_bound_violations"],
            "max_abs_dT": full["max_abs_dT"], "max_T_err_bound": full["max_T_err_bound"],
            "pairs_computed": rfull.pairs_computed}
        out["fp64"] = {"value": v64, "ms_per_step": t64 * 1e3, "pair_kernel_ms_per_step": k64 * 1e3,
                       "pairs_evaluated": res64[-1].pairs_evaluated, "pairs_computed": res64[-1].pairs_computed}
        out["speedup_fp32_vs_fp64"] = t64 / t_mix
        out["order_fp32_equals_fp64"] = same
        out["oracle"]["fp64_order"] = order_vs_fixture(res64[-1].order, fx3)
        slots64 = counters and counters.get("fp64", {}).get("lane_slots_per_pair_sample")
        if slots64:
            a64 = res64[-1].pairs_computed * n * slots64 / k64
            out["roofline_fp64"] = {"bound": "alu", "achieved": a64 / 1e12, "peak": PEAK_LANE_SLOTS / 1e12,
                                    "unit": "Tlane-slot/s", "frac": a64 / PEAK_LANE_SLOTS,
                                    "kernel": "k_pair_band<fp64>", "slots_per_pair_sample": slots64,
                                    "slots_source": "rocprofv3 SQ_INSTS_VALU (profiles/)",
                                    "avg_launch_us": k64 / max(l64, 1) * 1e6}
        log("fp64: %.1f ms/search, %.3e pair-samples/s, pair kernel %.1f ms; orders equal: %s" % (
            t64 * 1e3, v64, k64 * 1e3, same))
        # binary32 rows
        t32, res32, prof32 = timed_runs(lg, X, "fp32_storage", args.steps, min(args.warmup, 1))
        k32, l32 = kernel_stats(prof32)
        a32 = res32[-1].pair_samples * SLOTS_PER_PAIR_SAMPLE_FP32S / k32
        out["fp32_storage"] = {"value": res32[-1].pair_samples / t32, "ms_per_step": t32 * 1e3,
                               "pair_kernel_ms_per_step": k32 * 1e3, "pairs_evaluated": res32[-1].pairs_evaluated,
                               "pairs_computed": res32[-1].pairs_computed,
                               "roofline_frac": a32 / PEAK_LANE_SLOTS,
                               "slots_per_pair_sample": SLOTS_PER_PAIR_SAMPLE_FP32S,
                               "order_equals_fp64": bool(np.array_equal(res32[-1].order, res64[-1].order)),
                               "oracle_order": order_vs_fixture(res32[-1].order, fx3)}
        log("fp32 storage: %.1f ms/search, pair kernel %.1f ms, frac %.3f" % (t32 * 1e3, k32 * 1e3,
                                                                              a32 / PEAK_LANE_SLOTS))
    if not args.no_workloads:
        out["workloads"] = workload_legs(lg, synth)
    if not args.no_batch:
        out["batch"] = batch_report(lg, synth)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(ds.X, args.cpu_vars)
        log("cpu oracle: %.3e pair-samples/s on %d threads (%s)" % (
            out["cpu_baseline"]["value"], out["cpu_baseline"]["cores"], out["cpu_baseline"]["cpu_model"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
