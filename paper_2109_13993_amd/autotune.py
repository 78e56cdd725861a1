"""Autotuner of the search's launch parameters on the GPU it runs on.

What it tunes never changes a result: the order and every complete score
are the same for any value (the threshold's band schedule and multiplier c,
and for batches the device work queue and graph replay, only move work
around).  It only changes the time.  The sample chunk of the pair kernel's work-groups is not
tuned: it groups the per-sample sums, so another chunk length rounds them
differently, and every entry keeps the default of 2048 samples (a single
call and a batch then give the same bits whichever entries apply).

Parameters (lingam_opts fields):
  chunk_samples  samples per pair-kernel work-group chunk (fixed at 2048)
  first_band_blocks  target blocks of an iteration's first threshold band
  band_target    pair-samples a later band of round 0 aims at
  gamma_mult     the threshold's multiplier c between rounds (Sec. 3.2)
  batch_queue    batches: device work queue (1) or one grid slice per set (0)
  graph          batches: HIP-graph windows replayed from a workspace (1)

A tuned entry is keyed by the device (ISA and compute-unit count) and a bucket
of the problem: kind (single / batch), precision, and p and n rounded up to
powers of two.  Entries live in a JSON cache ($LINGAM_TUNE_CACHE, default
~/.cache/lingam_mi355x/tune.json); entries shipped with the package
(tuned.json beside this file, measured on MI355X) are used when the cache
has none.  fit_order / fit_order_batch apply the entry of their bucket unless
a parameter is passed explicitly (tune=False switches this off).

Tuning is coordinate descent: one parameter at a time over its candidates,
each timed as the median of `reps` calls on a seeded synthetic workload of
the bucket's shape (device-resident input), keeping the fastest.  A
candidate replaces the current best only when it is at least MIN_GAIN (1%)
faster, so that timing noise between nearly equal settings does not move an
entry.

    python -m paper_2109_13993_amd.autotune single --p 500 --n 20000 --precision mixed
    python -m paper_2109_13993_amd.autotune batch --precision mixed --workload bootstrap
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SHIPPED = os.path.join(HERE, "tuned.json")
CACHE = os.environ.get("LINGAM_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "lingam_mi355x", "tune.json"))

CHUNK_SAMPLES = 2048
MIN_GAIN = 0.01
SINGLE_SPACE = {
    "first_band_blocks": [1, 2, 4, 8],
    "band_target": [1e7, 2e7, 4e7, 6e7, 1e8, 2e8, 4e8, 8e8, 1.6e9],
    "gamma_mult": [1.5, 2.0, 4.0, 8.0],
}
BATCH_SPACE = dict(SINGLE_SPACE, batch_queue=[1, 0], graph=[0, 1])

_device_key = None
_tables = None


def device_key() -> str:
    """ISA and compute-unit count of device 0 (the marketing name is left
    out: it depends on the host's device-id tables)."""
    global _device_key
    if _device_key is None:
        import torch
        props = torch.cuda.get_device_properties(0)
        arch = getattr(props, "gcnArchName", "unknown").split(":")[0]
        _device_key = "%s|%d CUs" % (arch, props.multi_processor_count)
    return _device_key


def _pow2(x: int) -> int:
    return 1 << max(1, int(math.ceil(math.log2(max(int(x), 2)))))


def bucket(kind: str, precision: str, p: int, n: int) -> str:
    return "%s/%s/p%d/n%d" % (kind, precision, _pow2(p), _pow2(n))


def _read(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _load_tables():
    global _tables
    if _tables is None:
        _tables = (_read(CACHE), _read(SHIPPED))
    return _tables


def lookup(kind: str, precision: str, p: int, n: int):
    """Tuned parameters for this device and bucket, or None."""
    try:
        dev = device_key()
    except Exception:
        return None
    b = bucket(kind, precision, p, n)
    for table in _load_tables():
        entry = table.get(dev, {}).get(b)
        if entry:
            return dict(entry["params"])
    return None


def store(kind: str, precision: str, p: int, n: int, params: dict, seconds: float, path: str = None):
    """Write an entry (atomically) into the cache, or into `path`."""
    global _tables
    path = path or CACHE
    table = _read(path)
    table.setdefault(device_key(), {})[bucket(kind, precision, p, n)] = {
        "params": params, "seconds": seconds, "tuned_at": time.strftime("%Y-%m-%d %H:%M:%S")}
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    _tables = None


def _median_time(fn, reps):
    import torch
    fn()  # warm-up
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2]


def _descend(space, start, timer, log):
    best = dict(start)
    best_t = timer(best)
    log("start %s: %.2f ms" % (best, best_t * 1e3))
    for name, cands in space.items():
        for v in cands:
            if v == best.get(name):
                continue
            trial = dict(best, **{name: v})
            t = timer(trial)
            log("  %s=%s: %.2f ms" % (name, v, t * 1e3))
            if t < best_t * (1.0 - MIN_GAIN):
                best, best_t = trial, t
    return best, best_t


def tune_single(p: int, n: int, precision: str = "mixed", reps: int = 3, log=print, path: str = None):
    """Tune a single search of p variables and n samples; stores and returns
    (params, seconds)."""
    import torch
    import paper_2109_13993_amd as lg
    from paper_2109_13993_amd import synth
    q = min(0.3, 10.0 / p)
    ds = synth.lingam_dataset(p, n, q, "laplace", rng=np.random.default_rng([2109, p, n]))
    X = torch.from_numpy(ds.X).to("cuda:0")
    space = {k: (v[precision] if isinstance(v, dict) else v) for k, v in SINGLE_SPACE.items()}
    start = {"chunk_samples": CHUNK_SAMPLES, "first_band_blocks": 4 if precision != "fp64" else 1,
             "band_target": 6e7 if precision != "fp64" else 2e7, "gamma_mult": 4.0}

    def timer(params):
        return _median_time(lambda: lg.fit_order(X, precision=precision, want_T=False, want_H=False,
                                                 tune=False, **params), reps)
    best, t = _descend(space, start, timer, log)
    store("single", precision, p, n, best, t, path)
    return best, t


def batch_workload(name: str):
    from paper_2109_13993_amd import synth
    if name == "bootstrap":
        base = synth.config_dataset(4).X
        return [(base, idx) for idx in synth.bootstrap_indices(base.shape[1], 256, synth.rng_for(4, 1))]
    if name == "uneven":
        return [d.X for d in synth.uneven_datasets(64, synth.rng_for(4, 2))]
    raise ValueError(name)


def batch_shape(sets):
    p = max((it[0] if isinstance(it, tuple) else it).shape[0] for it in sets)
    n = max(it[1].size if isinstance(it, tuple) else it.shape[1] for it in sets)
    return p, n


def tune_batch(sets, precision: str = "mixed", reps: int = 3, log=print, path: str = None):
    """Tune a batch of data sets (bucket: the largest p and n); stores and
    returns (params, seconds)."""
    import torch
    import paper_2109_13993_amd as lg
    p, n = batch_shape(sets)
    space = {k: (v[precision] if isinstance(v, dict) else v) for k, v in BATCH_SPACE.items()}
    start = {"chunk_samples": CHUNK_SAMPLES, "first_band_blocks": 1, "band_target": 2e7, "gamma_mult": 4.0,
             "batch_queue": 1, "graph": 0}
    # one workspace for every trial (the layout depends on the chunk only)
    need = lg.batch_workspace_size(sets, precision, chunk_samples=CHUNK_SAMPLES)
    ws = torch.empty(need + 4096, dtype=torch.uint8, device="cuda:0")

    def timer(params):
        kw = dict(params)
        kw["queue"] = bool(kw.pop("batch_queue"))
        kw["graph"] = bool(kw["graph"])
        return _median_time(lambda: lg.fit_order_batch(sets, precision=precision, want_T=False, tune=False,
                                                       workspace=ws, **kw), reps)
    best, t = _descend(space, start, timer, log)
    store("batch", precision, p, n, best, t, path)
    return best, t


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("kind", choices=["single", "batch"])
    ap.add_argument("--p", type=int, default=500)
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed", "fp32_storage"])
    ap.add_argument("--workload", default="bootstrap", choices=["bootstrap", "uneven"])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=None, help="JSON file to write (default: the cache)")
    a = ap.parse_args()
    log = lambda *x: print(*x, file=sys.stderr, flush=True)   # noqa: E731
    if a.kind == "single":
        best, t = tune_single(a.p, a.n, a.precision, a.reps, log, a.out)
    else:
        best, t = tune_batch(batch_workload(a.workload), a.precision, a.reps, log, a.out)
    print(json.dumps({"device": device_key(), "params": best, "ms": t * 1e3}), flush=True)


if __name__ == "__main__":
    main()
