"""The full-size workloads against the FP64 oracle's stored results
(tests/golden/workload{3,4,5}.json, written by oracle/make_fixtures.py from
the oracle alone).

FP64 mode: the causal order must equal the oracle's exactly, and every
complete score must lie within the stored FP64 tolerance of the oracle's
(the tolerance of the parity tests: 1e-9 relative per test plus a floor
from binary64 rounding of the pair's correlation, propagated to the score),
times the conditioning of the iteration's data (below).  A pruned score is
partial, so it may only be larger (T is an upper bound).

Conditioning.  Each RegressRoot step (Alg. 1; the rank-1 update of Sec.
3.4) leaves a variable's residual with a fraction 1 - rho^2 of its variance,
and renormalising it magnifies the rounding that earlier steps left in it
by 1 / sqrt(1 - rho^2).  After t roots that factor is
c_i(t) = 1 / sqrt(1 - R_i^2), R_i^2 the share of x_i's variance the first t
roots explain; both the oracle and the GPU carry binary64 rounding of that
size in their normalised rows.  c_i(t) is the inverse square root of the
diagonal of the correlation matrix's Schur complement after eliminating the
oracle's first t roots (computed here from the input alone), and the
tolerance of iteration t is scaled by max(1, max_i c_i(t)).  Well-posed
workloads keep it near 1; data sets whose variables become near-exact
functions of the roots (deep, dense graphs) reach 1e5-1e6.

Mixed precision (binary32 per-sample terms): up to the first iteration
where its order leaves the oracle's, every iteration the rounding bounds
certify (the gap rule: the top score minus its bound above every other
score plus its bound) must have the oracle's root, so the iteration where
the orders part, if any, must be one that neither bound certifies (after
it the remaining variables differ and nothing is compared).  On the
well-separated workloads the orders must not part at all.
"""
import json
import os
import sys

import numpy as np
import pytest

import paper_2109_13993_amd as lg
from paper_2109_13993_amd import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _fixture(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip("oracle fixture %s not written yet (python -m oracle.make_fixtures)" % name)
    with open(path) as f:
        return json.load(f)


def conditioning(X, order):
    """max_i c_i(t) for t = 0 .. len(order) - 1: the largest magnification of
    binary64 rounding in the normalised residual rows after the first t roots
    of `order` have been regressed out (see the module docstring)."""
    C = np.corrcoef(np.asarray(X, dtype=np.float64))
    left = np.ones(C.shape[0], dtype=bool)
    out = []
    for root in order:
        d = np.diag(C)[left]
        out.append(float(np.max(1.0 / np.sqrt(np.maximum(d, 1e-300)))))
        col = C[:, root].copy()
        C = C - np.outer(col, col) / C[root, root]
        left[root] = False
    return np.maximum(1.0, np.array(out))


def check_fp64_scores(g, fx, iters, tag, cond=None):
    """Root and runner-up scores of every listed iteration, and the stored
    full rows, against the oracle within the stored tolerance times the
    conditioning cond[t] (1 if not given).  Returns the worst |dT| over the
    scaled tolerance."""
    worst = 0.0
    for t in iters:
        rec = fx["top_two"][t]
        kappa = cond[t] if cond is not None else 1.0
        for k in range(0, len(rec), 3):
            v, To, tol = rec[k], rec[k + 1], rec[k + 2] * kappa
            got, state = g.T[t, v], g.T_state[t, v]
            if state == 1:
                err = abs(got - To)
                worst = max(worst, err / tol if err else 0.0)
                assert err <= tol, "%s t=%d v=%d: |dT| %.3e > tol %.3e" % (tag, t, v, err, tol)
            else:
                assert state == 2 and got >= To - tol, (tag, t, v)
    for ts, row in fx.get("rows", {}).items():
        t = int(ts)
        if t >= g.T.shape[0] or t not in iters:
            continue
        v = np.array(row["vars"])
        To, tol = np.array(row["T"]), np.array(row["tol"]) * (cond[t] if cond is not None else 1.0)
        got, state = g.T[t, v], g.T_state[t, v]
        assert np.all(state > 0), (tag, t)
        comp = state == 1
        err = np.abs(got[comp] - To[comp])
        assert np.all(err <= tol[comp]), "%s row t=%d: worst |dT|/tol %.3f" % (
            tag, t, float(np.max(err / tol[comp])))
        if err.size:
            worst = max(worst, float(np.max(np.where(err > 0, err / tol[comp], 0.0))))
        assert np.all(got[~comp] >= To[~comp] - tol[~comp]), (tag, t)
    return worst


def gap_rule(g, fx_order, iters, probable=False):
    """(certified iterations, iterations whose root differs from the oracle's
    although certified) of a mixed-precision run, over the given iterations
    up to the first where its order leaves fx_order, with the worst-case
    bounds T_err or the probable ones T_err_prob."""
    cert = bad = 0
    E = g.T_err_prob if probable else g.T_err
    diff = np.flatnonzero(np.asarray(g.order)[:len(fx_order)] != np.asarray(fx_order))
    last = int(diff[0]) if diff.size else len(fx_order)
    for t in iters:
        if t > last:
            break
        row, err = g.T[t], E[t]
        live = np.isfinite(row)
        comp = live & (g.T_state[t] == 1)
        top = int(np.flatnonzero(comp)[np.argmax(row[comp])])
        others = live.copy()
        others[top] = False
        if not others.any() or row[top] - err[top] > np.max(row[others] + err[others]):
            cert += 1
            bad += int(top != fx_order[t])
    return cert, bad


# ---- workload 3: p=500, n=20000 (Laplace noise) ---------------------------------

@pytest.fixture(scope="module")
def w3():
    return synth.config_dataset(3), _fixture("workload3.json")


def test_workload3_fp64_order_and_scores(w3):
    ds, fx = w3
    p = ds.X.shape[0]
    g = lg.fit_order(ds.X, precision="fp64")
    assert list(g.order) == fx["order"]
    cond = conditioning(ds.X, fx["order"])
    worst = check_fp64_scores(g, fx, range(p - 1), "w3 fp64", cond)
    _log("workload 3 fp64 (threshold on): order equals the oracle's; worst |dT|/tol %.3f "
         "(conditioning up to %.3g)" % (worst, cond.max()))


def test_workload3_fp64_unpruned_rows(w3):
    # without the threshold every score is complete: the stored full rows
    ds, fx = w3
    iters = sorted(int(t) for t in fx["rows"])
    g = lg.fit_order(ds.X, precision="fp64", use_threshold=False, max_roots=max(iters) + 1)
    assert list(g.order[:max(iters) + 1]) == fx["order"][:max(iters) + 1]
    worst = check_fp64_scores(g, fx, iters, "w3 fp64 unpruned", conditioning(ds.X, fx["order"]))
    _log("workload 3 fp64 unpruned: rows at %s, worst |dT|/tol %.3f" % (iters, worst))


def test_workload3_mixed_order(w3):
    ds, fx = w3
    p = ds.X.shape[0]
    g = lg.fit_order(ds.X, precision="mixed")
    diff = np.flatnonzero(g.order != np.array(fx["order"]))
    cert, bad = gap_rule(g, fx["order"], range(p - 1))
    cert_p, bad_p = gap_rule(g, fx["order"], range(p - 1), probable=True)
    _log("workload 3 mixed, probable bound: certifies %d of %d iterations, %d violations" % (cert_p, p - 1, bad_p))
    assert bad_p == 0
    # score error against the oracle on the roots and runners-up
    dT = []
    for t in range(p - 1):
        rec = fx["top_two"][t]
        for k in range(0, len(rec), 3):
            v = rec[k]
            if g.T_state[t, v] == 1 and g.order[t] == fx["order"][t]:
                dT.append(abs(g.T[t, v] - rec[k + 1]) / (g.T_err[t, v] + rec[k + 2]))
    _log("workload 3 mixed: order differs at %s; gap rule certifies %d of %d iterations, %d violations; "
         "max |dT|/(bound+tol) %.3e" % (diff[:5].tolist(), cert, p - 1, bad, max(dT)))
    assert bad == 0
    assert max(dT) <= 1.0
    assert diff.size == 0, "mixed order departs from the oracle's at iteration %d" % diff[0]


# ---- workload 5: p=1000, n=50000, binary32 input ----------------------------------

@pytest.fixture(scope="module")
def w5():
    return synth.config_dataset(5, dtype=np.float32), _fixture("workload5.json")


def test_workload5_first_roots(w5):
    ds, fx = w5
    g = lg.fit_order(ds.X, precision="fp64", max_roots=5)
    assert list(g.order[:5]) == fx["order"]
    worst = check_fp64_scores(g, fx, range(5), "w5 fp64", conditioning(ds.X, fx["order"]))
    _log("workload 5 fp64: first 5 roots equal the oracle's; worst |dT|/tol %.3f" % worst)
    # the workload as specified: binary32 storage with binary64 covariance
    # (and the mixed mode on binary64 rows)
    for precision in ("fp32_storage", "mixed"):
        gm = lg.fit_order(ds.X, precision=precision, max_roots=5)
        cert, bad = gap_rule(gm, fx["order"], range(5))
        cert_p, bad_p = gap_rule(gm, fx["order"], range(5), probable=True)
        _log("workload 5 %s: first roots %s (oracle %s), %d of 5 certified (%d by the probable bound)" % (
            precision, gm.order[:5].tolist(), fx["order"], cert, cert_p))
        assert bad == 0 and bad_p == 0
        assert list(gm.order[:5]) == fx["order"], precision


# ---- workload 4: bootstrap resamples and uneven data sets -----------------------

@pytest.fixture(scope="module")
def w4():
    fx = _fixture("workload4.json")
    base = synth.config_dataset(4).X
    idx = synth.bootstrap_indices(base.shape[1], 256, synth.rng_for(4, 1))
    uneven = synth.uneven_datasets(64, synth.rng_for(4, 2))
    boot = [((base, idx[r["resample"]]), r) for r in fx["bootstrap"]]
    sets = [(uneven[r["set"]].X, r) for r in fx["uneven"]]
    return boot + sets


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_workload4_batch_orders(w4, precision):
    items = [it for it, _ in w4]
    res = lg.fit_order_batch(items, precision=precision)
    certified = certified_p = total = 0
    worst, kmax = 0.0, 1.0
    parted = []
    for r, (it, fx) in zip(res, w4):
        tag = "resample %s" % fx["resample"] if "resample" in fx else "set %s" % fx["set"]
        assert r.extra["status"] == 0, tag
        p = len(fx["order"])
        if precision == "fp64":
            Xs = it[0][:, it[1]] if isinstance(it, tuple) else it
            cond = conditioning(Xs, fx["order"])
            worst = max(worst, check_fp64_scores(r, fx, range(p - 1), tag, cond))
            kmax = max(kmax, float(cond.max()))
        else:
            cert, bad = gap_rule(r, fx["order"], range(p - 1))
            cert_p, bad_p = gap_rule(r, fx["order"], range(p - 1), probable=True)
            certified += cert
            certified_p += cert_p
            total += p - 1
            assert bad == 0 and bad_p == 0, tag
            diff = np.flatnonzero(np.asarray(r.order) != np.asarray(fx["order"]))
            if diff.size:
                parted.append("%s at iteration %d" % (tag, diff[0]))
            continue
        assert list(r.order) == fx["order"], tag
    if precision == "mixed":
        _log("workload 4 mixed batch: %d of %d data sets have the oracle's order (parted, uncertified: %s); "
             "gap rule certifies %d of %d iterations (%d by the probable bound)" % (
                 len(res) - len(parted), len(res), parted or "none", certified, total, certified_p))
        # a parting is allowed only where the scores are closer than the bounds: rare
        assert len(parted) <= max(1, len(res) // 8), parted
    else:
        _log("workload 4 fp64 batch: %d data sets equal the oracle's orders; worst |dT|/tol %.3f "
             "(conditioning up to %.3g)" % (len(res), worst, kmax))
