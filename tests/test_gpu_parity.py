"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

FP64 mode.  The stated tolerance is a relative error of 1e-9 on the scores.
A purely relative test is ill-posed for tests near zero, and both
implementations round, so each test I_ij may also differ by an absolute
amount derived from FP64 arithmetic:
  |dM_ij| <= 1e-9 |M_ij| + 1e-14 max(1, s_ij^2),   s_ij^2 = 1 / (1 - b_ij^2),
where b_ij is the pair's correlation (from the oracle).  Derivation: an
entropy term moves by |dH| <= 2 k1 |E1 - beta| |dE1| + 2 k2 |E2| |dE2| <= 16 |dE1|
(|E1 - beta| <= 0.1), and the sample moment of a normalised residual
u = s (z_i - b z_j) moves by about s^2 times the ~5 ulp rounding of b and s,
so |dM| <~ 16 * 5 * 1.1e-16 * s^2 ~ 1e-14 s^2.  The score tolerance follows
from S_i = sum_j min(0, M_ij)^2:
  |dT_i| <= 1e-9 |T_i| + sum_j (2 |min(0, M_ij)| lim_ij + lim_ij^2).
The causal order must be identical.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_2109_13993_amd as lg
from paper_2109_13993_amd import synth

pytestmark = pytest.mark.gpu

REL = 1e-9
M_ABS = 1e-14
H_ABS = 1e-12


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def m_limit(Mo, Bo):
    return REL * np.abs(Mo) + M_ABS * np.maximum(1.0, 1.0 / (1.0 - Bo * Bo))


def t_limit(To, Mo, Bo):
    """Limits for T[t, v] given the oracle's M[t, v, :] and B[t, v, :] (NaN-safe)."""
    lim = m_limit(Mo, Bo)
    neg = np.abs(np.minimum(Mo, 0.0))
    extra = np.nansum(2.0 * neg * lim + lim * lim, axis=-1)
    return REL * np.abs(To) + extra


def check_limit(got, exp, lim, what):
    got, exp, lim = (np.asarray(a, dtype=float) for a in (got, exp, lim))
    fin = np.isfinite(exp)
    assert np.array_equal(np.isfinite(got), fin), what + ": NaN pattern differs"
    if not fin.any():
        return 0.0
    err = np.abs(got[fin] - exp[fin])
    with np.errstate(invalid="ignore", divide="ignore"):
        ratio = np.where(err == 0.0, 0.0, err / lim[fin])
    worst = float(np.max(ratio))
    _log("%s: max |d| %.3e  worst d/limit %.3f" % (what, float(err.max()), worst))
    assert worst <= 1.0, what
    return worst


def check_fp64(g, o, iters):
    """Compare T, H, M of iterations [0, iters) (oracle run with M_iters >= iters)."""
    check_limit(g.M[:iters], o["M"][:iters], m_limit(o["M"][:iters], o["B"][:iters]), "M")
    check_limit(g.T[:iters], o["T"][:iters], t_limit(o["T"][:iters], o["M"][:iters], o["B"][:iters]), "T")
    check_limit(g.H, o["H"], np.full(o["H"].shape, H_ABS), "H")


def full_parity(X, M_iters=None, **kw):
    p = X.shape[0]
    M_iters = p if M_iters is None else M_iters
    o = oracle.fit_order(X, M_iters=M_iters)
    g = lg.fit_order(X, precision="fp64", use_threshold=False, record_M_iters=M_iters, **kw)
    assert list(g.order) == list(o["order"])
    check_fp64(g, o, M_iters)
    return g, o


# ---- full parity at small sizes ----------------------------------------------

def test_config1_fp64_full_parity():
    ds = synth.config_dataset(1)   # p=10, n=1000
    full_parity(ds.X)


@pytest.mark.parametrize("p,n,noise,seed", [(27, 3001, "laplace", 1), (17, 700, "mixed", 2),
                                            (9, 256, "uniform", 3), (33, 4097, "power15", 4)])
def test_ragged_fp64_full_parity(p, n, noise, seed):
    # p not a multiple of the 8-variable tiles, n not a multiple of the 256-sample stages
    ds = synth.lingam_dataset(p, n, 0.3, noise, rng=np.random.default_rng(seed))
    full_parity(ds.X)


def test_small_chunks_and_bands_fp64_parity():
    # many sample chunks per tile and one block distance per band
    ds = synth.lingam_dataset(40, 5000, 0.2, "laplace", rng=np.random.default_rng(7))
    g, o = full_parity(ds.X, M_iters=3, chunk_samples=512)
    t = lg.fit_order(ds.X, precision="fp64", chunk_samples=512, band_blocks=1)
    assert list(t.order) == list(o["order"])


def test_threshold_keeps_order_and_complete_scores():
    # one target block per band so the threshold has many chances to prune
    for seed, (p, n) in enumerate([(10, 1000), (27, 3001), (60, 4000)]):
        ds = synth.lingam_dataset(p, n, 0.3, "mixed", rng=np.random.default_rng(50 + seed))
        off = lg.fit_order(ds.X, use_threshold=False)
        # every unordered pair of every iteration, counted once (device-wide counters)
        assert off.pairs_evaluated == (p + 1) * p * (p - 1) // 6
        for g0, c, bt in ((1e-6, 4.0, 1), (1e-9, 2.0, 1), (1e-3, 10.0, 1), (0.0, 4.0, 1),
                          (0.0, 1.5, 2), (1e-6, 4.0, 0)):
            on = lg.fit_order(ds.X, use_threshold=True, gamma0=g0, gamma_mult=c, band_blocks=bt)
            assert list(on.order) == list(off.order)
            comp = on.T_state == 1
            pruned = on.T_state == 2
            assert np.array_equal(on.T[comp], off.T[comp])          # same values, bitwise
            assert np.all(on.T[pruned] >= off.T[pruned])           # partial S <= full S
            assert np.array_equal(on.T_state > 0, off.T_state > 0)
            assert on.pairs_evaluated <= off.pairs_evaluated
            _log("p=%d gamma0=%g c=%g band_blocks=%d: pairs %d / %d, rounds %d, bands %d" % (
                p, g0, c, bt, on.pairs_evaluated, off.pairs_evaluated, on.threshold_rounds, on.bands))
            if p >= 27 and bt == 1 and g0 != 1e-3:
                assert on.pairs_evaluated < off.pairs_evaluated


def test_messaging_off_gives_the_same_results_with_twice_the_pairs():
    # without messaging every variable evaluates its own direction of each
    # pair (Sec. 3.1 ablation): the same order and bitwise the same scores,
    # with every pair evaluated twice when nothing is pruned
    for seed, (p, n) in enumerate([(27, 3001), (60, 4000)]):
        ds = synth.lingam_dataset(p, n, 0.3, "mixed", rng=np.random.default_rng(70 + seed))
        for precision in ("fp64", "mixed"):
            on = lg.fit_order(ds.X, precision=precision, use_threshold=False, record_M_iters=2)
            off = lg.fit_order(ds.X, precision=precision, use_threshold=False, record_M_iters=2, messaging=False)
            assert np.array_equal(on.order, off.order)
            assert np.array_equal(on.T, off.T, equal_nan=True) and np.array_equal(on.M, off.M, equal_nan=True)
            assert off.pairs_evaluated == 2 * on.pairs_evaluated == (p + 1) * p * (p - 1) // 3
            th = lg.fit_order(ds.X, precision=precision, messaging=False, band_blocks=1)
            assert np.array_equal(th.order, on.order)
            comp = th.T_state == 1
            assert np.array_equal(th.T[comp], on.T[comp])
            _log("p=%d %s messaging off: %d pairs with the threshold, %d without" % (
                p, precision, th.pairs_evaluated, off.pairs_evaluated))


def test_flux_like_stand_in():
    # data shaped like sampled metabolic fluxes (rows near the null space of
    # a sparse stoichiometric-like matrix, E. coli core's p = 85): the FP64
    # order equals the oracle's; exactly collinear rows must end DEGENERATE
    # in both
    ds = synth.flux_like_dataset(85, 10000, np.random.default_rng(85))
    o = oracle.fit_order(ds.X, pair_once=True)
    g = lg.fit_order(ds.X, precision="fp64")
    assert list(g.order) == list(o["order"])
    gm = lg.fit_order(ds.X, precision="mixed")
    _log("flux-like p=85: mixed order %s the oracle's" % ("equals" if np.array_equal(gm.order, o["order"])
                                                         else "differs from"))
    ex = synth.flux_like_dataset(85, 2000, np.random.default_rng(86), noise=0.0)
    with pytest.raises(oracle.OracleError) as eo:
        oracle.fit_order(ex.X, pair_once=True)
    assert eo.value.status == oracle.E_DEGENERATE
    with pytest.raises(lg.LingamError) as e:
        lg.fit_order(ex.X, precision="fp64")
    assert e.value.status == lg.E_DEGENERATE


@pytest.fixture(scope="module")
def cfg2():
    ds = synth.config_dataset(2)   # p=100, n=10000
    return ds, oracle.fit_order(ds.X, M_iters=100)


def test_config2_fp64_parity(cfg2):
    ds, o = cfg2
    g = lg.fit_order(ds.X, precision="fp64", use_threshold=False, record_M_iters=100)
    assert list(g.order) == list(o["order"])
    assert g.pairs_evaluated == 101 * 100 * 99 // 6
    check_fp64(g, o, 100)
    on = lg.fit_order(ds.X, precision="fp64")   # default: threshold on
    assert list(on.order) == list(o["order"])
    small = lg.fit_order(ds.X, precision="fp64", band_blocks=1)
    assert list(small.order) == list(o["order"])
    assert small.pairs_evaluated < g.pairs_evaluated


def test_config2_mixed_free_running_order(cfg2):
    # the mixed-precision search run free (not teacher-forced) must find the
    # oracle's order; the gap rule must hold wherever it certifies
    ds, o = cfg2
    g = lg.fit_order(ds.X, precision="mixed")
    p = ds.X.shape[0]
    diff = np.flatnonzero(g.order != o["order"])
    cert = 0
    for t in range(p - 1):
        top, ok = _gap_certified(g.T, g.T_err, g.T_state, t)
        cert += ok
        if ok:
            assert o["order"][t] == top, "iteration %d certified but the oracle's root differs" % t
    _log("mixed cfg2 free running: order differs at %s; %d of %d iterations certified" % (
        diff[:5].tolist(), cert, p - 1))
    assert diff.size == 0


@pytest.mark.parametrize("every", [4, 0])
def test_refresh_period_fp64(cfg2, every):
    # Gram refresh every 4 iterations, or only the rank-1 UpdateCovMat
    # recursion: the recursion drifts from the data, so only the order and a
    # loose score agreement are expected
    ds, o = cfg2
    g = lg.fit_order(ds.X, precision="fp64", cov_refresh_every=every)
    assert list(g.order) == list(o["order"])
    both = (g.T_state == 1) & np.isfinite(o["T"])
    rel = np.abs(g.T[both] - o["T"][both]) / np.maximum(np.abs(o["T"][both]), 1e-12)
    _log("refresh every %d: max rel |dT| %.3e" % (every, rel.max()))
    assert rel.max() < 1e-4


# ---- full size (p=500, n=20000): sampled outputs --------------------------------

@pytest.fixture(scope="module")
def cfg3():
    return synth.config_dataset(3)


def _sampled_check(X, g, prefix, t, rest, rng, nvars, npairs, tag):
    vars_ = sorted(rng.choice(rest, nvars, replace=False).tolist())
    pairs = [tuple(rng.choice(rest, 2, replace=False).tolist()) for _ in range(npairs)]
    # all tests of the sampled variables, for the score limits
    rows = [(v, j) for v in vars_ for j in rest if j != v]
    T, Mrow, Brow = oracle.sampled_at(X, prefix, t, vars=vars_, pairs=rows + pairs, with_corr=True)
    k = len(rows)
    M, B = Mrow[k:], Brow[k:]
    Mv = np.array(Mrow[:k]).reshape(len(vars_), -1)
    Bv = np.array(Brow[:k]).reshape(len(vars_), -1)
    check_limit(g.T[t, vars_], T, t_limit(T, Mv, Bv), "T(t=%d) %s" % (t, tag))
    check_limit(np.array([g.M[t, i, j] for i, j in pairs]), M, m_limit(M, B), "M(t=%d) %s" % (t, tag))
    check_limit(np.array([g.M[t, i, j] for i, j in rows]), Mv.ravel(), m_limit(Mv.ravel(), Bv.ravel()),
                "M rows(t=%d) %s" % (t, tag))


def test_fullsize_sampled_fp64_iteration0(cfg3):
    X = cfg3.X
    p = X.shape[0]
    g = lg.fit_order(X, precision="fp64", use_threshold=False, max_roots=1, record_M_iters=1)
    _sampled_check(X, g, [], 0, list(range(p)), np.random.default_rng(0), 6, 32, "cfg3")
    # antisymmetry of the whole matrix, bitwise
    Mg = g.M[0]
    off = ~np.eye(p, dtype=bool)
    assert np.array_equal(Mg[off], -Mg.T[off])


def test_fullsize_sampled_fp64_teacher_forced(cfg3):
    X = cfg3.X
    t = 5
    prefix = [int(v) for v in cfg3.true_order[:t]]
    g = lg.fit_order(X, precision="fp64", use_threshold=False, forced_order=prefix,
                     max_roots=t + 1, record_M_iters=t + 1)
    assert list(g.order[:t]) == prefix
    rest = sorted(set(range(X.shape[0])) - set(prefix))
    _sampled_check(X, g, prefix, t, rest, np.random.default_rng(1), 4, 24, "cfg3 forced")


def test_largest_config_first_roots():
    # p=1000, n=50000 (uniform noise): the first 5 roots of the FP64 search.
    # The oracle cannot run this search whole; at each of the 5 iterations it
    # scores (with the GPU's root prefix) the GPU root and 5 other sampled
    # variables: the scores must agree and the root's must be the largest.
    ds = synth.config_dataset(5)
    X = ds.X
    p = X.shape[0]
    g = lg.fit_order(X, precision="fp64", max_roots=5)
    rng = np.random.default_rng(5)
    for t in range(5):
        prefix = [int(v) for v in g.order[:t]]
        root = int(g.order[t])
        rest = sorted(set(range(p)) - set(prefix) - {root})
        vars_ = sorted([root] + rng.choice(rest, 5, replace=False).tolist())
        T, _ = oracle.sampled_at(X, prefix, t, vars=vars_, pairs=[])
        T = np.asarray(T)
        got = g.T[t, vars_]
        fin = g.T_state[t, vars_] == 1
        rel = np.abs(got[fin] - T[fin]) / np.maximum(np.abs(T[fin]), 1e-12)
        _log("p=1000 t=%d root %d: T %.6e, sampled max %.6e, max rel |dT| %.2e" % (
            t, root, T[vars_.index(root)], np.max(np.delete(T, vars_.index(root))),
            rel.max() if rel.size else 0.0))
        assert fin[vars_.index(root)]
        assert rel.size == 0 or rel.max() < 1e-8
        # the oracle's full score of the root is the largest (up to the FP64 tolerance)
        others = np.delete(T, vars_.index(root))
        assert np.all(T[vars_.index(root)] >= others - 1e-8 * np.abs(others) - 1e-15)
    # the whole mixed-precision search at this size
    gm = lg.fit_order(X, precision="mixed")
    assert list(gm.order[:5]) == list(g.order[:5])
    _log("p=1000 n=50000 mixed: full order in %.2f s, %d pairs evaluated" % (gm.seconds_total, gm.pairs_evaluated))


def test_many_variables_first_roots():
    # p=2100: more rows than the decision keeps in registers (2048) and than
    # one tile of the rank kernel (1024), so both take their long paths.  The
    # first 4 roots of the FP64 search are checked against the oracle at
    # their iterations (the root and 5 sampled variables, with the GPU's root
    # prefix), and the mixed search must give the same first roots.
    ds = synth.lingam_dataset(2100, 2000, 0.005, "uniform", rng=np.random.default_rng(21))
    X = ds.X
    p = X.shape[0]
    g = lg.fit_order(X, precision="fp64", max_roots=4)
    rng = np.random.default_rng(22)
    for t in range(4):
        prefix = [int(v) for v in g.order[:t]]
        root = int(g.order[t])
        rest = sorted(set(range(p)) - set(prefix) - {root})
        vars_ = sorted([root] + rng.choice(rest, 5, replace=False).tolist())
        T, _ = oracle.sampled_at(X, prefix, t, vars=vars_, pairs=[])
        T = np.asarray(T)
        got = g.T[t, vars_]
        fin = g.T_state[t, vars_] == 1
        rel = np.abs(got[fin] - T[fin]) / np.maximum(np.abs(T[fin]), 1e-12)
        _log("p=2100 t=%d root %d: max rel |dT| %.2e" % (t, root, rel.max() if rel.size else 0.0))
        assert fin[vars_.index(root)]
        assert rel.size == 0 or rel.max() < 1e-8
        others = np.delete(T, vars_.index(root))
        assert np.all(T[vars_.index(root)] >= others - 1e-8 * np.abs(others) - 1e-15)
    gm = lg.fit_order(X, precision="mixed", max_roots=4)
    assert list(gm.order[:4]) == list(g.order[:4])


def test_more_rows_than_the_rank_kernel_orders():
    # p=16500 > 16384: past the rank kernel's limit the positions keep the
    # original order; every index offset into the p x p matrices exceeds 2^28.
    # Two iterations of the FP64 search without the threshold (every pair in
    # one band); at each, the oracle scores the GPU root and 5 sampled
    # variables (with the GPU's root prefix): the scores must agree and the
    # root's must be the largest.  Independent rows of uniform noise with a
    # few planted edges keep the data cheap to make at this size.
    p, n = 16500, 256
    rng = np.random.default_rng(165)
    X = rng.uniform(-1.0, 1.0, size=(p, n))
    for k in range(0, 40, 2):
        X[k + 1] += 0.8 * X[k]
    g = lg.fit_order(X, precision="fp64", use_threshold=False, max_roots=2, want_H=False)
    for t in range(2):
        prefix = [int(v) for v in g.order[:t]]
        root = int(g.order[t])
        rest = sorted(set(range(p)) - set(prefix) - {root})
        vars_ = sorted([root] + rng.choice(rest, 5, replace=False).tolist())
        T, _ = oracle.sampled_at(X, prefix, t, vars=vars_, pairs=[])
        T = np.asarray(T)
        got = g.T[t, vars_]
        rel = np.abs(got - T) / np.maximum(np.abs(T), 1e-12)
        _log("p=16500 t=%d root %d: max rel |dT| %.2e" % (t, root, rel.max()))
        assert rel.max() < 1e-8
        others = np.delete(T, vars_.index(root))
        assert np.all(T[vars_.index(root)] >= others - 1e-8 * np.abs(others) - 1e-15)


def test_fullsize_runs_are_deterministic_and_threshold_exact(cfg3):
    X = cfg3.X
    a = lg.fit_order(X, precision="mixed")
    b = lg.fit_order(X, precision="mixed")
    assert np.array_equal(a.order, b.order)
    assert np.array_equal(a.T, b.T, equal_nan=True)
    assert sorted(a.order.tolist()) == list(range(X.shape[0]))
    off = lg.fit_order(X, precision="mixed", use_threshold=False, max_roots=10)
    assert list(off.order[:10]) == list(a.order[:10])
    _log("cfg3 mixed: pairs %d computed %d rounds %d bands %d, %.3f s" % (
        a.pairs_evaluated, a.pairs_computed, a.threshold_rounds, a.bands, a.seconds_device))


# ---- mixed precision -------------------------------------------------------------

def test_mixed_teacher_forced_scores():
    ds = synth.config_dataset(2)
    o = oracle.fit_order(ds.X, M_iters=3)
    g = lg.fit_order(ds.X, precision="mixed", use_threshold=False, forced_order=o["order"],
                     record_M_iters=3)
    dM = np.nanmax(np.abs(g.M - o["M"]))
    fin = np.isfinite(o["T"])
    dT = np.abs(g.T[fin] - o["T"][fin])
    dH = np.nanmax(np.abs(g.H - o["H"]))
    _log("mixed cfg2: max|dM| %.3e  max|dT| %.3e  max|dH| %.3e" % (dM, dT.max(), dH))
    assert dM < 1e-5 and dH < 1e-6
    # the a-priori rounding bound of every score holds against the FP64 oracle
    # (plus the FP64 pipeline tolerance of the end-to-end comparison)
    tol64 = 1e-9 * np.abs(o["T"][fin]) + 1e-12
    ratio = dT / (g.T_err[fin] + tol64)
    _log("mixed cfg2: max |dT| / (bound + tol) = %.3e, max bound %.3e" % (ratio.max(), g.T_err[fin].max()))
    assert np.all(g.T_err[fin] >= 0.0) and ratio.max() <= 1.0
    # gap rule: where the bound separates the top score from every other, the
    # mixed argmax is the oracle's root
    certified = 0
    for t in range(ds.X.shape[0] - 1):
        row, err = g.T[t], g.T_err[t]
        live = np.isfinite(row)
        top = int(np.flatnonzero(live)[np.argmax(row[live])])
        others = live.copy()
        others[top] = False
        if row[top] - err[top] > np.max(row[others] + err[others]):
            certified += 1
            assert top == o["order"][t], "iteration %d certified but argmax differs" % t
    _log("mixed cfg2: %d of %d iterations certified by the gap rule" % (certified, ds.X.shape[0] - 1))


def test_fp32_storage_scores_and_order(cfg2):
    # binary32 rows: iteration 0 holds the rows as first rounded, so every
    # score must lie within its stated bound of the oracle's; the search
    # run free must find the oracle's order, and the gap rule must hold
    ds, o = cfg2
    p = ds.X.shape[0]
    g = lg.fit_order(ds.X, precision="fp32_storage", use_threshold=False, record_M_iters=1)
    fin = np.isfinite(o["T"][0])
    dT = np.abs(g.T[0][fin] - o["T"][0][fin])
    tol = 1e-9 * np.abs(o["T"][0][fin]) + 1e-12
    ratio = dT / (g.T_err[0][fin] + tol)
    dM = np.nanmax(np.abs(g.M[0] - o["M"][0]))
    _log("fp32 storage cfg2 t=0: max|dM| %.3e max|dT| %.3e, max |dT|/(bound+tol) %.3e" % (
        dM, dT.max(), ratio.max()))
    assert ratio.max() <= 1.0
    f = lg.fit_order(ds.X, precision="fp32_storage")
    cert = 0
    for t in range(p - 1):
        top, ok = _gap_certified(f.T, f.T_err, f.T_state, t)
        cert += ok
        if ok:
            assert o["order"][t] == top, "iteration %d certified but the oracle's root differs" % t
    diff = np.flatnonzero(f.order != o["order"])
    _log("fp32 storage cfg2 free running: order differs at %s; %d of %d certified" % (
        diff[:5].tolist(), cert, p - 1))
    assert diff.size == 0
    # half the row storage of the binary64 modes
    assert lg.workspace_size(10000, 100, "fp32_storage") < lg.workspace_size(10000, 100, "mixed")


def test_probable_bound_holds_and_certifies(cfg2):
    # the probable bound (independent rounding errors, Hoeffding) against
    # the FP64 oracle, teacher-forced: every score within it, and it
    # certifies more iterations than the worst-case bound, none wrongly
    ds, o = cfg2
    p = ds.X.shape[0]
    for precision in ("mixed", "fp32_storage"):
        g = lg.fit_order(ds.X, precision=precision, use_threshold=False, forced_order=o["order"])
        fin = np.isfinite(o["T"])
        dT = np.abs(g.T[fin] - o["T"][fin])
        tol64 = 1e-9 * np.abs(o["T"][fin]) + 1e-12
        if precision == "mixed":     # binary64 rows: the same data, so every score is covered
            ratio = dT / (g.T_err_prob[fin] + tol64)
            assert ratio.max() <= 1.0, ratio.max()
        cw = cp = 0
        for t in range(p - 1):
            top, ok = _gap_certified(g.T, g.T_err, g.T_state, t)
            top_p, ok_p = _gap_certified(g.T, g.T_err_prob, g.T_state, t)
            cw += ok
            cp += ok_p
            if ok_p:
                assert top_p == o["order"][t], "%s iteration %d" % (precision, t)
        _log("%s cfg2: probable bound / worst case %.3e (median), max |dT|/prob-bound %.3e; certified %d "
             "(probable) vs %d (worst case) of %d" % (
                 precision, float(np.median(g.T_err_prob[fin] / np.maximum(g.T_err[fin], 1e-300))),
                 float(np.max(dT / (g.T_err_prob[fin] + tol64))), cp, cw, p - 1))
        assert cp >= cw


def _gap_certified(T, E, state, t):
    """Root position of iteration t of a mixed run and whether the rounding
    bounds separate it from every other variable (a pruned variable's partial
    T is an upper bound of its full score, so it competes with that value)."""
    row, err = T[t], E[t]
    live = np.isfinite(row)
    comp = live & (state[t] == 1)
    top = int(np.flatnonzero(comp)[np.argmax(row[comp])])
    others = live.copy()
    others[top] = False
    if not others.any():
        return top, True
    return top, bool(row[top] - err[top] > np.max(row[others] + err[others]))


@pytest.mark.gpu
@pytest.mark.parametrize("chunk", [0, 1024])
def test_mixed_free_running_order_gap_rule(cfg3, chunk):
    """Free-running mixed order against the FP64 order at full size: the first
    iteration where they differ must be one the rounding bound cannot certify."""
    X = cfg3.X
    g64 = lg.fit_order(X, precision="fp64")
    gm = lg.fit_order(X, precision="mixed", chunk_samples=chunk)
    p = X.shape[0]
    diff = np.flatnonzero(gm.order != g64.order)
    first = int(diff[0]) if diff.size else p
    cert = 0
    for t in range(min(first + 1, p - 1)):
        top, ok = _gap_certified(gm.T, gm.T_err, gm.T_state, t)
        assert top == gm.order[t]
        cert += ok
        if t == first:
            assert not ok, "iteration %d: mixed root %d certified but FP64 root is %d" % (
                t, gm.order[t], g64.order[t])
    both = (gm.T_state[:first] == 1) & (g64.T_state[:first] == 1)
    dT = np.abs(gm.T[:first][both] - g64.T[:first][both])
    bound = gm.T_err[:first][both] + 1e-9 * np.abs(g64.T[:first][both]) + 1e-12
    _log("mixed chunk=%d: orders agree on %d of %d iterations; %d certified; max|dT| %.3e; "
         "max |dT|/bound %.3e" % (chunk, first, p, cert, dT.max(), (dT / bound).max()))
    assert np.all(dT <= bound)


# ---- edge cases and input forms ------------------------------------------------

def _hadamard_rows(p):
    # p <= 3 mutually orthogonal zero-mean rows of +-1 over n = 4 samples:
    # every covariance is exactly 0 (all partial sums of +-c^2 are exact),
    # every row has the same |values| and its u exp(-u^2/2) terms cancel
    # exactly, so every test is exactly 0 and every score ties at 0
    return np.array([[1.0, 1.0, -1.0, -1.0], [1.0, -1.0, 1.0, -1.0], [1.0, -1.0, -1.0, 1.0]])[:p]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ties_go_to_the_lowest_original_index(precision):
    import itertools
    for p in (2, 3):
        H = _hadamard_rows(p)
        for perm in itertools.permutations(range(p)):
            X = H[list(perm)]
            g = lg.fit_order(X, precision=precision, record_M_iters=1)
            off = ~np.eye(p, dtype=bool)
            assert np.all(g.M[0][off] == 0.0), (precision, perm, g.M[0])   # an exact tie
            assert list(g.order) == list(range(p)), (precision, perm, g.order)
            assert list(oracle.fit_order(X)["order"]) == list(range(p))


def test_degenerate_pair_found_when_pruned():
    # a nearly collinear pair (1 - corr^2 < 1e-12) among 64 variables, with the
    # threshold on and one target block per band: the pair is checked at the
    # start of the iteration whether or not the threshold would prune it
    ds = synth.lingam_dataset(64, 4000, 0.1, "laplace", rng=np.random.default_rng(31))
    X = ds.X.copy()
    X[63] = 2.0 * X[40] + 1e-7 * np.random.default_rng(32).standard_normal(4000) * X[40].std()
    with pytest.raises(oracle.OracleError) as eo:
        oracle.fit_order(X)
    assert eo.value.status == oracle.E_DEGENERATE
    for kw in (dict(precision="fp64", band_blocks=1), dict(precision="mixed")):
        with pytest.raises(lg.LingamError) as e:
            lg.fit_order(X, **kw)
        assert e.value.status == lg.E_DEGENERATE and {e.value.bad_i, e.value.bad_j} == {40, 63}, kw


def test_caller_workspace_gives_the_same_result():
    import torch
    ds = synth.lingam_dataset(40, 6000, 0.2, "mixed", rng=np.random.default_rng(33))
    need = lg.workspace_size(6000, 40, precision="mixed")
    ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    a = lg.fit_order(ds.X, precision="mixed")
    b = lg.fit_order(ds.X, precision="mixed", workspace=ws)
    assert np.array_equal(a.order, b.order)
    assert np.array_equal(a.T, b.T, equal_nan=True) and np.array_equal(a.T_err, b.T_err, equal_nan=True)
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(lg.LingamError) as e:
        lg.fit_order(ds.X, precision="mixed", workspace=small)
    assert e.value.status == lg.E_NOMEM

def test_one_and_two_variables():
    rng = np.random.default_rng(3)
    r = lg.fit_order(rng.uniform(size=(1, 100)))
    assert list(r.order) == [0]
    X = rng.laplace(size=(2, 3000))
    X[1] += 0.5 * X[0]
    o = oracle.fit_order(X, M_iters=1)
    g = lg.fit_order(X, record_M_iters=1)
    assert list(g.order) == list(o["order"])
    check_limit(g.M, o["M"], m_limit(o["M"], o["B"]), "M(p=2)")


def test_degenerate_and_nonfinite_inputs():
    rng = np.random.default_rng(0)
    X = rng.uniform(size=(5, 300))
    Y = X.copy(); Y[2] = 4.0
    with pytest.raises(lg.LingamError) as e:
        lg.fit_order(Y)
    assert e.value.status == lg.E_DEGENERATE and e.value.bad_i == 2
    Y = X.copy(); Y[4] = -3.0 * Y[1] + 2.0
    with pytest.raises(lg.LingamError) as e:
        lg.fit_order(Y)
    assert e.value.status == lg.E_DEGENERATE and {e.value.bad_i, e.value.bad_j} == {1, 4}
    Y = X.copy(); Y[3, 7] = np.inf
    with pytest.raises(lg.LingamError) as e:
        lg.fit_order(Y)
    assert e.value.status == lg.E_NONFINITE and e.value.bad_i == 3


def test_max_roots_forced_order_and_input_forms():
    ds = synth.lingam_dataset(12, 2000, 0.3, "uniform", rng=np.random.default_rng(8))
    o = oracle.fit_order(ds.X)
    g = lg.fit_order(ds.X)
    assert list(g.order) == list(o["order"])
    part = lg.fit_order(ds.X, max_roots=4)
    assert list(part.order[:4]) == list(o["order"][:4]) and list(part.order[4:]) == [-1] * 8
    forced = [int(o["order"][5]), int(o["order"][2])]
    of = oracle.fit_order(ds.X, forced_order=forced)
    gf = lg.fit_order(ds.X, forced_order=forced)
    assert list(gf.order) == list(of["order"])
    # sample-major layout and binary32 input give the same order
    gs = lg.fit_order(np.ascontiguousarray(ds.X.T), layout="sample_major")
    assert list(gs.order) == list(o["order"])
    X32 = ds.X.astype(np.float32)
    o32 = oracle.fit_order(X32.astype(np.float64))
    g32 = lg.fit_order(X32)
    assert list(g32.order) == list(o32["order"])


def test_device_tensor_input():
    import torch
    ds = synth.lingam_dataset(20, 3000, 0.3, "laplace", rng=np.random.default_rng(9))
    o = oracle.fit_order(ds.X)
    Xd = torch.from_numpy(ds.X).to("cuda:0")
    g = lg.fit_order(Xd)
    assert list(g.order) == list(o["order"])
    s = torch.cuda.Stream()
    g2 = lg.fit_order(Xd, stream=s)
    assert list(g2.order) == list(o["order"])
