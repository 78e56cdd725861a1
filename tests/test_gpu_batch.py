"""Batched searches (lingam_fit_order_batch) on the GPU: every data set's
result must be the one a separate lingam_fit_order call gives -- the same
order, and bit for bit the same score and rounding bound for every variable
whose score is complete in both (the same kernels and per-set arithmetic run
in both; a batch may schedule its threshold bands differently, which changes
only which variables end an iteration pruned and with which partial score)
-- including sets that leave the batch to finish alone, sets with an error,
and bootstrap sets."""
import numpy as np
import pytest

import paper_2109_13993_amd as lg
from paper_2109_13993_amd import synth

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)


def _same(b, s, tag):
    assert b.extra["status"] == 0, tag
    assert np.array_equal(b.order, s.order), tag
    # the same variables take part in each iteration
    assert np.array_equal(np.isfinite(b.T), np.isfinite(s.T)), tag
    both = (b.T_state == 1) & (s.T_state == 1)
    # every iteration has its root complete in both
    assert both.any(axis=1)[:int((s.order >= 0).sum()) - 1].all(), tag
    assert np.array_equal(b.T[both], s.T[both]), tag          # bitwise
    assert np.array_equal(b.T_err[both], s.T_err[both]), tag
    assert np.array_equal(b.T_err_prob[both], s.T_err_prob[both]), tag


def _mixed_batch(seed):
    rng = np.random.default_rng(seed)
    sets = []
    for k, (p, n) in enumerate([(12, 1500), (40, 3000), (9, 700), (67, 5000), (25, 9000), (2, 300)]):
        ds = synth.lingam_dataset(p, n, 0.2, "mixed", rng=np.random.default_rng(seed * 100 + k))
        sets.append(ds.X)
    base = synth.lingam_dataset(30, 4000, 0.15, "laplace", rng=np.random.default_rng(seed + 7)).X
    for idx in synth.bootstrap_indices(4000, 3, rng):
        sets.append((base, idx))
    return sets


def _single(item, **kw):
    if isinstance(item, tuple):
        base, idx = item
        return lg.fit_order(np.ascontiguousarray(base[:, idx]), **kw)
    return lg.fit_order(item, **kw)


@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp32_storage"])
def test_batch_equals_single_runs(precision):
    # on the device work queue (default) and with one grid slice per set
    sets = _mixed_batch(3)
    for queue in (True, False):
        res = lg.fit_order_batch(sets, precision=precision, queue=queue)
        assert len(res) == len(sets)
        for k, item in enumerate(sets):
            _same(res[k], _single(item, precision=precision), "%s queue=%s set %d" % (precision, queue, k))
        _log("%s batch of %d (queue %s): %.1f ms" % (precision, len(sets), queue, res[0].seconds_total * 1e3))


def test_batch_stragglers_and_options():
    # a tiny initial threshold and multiplier need many threshold rounds, so
    # sets halt in the batch and finish alone; max_roots and no-threshold too
    sets = _mixed_batch(5)
    for kw in (dict(gamma0=1e-14, gamma_mult=1.5), dict(max_roots=5), dict(use_threshold=False),
               dict(chunk_samples=512, band_blocks=1)):
        res = lg.fit_order_batch(sets, precision="mixed", **kw)
        for k, item in enumerate(sets):
            _same(res[k], _single(item, precision="mixed", **kw), "%s set %d" % (kw, k))
        _log("%s: rounds %s" % (kw, [r.threshold_rounds for r in res]))


def test_batch_error_in_one_set():
    sets = _mixed_batch(9)[:4]
    bad = sets[1].copy()
    bad[3, 17] = np.nan
    sets[1] = bad
    col = sets[2].copy()
    col[4] = 0.0                       # zero-variance row
    sets[2] = col
    res = lg.fit_order_batch(sets, precision="fp64")
    assert res[1].extra["status"] == lg.E_NONFINITE and res[1].extra["bad_i"] == 3
    assert res[2].extra["status"] == lg.E_DEGENERATE and res[2].extra["bad_i"] == 4
    for k in (0, 3):
        _same(res[k], _single(sets[k], precision="fp64"), "set %d" % k)


def test_bootstrap_batch_config4_shape():
    # 32 bootstrap resamples of one p=100, n=5000 data set (the shape of the
    # bootstrap workload, fewer resamples), checked against single runs
    base = synth.config_dataset(4).X
    rng = synth.rng_for(4, 1)
    sets = [(base, idx) for idx in synth.bootstrap_indices(base.shape[1], 32, rng)]
    res = lg.fit_order_batch(sets, precision="mixed")
    for k in (0, 13, 31):
        _same(res[k], _single(sets[k], precision="mixed"), "resample %d" % k)
    assert all(r.extra["status"] == 0 for r in res)
    ps = sum(r.pair_samples for r in res)
    _log("bootstrap 32 x (100 x 5000): %.1f ms, %.3e pair-samples/s" % (
        res[0].seconds_total * 1e3, ps / res[0].seconds_total))


def test_batch_graph_windows_replay():
    # windows of 16 iterations captured into HIP graphs on the first call and
    # replayed by later calls on the same workspace, with other device work
    # and synchronisations in between: every replay gives the eager results
    import torch
    sets = _mixed_batch(11)
    eager = lg.fit_order_batch(sets, precision="mixed")
    need = lg.batch_workspace_size(sets, precision="mixed")
    ws = torch.empty(need + 4096, dtype=torch.uint8, device="cuda:0")
    x = torch.randn(1 << 20, device="cuda:0")
    for rep in range(4):
        res = lg.fit_order_batch(sets, precision="mixed", workspace=ws, graph=True)
        for k in range(len(sets)):
            _same(res[k], eager[k], "graph replay %d set %d" % (rep, k))
        # eager work of the program between replays
        lg.fit_order(sets[1], precision="mixed")
        x.mul_(1.0001).add_(0.5)
        torch.cuda.synchronize()
        _log("graph replay %d: %.1f ms" % (rep, res[0].seconds_total * 1e3))
