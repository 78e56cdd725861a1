"""The paper's baseline mappings of the tests onto the GPU (Sec. 5.3: block
worker, thread worker, block compare), run as ablation variants of the pair
step (opts.pair_strategy).  They compute the same sample sums as the pair
kernel in another order, so each must give the oracle's order with every
test, score and entropy within the FP64 limits of the parity tests
(test_gpu_parity.full_parity), and agree with the library's own pair kernel
(threshold and messaging off) to rounding."""
import numpy as np
import pytest

import paper_2109_13993_amd as lg
from paper_2109_13993_amd import synth
from test_gpu_parity import _log, full_parity

pytestmark = pytest.mark.gpu

STRATEGIES = ("block_worker", "thread_worker", "block_compare")


def _ordered_pairs(p, iters=None):
    # every ordered pair of every iteration (r = p, p - 1, ..., 2 variables left)
    rs = range(p, 1, -1) if iters is None else range(p, p - iters, -1)
    return sum(r * (r - 1) for r in rs)


@pytest.mark.parametrize("strategy", STRATEGIES)
def test_baseline_strategy_matches_the_oracle(strategy):
    X = synth.config_dataset(1).X            # p=10, n=1000: one chunk
    g, _ = full_parity(X, messaging=False, pair_strategy=strategy)
    assert g.pairs_evaluated == _ordered_pairs(X.shape[0])
    _log("%s p=10: order equals the oracle's, %d ordered pairs" % (strategy, g.pairs_evaluated))


@pytest.mark.parametrize("strategy", STRATEGIES)
def test_baseline_strategy_ragged_chunks(strategy):
    # three chunks of 2048 samples and a ragged last one; p neither a multiple
    # of the 8-variable target block nor of the work-group
    ds = synth.lingam_dataset(27, 5000, 0.2, "laplace", rng=np.random.default_rng(27))
    g, _ = full_parity(ds.X, messaging=False, pair_strategy=strategy)
    assert g.pairs_evaluated == _ordered_pairs(27)


def test_baseline_strategies_agree_with_the_pair_kernel():
    ds = synth.lingam_dataset(40, 4097, 0.15, "mixed", rng=np.random.default_rng(40))
    kw = dict(precision="fp64", use_threshold=False, messaging=False, record_M_iters=6)
    ref = lg.fit_order(ds.X, **kw)
    fin = np.isfinite(ref.M)
    for s in STRATEGIES:
        g = lg.fit_order(ds.X, pair_strategy=s, **kw)
        assert np.array_equal(g.order, ref.order), s
        assert np.array_equal(np.isfinite(g.M), fin), s
        # the same sums in another order: a few units of 1e-16 per entropy
        d = float(np.max(np.abs(g.M[fin] - ref.M[fin])))
        assert d <= 1e-13, (s, d)
        assert np.allclose(g.T[np.isfinite(ref.T)], ref.T[np.isfinite(ref.T)], rtol=1e-9, atol=1e-14), s
        _log("%s p=40: order equals the pair kernel's, max |dM| %.2e" % (s, d))
