"""lingam_fit_order_noalloc (the entry point for callers that cannot
allocate) against lingam_fit_order, through the C ABI: the same kernels run
on buffers carved from the library's fixed per-GPU device array instead of
an allocation, so every output must be bitwise the same.  Two calls in a
row, the second smaller, show that what the array keeps from the last call
does not leak into the next."""
import numpy as np
import pytest

import paper_2109_13993_amd as lg
from paper_2109_13993_amd import synth

pytestmark = pytest.mark.gpu


def _same(a, b, tag):
    assert np.array_equal(a.order, b.order), tag
    for k in ("T", "T_state", "H", "T_err"):
        assert np.array_equal(getattr(a, k), getattr(b, k), equal_nan=True), (tag, k)
    assert a.pairs_evaluated == b.pairs_evaluated, tag


def test_noalloc_matches_fit_order_two_calls():
    import torch
    big = synth.config_dataset(2)                     # p=100, n=10000
    small = synth.lingam_dataset(23, 3001, 0.3, "laplace", rng=np.random.default_rng(41))
    for precision in ("fp64", "mixed"):
        for ds, tag in ((big, "p=100 n=10000"), (small, "p=23 n=3001")):
            print("noalloc %s %s" % (precision, tag), flush=True)
            ref = lg.fit_order(ds.X, precision=precision)
            got = lg.fit_order(ds.X, precision=precision, noalloc=True)
            _same(got, ref, "%s %s" % (precision, tag))
    # device input on a torch stream, and the M record
    Xd = torch.from_numpy(small.X).to("cuda:0")
    s = torch.cuda.Stream()
    ref = lg.fit_order(Xd, precision="fp64", record_M_iters=2, stream=s)
    got = lg.fit_order(Xd, precision="fp64", record_M_iters=2, stream=s, noalloc=True)
    _same(got, ref, "device input")
    assert np.array_equal(got.M, ref.M, equal_nan=True)


def test_noalloc_rejects_what_does_not_fit():
    X = np.random.default_rng(0).laplace(size=(500, 20000))
    with pytest.raises(lg.LingamError) as e:
        lg.fit_order(X, precision="mixed", noalloc=True)
    assert e.value.status == lg.E_NOMEM and "at most" in str(e.value)
    with pytest.raises(lg.LingamError) as e:
        lg.fit_order(X[:5, :100], profile=True, noalloc=True)
    assert e.value.status == lg.E_UNSUPPORTED
