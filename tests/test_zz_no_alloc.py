"""The allocation-free sigma call (im_estimate_sigma_noalloc) against
im_estimate_sigma, through the C ABI.

Two calls in a row on the same GPU share the library's scratch array: the
first with a large seed set (bitmap path), the second with a smaller one
(pairwise path), then a smaller graph after a larger one.  Counts are
integers and must be identical to the allocating call's (and to the
oracle's).  Also: refusal without a resident memo, refusal of a query whose
scratch would exceed the array, ids >= n.
"""

import numpy as np
import pytest

import oracle
import paper_2008_03095_amd as P
from tests.conftest import announce
from workloads import chung_lu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU device")
    c = P.Context(device=0)
    yield c
    c.close()


def _check(G, g, S, p, R, seed):
    want, sig_want = G.estimate_sigma(S)
    got, sig = G.estimate_sigma_noalloc(S)
    assert got == want, (len(S), got, want)
    assert sig == sig_want
    assert got == oracle.sigma_count(g, oracle.Sampler("hash", p=p, R=R, seed=seed), sorted(set(S)), threads=4)
    return got


def test_noalloc_two_calls_then_smaller(ctx):
    rng = np.random.default_rng(7)
    g1 = chung_lu(4000, 16000, 2.5, 71)
    g2 = chung_lu(1500, 6000, 2.5, 72)
    G1 = P.Graph.from_csr(ctx, g1)
    G2 = P.Graph.from_csr(ctx, g2)
    try:
        announce("noalloc sigma: n=4000 R=1024, 300 then 40 seeds")
        G1.set_params(0.05, 1024, 9)
        G1.build_memo()
        big = rng.choice(g1.n, size=300, replace=False).astype(np.uint32)
        _check(G1, g1, big, 0.05, 1024, 9)  # > 128 seeds: bitmap in the scratch array
        small = np.concatenate([big[:40], big[:5]])  # duplicates count once
        _check(G1, g1, small, 0.05, 1024, 9)
        announce("noalloc sigma: smaller graph n=1500 R=300 after the larger one")
        G2.set_params(0.08, 300, 3)
        G2.build_memo()
        S2 = rng.choice(g2.n, size=200, replace=False).astype(np.uint32)
        _check(G2, g2, S2, 0.08, 300, 3)
        _check(G2, g2, S2[:17], 0.08, 300, 3)
        assert G2.estimate_sigma_noalloc([]) == (0, 0.0)
    finally:
        G1.free()
        G2.free()


def test_noalloc_refusals(ctx):
    g = chung_lu(40000, 120000, 2.5, 73)
    G = P.Graph.from_csr(ctx, g)
    try:
        announce("noalloc sigma: refusals")
        G.set_params(0.01, 8192, 5)
        with pytest.raises(P.InfuseError) as e:
            G.estimate_sigma_noalloc([1, 2, 3])  # no resident memo
        assert e.value.status == 1
        G.build_memo()
        with pytest.raises(P.InfuseError) as e:
            G.estimate_sigma_noalloc([g.n])  # id >= n
        assert e.value.status == 1
        # 200 seeds need an n * R / 8 = 41 MB bitmap: more than the array holds
        S = np.arange(0, 40000, 200, dtype=np.uint32)
        with pytest.raises(P.InfuseError) as e:
            G.estimate_sigma_noalloc(S)
        assert e.value.status == 1 and "scratch" in str(e.value)
        # at most 128 distinct seeds fit whatever the graph
        want, _ = G.estimate_sigma(S[:100])
        assert G.estimate_sigma_noalloc(S[:100])[0] == want
    finally:
        G.free()
