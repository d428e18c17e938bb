"""Failure handling at the C ABI on a device: an allocator callback that
returns NULL must surface as IM_ERR_OUT_OF_MEMORY (not a crash, not a
silent wrong result), leave the context usable, and a later call with memory
available must return the oracle's result."""

import numpy as np
import pytest

import oracle
import paper_2008_03095_amd as P
from tests.conftest import announce
from workloads import chung_lu

pytestmark = pytest.mark.gpu

IM_ERR_OUT_OF_MEMORY = 3


class _Limited:
    """torch's caching allocator behind a byte limit per request (None: refuse all)."""

    def __init__(self, limit):
        import torch

        self.torch = torch
        self.limit = limit
        self.refused = 0
        self.live = {}

    def alloc(self, nbytes):
        if self.limit is None or nbytes > self.limit:
            self.refused += 1
            return None
        ptr = self.torch.cuda.caching_allocator_alloc(nbytes, 0)
        self.live[ptr] = nbytes
        return ptr

    def free(self, ptr):
        self.live.pop(ptr, None)
        self.torch.cuda.caching_allocator_delete(ptr)


def _ctx(lim):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU device")
    return P.Context(device=0, allocator=(lim.alloc, lim.free))


def test_graph_load_out_of_memory():
    lim = _Limited(None)
    ctx = _ctx(lim)
    try:
        announce("allocator returning NULL: graph load")
        g = chung_lu(500, 2000, 2.5, 41)
        with pytest.raises(P.InfuseError) as e:
            P.Graph.from_csr(ctx, g)
        assert e.value.status == IM_ERR_OUT_OF_MEMORY
        assert lim.refused >= 1
    finally:
        ctx.close()


def test_memo_out_of_memory_then_recovers():
    g = chung_lu(3000, 12000, 2.5, 42)
    p, R, seed, K = 0.05, 1024, 6, 12
    lim = _Limited(4 << 20)  # the graph fits, the 3000 x 1024 memo does not
    ctx = _ctx(lim)
    G = None
    try:
        announce("allocator refusing the memo, then allowing it")
        G = P.Graph.from_csr(ctx, g)
        G.set_params(p, R, seed)
        with pytest.raises(P.InfuseError) as e:
            G.select_seeds(K)
        assert e.value.status == IM_ERR_OUT_OF_MEMORY
        with pytest.raises(P.InfuseError) as e:
            G.estimate_sigma([1, 2, 3])
        assert e.value.status == IM_ERR_OUT_OF_MEMORY
        held = ctx.bytes_in_use()
        lim.limit = 1 << 40
        seeds, marg, cover = G.select_seeds(K)
        ref = oracle.run(g, oracle.Sampler("hash", p=p, R=R, seed=seed), K, threads=4)
        assert list(seeds) == list(ref["seeds"]) and list(marg) == list(ref["marginal"])
        assert cover == ref["cover"]
        assert ctx.bytes_in_use() >= held
        G.drop_memo()
        assert ctx.bytes_in_use() == held  # the failed attempts left nothing allocated
    finally:
        if G is not None:
            G.free()
        ctx.close()
    assert not lim.live  # everything returned to the allocator
