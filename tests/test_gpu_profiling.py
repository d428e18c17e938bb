"""Profiling levels of the context: which launches are timed, and the work
counts of a memo construction kept at level 4 (their totals must agree with
the memo's own statistics)."""

import numpy as np
import pytest

import paper_2008_03095_amd as P
from tests.conftest import announce
from workloads import chung_lu

pytestmark = pytest.mark.gpu


def test_profiling_levels(gpu_ctx):
    g = chung_lu(3000, 15000, 2.1, 61)
    announce("profiling levels 0..4")
    G = P.Graph.from_csr(gpu_ctx, g)
    try:
        G.set_params(0.03, 512, 61)
        with pytest.raises(P.InfuseError) as e:
            gpu_ctx.set_profiling(5)
        assert e.value.status == 1
        seen = {}
        for level in range(5):
            gpu_ctx.set_profiling(level)
            gpu_ctx.reset_kernel_stats()
            G.drop_memo()
            seeds, marg, cover = G.select_seeds(10)
            gpu_ctx.set_profiling(0)
            seen[level] = {k: gpu_ctx.kernel_stats(k)[0] for k in ("celf", "hook", "link", "gain0")}
            if level == 0:
                ref = (list(seeds), list(marg), cover)
            assert (list(seeds), list(marg), cover) == ref, level
        assert seen[0] == {"celf": 0, "hook": 0, "link": 0, "gain0": 0}
        assert seen[1] == {"celf": 1, "hook": 0, "link": 0, "gain0": 0}
        for level in (2, 3, 4):
            assert seen[level] == {"celf": 1, "hook": 1, "link": 1, "gain0": 1}, level
        # the memo built at level 4 kept its work counts
        work = G.memo_work()
        st = G.memo_stats()
        assert work["row_tiles"] + work["hub_tiles"] == st["listed_tiles"]
        # members (entries whose label is another vertex): each is re-pointed
        # by the flatten at most once and decrements its root once, and a
        # component of k vertices holds at least k - 1 live edges
        lab = G.labels()
        members = int((lab != np.arange(g.n, dtype=np.int32)[:, None]).sum())
        assert 0 < work["flatten_rewrites"] <= members
        assert 0 < work["count_atomics"] <= members <= work["live_pairs"]
        # a memo built below level 4 has none
        G.drop_memo()
        G.build_memo()
        with pytest.raises(P.InfuseError):
            G.memo_work()
    finally:
        gpu_ctx.set_profiling(0)
        G.free()
