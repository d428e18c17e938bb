"""Directed graphs: the memo-free spread (reachability over hashed arcs) on
the device equals the oracle's count, sample for sample in total; memo calls
are refused.  Integers, so the comparison is exact."""

import numpy as np
import pytest

import oracle
import paper_2008_03095_amd as P
from tests.conftest import announce
from workloads import from_arc_list, random_small_digraph, rmat_directed, wc_p

pytestmark = pytest.mark.gpu


def _seed_sets(g, rng):
    deg = np.diff(g.row_ptr.astype(np.int64))
    top = list(np.argsort(-deg, kind="stable")[:min(20, g.n)])
    return [[0], list(rng.choice(g.n, min(5, g.n), replace=False)), top, list(range(g.n))[:200]]


CASES = {
    "drand12": (lambda: random_small_digraph(12, 40, 1), 0.3, 64, 1, False),
    "drand300_ragged": (lambda: random_small_digraph(60, 900, 2), 0.05, 300, 2, False),
    "rmat12_p01": (lambda: rmat_directed(12, 8, 0.57, 0.19, 0.19, 4), 0.01, 1024, 4, False),
    "rmat12_wc": (lambda: rmat_directed(12, 8, 0.57, 0.19, 0.19, 5), 0.0, 512, 5, True),
    "rmat14_wc_R257": (lambda: rmat_directed(14, 6, 0.57, 0.19, 0.19, 6), 0.0, 257, 6, True),
    # more than 8,192 samples: 36 tiles per vertex
    "rmat11_R9000": (lambda: rmat_directed(11, 4, 0.57, 0.19, 0.19, 8), 0.02, 9000, 8, False),
}


@pytest.mark.parametrize("case", list(CASES))
def test_directed_spread_matches_oracle(gpu_ctx, case):
    make, p, R, seed, wc = CASES[case]
    g = make()
    if wc:
        g.p_slot = wc_p(g)
    announce(f"directed spread {case}: n={g.n} arcs={g.nnz} R={R}")
    G = P.Graph.from_csr(gpu_ctx, g)
    try:
        G.set_params(p, R, seed)
        s = oracle.Sampler("hash", p=p, R=R, seed=seed)
        for S in _seed_sets(g, np.random.default_rng(seed)):
            cnt, sig, _ = G.estimate_sigma_direct(S)
            assert cnt == oracle.sigma_count(g, s, S, threads=8), S[:5]
            assert sig == pytest.approx(cnt / R)
    finally:
        G.free()


def test_directed_spread_full_size(gpu_ctx):
    """The directed benchmark workload at full size: R-MAT scale 18, edge
    factor 5, seed 3, weighted cascade, R = 8,192, S = the 100 vertices of
    largest out-degree; the device count equals the oracle's over all
    samples, in the launch configuration the benchmark times."""
    import os

    g = rmat_directed(18, 5, 0.57, 0.19, 0.19, 3)
    g.p_slot = wc_p(g)
    deg = np.diff(g.row_ptr.astype(np.int64))
    S = [int(v) for v in np.argsort(-deg, kind="stable")[:100]]
    announce(f"directed spread full size: n={g.n} arcs={g.nnz} R=8192 |S|=100")
    G = P.Graph.from_csr(gpu_ctx, g)
    try:
        G.set_params(0.0, 8192, 3)
        cnt, _, levels = G.estimate_sigma_direct(S)
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        assert cnt == oracle.sigma_count(g, oracle.Sampler("hash", R=8192, seed=3), S, threads=threads)
        assert levels > 1
    finally:
        G.free()


def test_directed_forced_live_path_and_no_live_arcs(gpu_ctx):
    k = 300
    a = np.arange(k - 1)
    g = from_arc_list(k, a, a + 1)
    announce("directed path, p = 1 and p = 0")
    G = P.Graph.from_csr(gpu_ctx, g)
    try:
        G.set_params(1.0, 128, 3)
        for i in (0, 17, k - 1):
            assert G.estimate_sigma_direct([i])[0] == 128 * (k - i)
        G.set_params(0.0, 128, 3)
        assert G.estimate_sigma_direct([0, 5, 9])[0] == 128 * 3
    finally:
        G.free()


def test_directed_graph_refuses_memo_calls(gpu_ctx):
    g = random_small_digraph(20, 60, 3)
    announce("directed graph memo refusal")
    G = P.Graph.from_csr(gpu_ctx, g)
    try:
        G.set_params(0.1, 64, 1)
        for call in (G.build_memo, lambda: G.select_seeds(2), lambda: G.estimate_sigma([1])):
            with pytest.raises(P.InfuseError) as e:
                call()
            assert e.value.status == 1  # IM_ERR_INVALID_ARG
        assert G.estimate_sigma_direct([1])[0] == oracle.sigma_count(g, oracle.Sampler("hash", p=0.1, R=64, seed=1), [1])
    finally:
        G.free()


def test_arc_loader_rejects_malformed_rows(gpu_ctx):
    with pytest.raises(P.InfuseError):
        P.Graph(gpu_ctx, 3, np.array([0, 2, 2, 2], np.uint64), np.array([2, 1], np.uint32), directed=True)
    with pytest.raises(P.InfuseError):
        P.Graph(gpu_ctx, 3, np.array([0, 1, 1, 1], np.uint64), np.array([0], np.uint32), directed=True)


SELECT_CASES = {
    "drand12_K12": (lambda: random_small_digraph(12, 40, 1), 0.3, 64, 1, False, 12),
    "drand60_ragged": (lambda: random_small_digraph(60, 500, 2), 0.05, 300, 2, False, 10),
    "rmat11_wc": (lambda: rmat_directed(11, 6, 0.57, 0.19, 0.19, 5), 0.0, 256, 5, True, 15),
    "rmat12_p02": (lambda: rmat_directed(12, 5, 0.57, 0.19, 0.19, 7), 0.02, 128, 7, False, 8),
    # the selection of the directed benchmark line, at its size
    "rmat14_wc_K50": (lambda: rmat_directed(14, 5, 0.57, 0.19, 0.19, 4), 0.0, 1024, 4, True, 50),
    # more than 8,192 samples
    "drand80_R9000": (lambda: random_small_digraph(80, 400, 3), 0.05, 9000, 3, False, 5),
}


@pytest.mark.parametrize("case", list(SELECT_CASES))
def test_directed_selection_matches_oracle(gpu_ctx, case):
    make, p, R, seed, wc, K = SELECT_CASES[case]
    g = make()
    if wc:
        g.p_slot = wc_p(g)
    announce(f"directed selection {case}: n={g.n} arcs={g.nnz} R={R} K={K}")
    ref = oracle.celf_arcs(g, oracle.Sampler("hash", p=p, R=R, seed=seed), K)
    G = P.Graph.from_csr(gpu_ctx, g)
    try:
        G.set_params(p, R, seed)
        seeds, marg, cover = G.select_seeds_direct(K)
        assert list(seeds) == list(ref["seeds"])
        assert list(marg) == list(ref["marginal"])
        assert cover == ref["cover"] == G.estimate_sigma_direct(seeds)[0]
        assert G.select_seeds_direct(0)[2] == 0
        with pytest.raises(P.InfuseError):
            G.select_seeds_direct(g.n + 1)
    finally:
        G.free()


def test_memo_free_selection_equals_memo_selection_undirected(gpu_ctx):
    from workloads import make_config

    w = make_config("c1")
    g = w.graphs[0]
    announce("memo-free selection on c1 (undirected)")
    G = P.Graph.from_csr(gpu_ctx, g)
    try:
        G.set_params(w.p, w.R, w.seeds[0])
        s1, m1, c1 = G.select_seeds(w.K)
        s2, m2, c2 = G.select_seeds_direct(w.K)
        assert list(s1) == list(s2) and list(m1) == list(m2) and c1 == c2
    finally:
        G.free()


def test_search_work_counts_on_a_forced_live_path(gpu_ctx):
    """Work counts of the memo-free search, exact on a path with every arc
    live: from seed i the frontier is one vertex per level in one tile, each
    frontier vertex but the last has one arc, live in every column."""
    k = 300
    a = np.arange(k - 1)
    g = from_arc_list(k, a, a + 1)
    announce("search work counts, directed path, p = 1")
    G = P.Graph.from_csr(gpu_ctx, g)
    try:
        G.set_params(1.0, 128, 3)
        gpu_ctx.set_profiling(1)
        try:
            for i in (0, 117, k - 1):
                cnt, _, levels = G.estimate_sigma_direct([i])
                assert cnt == 128 * (k - i) and levels == k - i
                assert G.search_stats() == dict(levels=k - i, items=k - i, arcs=k - 1 - i, live_pairs=k - 1 - i)
            # selection: every search's counts summed, consistent with the work done
            G.select_seeds_direct(3)
            st = G.search_stats()
            assert st["levels"] > 0 and st["items"] >= st["levels"] and st["arcs"] >= st["live_pairs"] > 0
        finally:
            gpu_ctx.set_profiling(0)
        # without profiling only the level count is kept
        G.estimate_sigma_direct([5])
        assert G.search_stats() == dict(levels=k - 5, items=0, arcs=0, live_pairs=0)
    finally:
        G.free()


def test_search_on_a_split_row(gpu_ctx):
    """A row longer than the split threshold is walked in pieces by several
    wavefronts: on a forced-live out-star with 1,000 arcs the spread, the
    levels and the work counts are exact (the centre's item counts once,
    every arc once, every arc is live)."""
    k = 1000
    g = from_arc_list(k + 1, np.zeros(k, np.int64), np.arange(1, k + 1))
    announce("search on a split row: out-star with 1000 arcs, p = 1")
    G = P.Graph.from_csr(gpu_ctx, g)
    try:
        G.set_params(1.0, 300, 5)  # two tiles, the second ragged
        gpu_ctx.set_profiling(1)
        try:
            cnt, _, levels = G.estimate_sigma_direct([0])
            assert cnt == 300 * (k + 1) and levels == 2
            assert G.search_stats() == dict(levels=2, items=2 * (1 + k), arcs=2 * k, live_pairs=2 * k)
            cnt, _, levels = G.estimate_sigma_direct([0, 7])  # a leaf seed adds itself only
            assert cnt == 300 * (k + 1) and levels == 2
        finally:
            gpu_ctx.set_profiling(0)
        seeds, marg, cover = G.select_seeds_direct(2)
        assert list(seeds) == [0, 1] and list(marg) == [300 * (k + 1), 0] and cover == 300 * (k + 1)
    finally:
        G.free()
