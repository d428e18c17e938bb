"""Pins of the oracle's directed-graph spread (reachability over hashed arcs).

The paper leaves directed graphs to future work; the reading taken here
hashes an arc u -> v from the ordered pair (key u*n + v, folded like the
undirected key) and counts, per sample, the vertices reachable from S over
the live arcs (the independent-cascade spread of Algorithm 4).  These tests
pin it against closed forms and against a reachability computed by scipy
from liveness flags built in Python, not by the oracle's search.
"""

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import breadth_first_order, connected_components

import oracle
from workloads import from_arc_list, random_small_digraph, random_small_graph, wc_p


def test_arc_key_plain_below_2_32_and_folded_above():
    n = 40000
    for (u, v) in [(0, 1), (5, 39999), (39999, 5), (123, 4567), (4567, 123)]:
        assert oracle.arc_key(u, v, n) == u * n + v
    n = 1 << 18
    u, v = (1 << 17) + 3, (1 << 14) + 7  # u*n + v exceeds 2^32
    key = u * n + v
    assert oracle.arc_key(u, v, n) == (key & 0xFFFFFFFF) ^ oracle.fmix32(key >> 32)


def test_arc_key_agrees_with_edge_key_in_increasing_order_only():
    n = 1000
    for (u, v) in [(1, 2), (3, 700), (998, 999)]:
        assert oracle.arc_key(u, v, n) == oracle.edge_key(u, v, n)
        assert oracle.arc_key(v, u, n) != oracle.edge_key(v, u, n)
        assert oracle.arc_hash(9, u, v, n) != oracle.arc_hash(9, v, u, n)


def _path(k):
    a = np.arange(k - 1)
    return from_arc_list(k, a, a + 1)


@pytest.mark.parametrize("R", [1, 7])
def test_forced_live_directed_path(R):
    k = 9
    g = _path(k)
    s = oracle.Sampler("hash", p=1.0, R=R, seed=5)
    for i in range(k):
        assert oracle.sigma_count(g, s, [i]) == R * (k - i)  # i .. k-1
    assert oracle.sigma_count(g, s, [2, 6]) == R * (k - 2)
    assert oracle.sigma_count(g, s, []) == 0


def test_forced_live_out_star_and_in_star():
    n = 12
    leaves = np.arange(1, n)
    out_star = from_arc_list(n, np.zeros(n - 1, np.int64), leaves)
    in_star = from_arc_list(n, leaves, np.zeros(n - 1, np.int64))
    s = oracle.Sampler("hash", p=1.0, R=3, seed=1)
    assert oracle.sigma_count(out_star, s, [0]) == 3 * n
    assert oracle.sigma_count(out_star, s, [4]) == 3
    assert oracle.sigma_count(in_star, s, [0]) == 3
    assert oracle.sigma_count(in_star, s, [4]) == 3 * 2
    assert oracle.sigma_count(in_star, s, [4, 5]) == 3 * 3


def test_p_zero_counts_the_seeds():
    g = random_small_digraph(10, 40, 3)
    s = oracle.Sampler("hash", p=0.0, R=11, seed=2)
    assert oracle.sigma_count(g, s, [0, 3, 9]) == 11 * 3


def test_both_arcs_forced_live_give_components():
    und = random_small_graph(30, 40, 8)
    rows = np.repeat(np.arange(und.n), np.diff(und.row_ptr.astype(np.int64)))
    g = from_arc_list(und.n, rows, und.col.astype(np.int64))  # every edge as two arcs
    assert g.nnz == und.nnz
    s = oracle.Sampler("hash", p=1.0, R=2, seed=4)
    a = sp.csr_matrix((np.ones(und.nnz), und.col.astype(np.int64), und.row_ptr.astype(np.int64)),
                      shape=(und.n, und.n))
    _, lab = connected_components(a, directed=False)
    for v in range(und.n):
        assert oracle.sigma_count(g, s, [v]) == 2 * int(np.sum(lab == lab[v]))


def _reach_scipy(g, live_slots, S):
    """Vertices reachable from S over the live slots (a virtual source n
    points at every seed)."""
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr.astype(np.int64)))[live_slots]
    cols = g.col.astype(np.int64)[live_slots]
    rows = np.concatenate([rows, np.full(len(S), g.n)])
    cols = np.concatenate([cols, np.asarray(S, dtype=np.int64)])
    a = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(g.n + 1, g.n + 1))
    order = breadth_first_order(a, g.n, directed=True, return_predecessors=False)
    return len(order) - 1


def _live(g, p_slot, R, seed):
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr.astype(np.int64)))
    h = np.array([oracle.arc_hash(seed, int(u), int(v), g.n) for u, v in zip(rows, g.col)], dtype=np.uint64)
    t = np.array([oracle.threshold(float(p)) for p in p_slot], dtype=np.uint64)
    x = np.array([oracle.sample_value(seed, r) for r in range(R)], dtype=np.uint64)
    return (h[:, None] ^ x[None, :]) < t[:, None]


@pytest.mark.parametrize("n,m,p,R,seed", [(12, 40, 0.3, 16, 1), (25, 90, 0.1, 24, 2), (40, 160, 0.5, 8, 3)])
def test_directed_reachability_matches_scipy(n, m, p, R, seed):
    g = random_small_digraph(n, m, seed)
    live = _live(g, np.full(g.nnz, p), R, seed)
    rng = np.random.default_rng(seed)
    for S in ([0], list(rng.choice(n, 3, replace=False)), list(range(n))):
        want = sum(_reach_scipy(g, live[:, r], S) for r in range(R))
        assert oracle.sigma_count(g, oracle.Sampler("hash", p=p, R=R, seed=seed), S) == want


def test_weighted_cascade_matches_scipy():
    g = random_small_digraph(30, 120, 6)
    g.p_slot = wc_p(g)
    R, seed = 20, 6
    live = _live(g, g.p_slot, R, seed)
    S = [1, 7, 20]
    want = sum(_reach_scipy(g, live[:, r], S) for r in range(R))
    assert oracle.sigma_count(g, oracle.Sampler("hash", R=R, seed=seed), S, threads=3) == want


def _greedy_scipy(g, live, K):
    """Plain greedy by exhaustive evaluation: per step every unselected vertex's
    spread with the current seeds, via scipy reachability; ties to the smaller id."""
    R = live.shape[1]
    S, marg = [], []
    base = 0
    for _ in range(K):
        best, arg = -1, None
        for u in range(g.n):
            if u in S:
                continue
            tot = sum(_reach_scipy(g, live[:, r], S + [u]) for r in range(R))
            if tot - base > best:
                best, arg = tot - base, u
        S.append(arg)
        marg.append(best)
        base += best
    return S, marg


@pytest.mark.parametrize("n,m,p,R,K,seed", [(10, 25, 0.35, 8, 4, 1), (14, 40, 0.2, 6, 5, 2), (9, 30, 0.6, 5, 9, 3)])
def test_directed_lazy_greedy_equals_plain_greedy(n, m, p, R, K, seed):
    g = random_small_digraph(n, m, seed)
    live = _live(g, np.full(g.nnz, p), R, seed)
    want_s, want_m = _greedy_scipy(g, live, K)
    got = oracle.celf_arcs(g, oracle.Sampler("hash", p=p, R=R, seed=seed), K)
    assert list(got["seeds"]) == want_s
    assert list(got["marginal"]) == want_m
    assert got["cover"] == sum(want_m)
    assert got["cover"] == oracle.sigma_count(g, oracle.Sampler("hash", p=p, R=R, seed=seed), want_s)


def test_directed_greedy_marginals_do_not_increase_and_k_over_n_fails():
    g = random_small_digraph(30, 120, 9)
    g.p_slot = wc_p(g)
    r = oracle.celf_arcs(g, oracle.Sampler("hash", R=32, seed=9), 30)
    assert np.all(np.diff(r["marginal"]) <= 0)
    assert r["cover"] == 32 * 30  # every vertex reached once all are seeds
    with pytest.raises(ValueError):
        oracle.celf_arcs(g, oracle.Sampler("hash", R=4, seed=9), 31)
