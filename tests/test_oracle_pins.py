"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Each test checks the oracle against something it cannot be circular with:
published hash test vectors, exact decimal arithmetic, closed forms,
brute-force enumeration of live-edge worlds, a library connected-components
routine, the paper's worked example (Fig. 4), and invariants of coverage
functions.  None of these tests needs a GPU.
"""

import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests.helpers import min_id_labels
from workloads import Graph, chung_lu, from_edge_list, random_small_graph, star_graph
from workloads.graphs import splitmix64_stream

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# P8: the hash finaliser
# ---------------------------------------------------------------------------

def test_fmix32_published_vectors():
    # MurmurHash3_x86_32 of the empty key with seed s is fmix32(s) (no block
    # or tail step runs and the length xor is 0).  Published verification
    # values: seed 0 -> 0, seed 1 -> 0x514E28B7, seed 0xFFFFFFFF -> 0x81F16F39.
    assert oracle.fmix32(0) == 0
    assert oracle.fmix32(1) == 0x514E28B7
    assert oracle.fmix32(0xFFFFFFFF) == 0x81F16F39


def test_fmix32_is_injective_on_a_block():
    # fmix32 is a bijection of uint32 (each step is invertible); no collision
    # may appear on a contiguous block of inputs.
    xs = [oracle.fmix32(x) for x in range(0, 1 << 16)]
    assert len(set(xs)) == len(xs)


def test_sample_value_definition():
    # X_r = fmix32(s + r) with 32-bit wrap-around of s + r.
    assert oracle.sample_value(1, 0) == 0x514E28B7
    assert oracle.sample_value(0xFFFFFFFF, 1) == 0  # s + r wraps to 0
    assert oracle.sample_value(0, 0xFFFFFFFF) == 0x81F16F39


# ---------------------------------------------------------------------------
# Thresholds: floor(p * 2^32) from the exact value of the IEEE double p
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("p", [0.1, 0.05, 0.02, 0.01, 0.005, 0.001, 0.5, 0.3, 1e-9, 2.0 ** -32,
                               0.999999, 1.0 - 2.0 ** -40])
def test_threshold_exact(p):
    want = math.floor(Fraction(p) * (1 << 32))
    assert oracle.threshold(p) == want


def test_threshold_printed_values_and_ends():
    table = {0.1: 429496729, 0.05: 214748364, 0.02: 85899345, 0.01: 42949672,
             0.005: 21474836, 0.001: 4294967}
    for p, t in table.items():
        assert oracle.threshold(p) == t
    assert oracle.threshold(0.0) == 0
    assert oracle.threshold(-0.5) == 0
    assert oracle.threshold(1.0) == 1 << 32
    assert oracle.threshold(float("nan")) == 0


def test_liveness_is_strict_unsigned_compare():
    # live iff (h ^ X) < T as unsigned 32-bit values; T = 2^32 keeps all.
    assert oracle.is_live(0x80000000, 0, 0x80000001)
    assert not oracle.is_live(0x80000000, 0, 0x80000000)
    assert oracle.is_live(0xFFFFFFFF, 0, 1 << 32)
    assert not oracle.is_live(0, 0, 0)
    assert oracle.is_live(5, 5, 1)


# ---------------------------------------------------------------------------
# Edge key (Eq. 1 hashes min || max): symmetric, equal to u*n+v below 2^32,
# folded without collisions above it
# ---------------------------------------------------------------------------

def test_edge_key_small_is_plain_key():
    n = 40000
    for (u, v) in [(0, 1), (5, 39999), (39998, 39999), (123, 4567)]:
        assert oracle.edge_key(u, v, n) == u * n + v
        assert oracle.edge_key(v, u, n) == u * n + v


def test_edge_key_fold_above_2_32():
    n = 1 << 18
    u, v = (1 << 14) + 7, (1 << 17) + 3  # u*n + v exceeds 2^32
    key = u * n + v
    assert key >= 1 << 32
    want = (key & 0xFFFFFFFF) ^ oracle.fmix32(key >> 32)
    assert oracle.edge_key(u, v, n) == want
    # a literal 32-bit wrap would make (u, v) and (u + 2^14, v) collide
    assert ((u * n + v) & 0xFFFFFFFF) == (((u + (1 << 14)) * n + v) & 0xFFFFFFFF)
    assert oracle.edge_key(u, v, n) != oracle.edge_key(u + (1 << 14), v, n)


def test_edge_hash_symmetric():
    for (u, v) in [(1, 2), (7, 3), (100, 99)]:
        assert oracle.edge_hash(9, u, v, 1000) == oracle.edge_hash(9, v, u, 1000)


# ---------------------------------------------------------------------------
# P6: forced-live closed form (independent of the finaliser's constants)
# ---------------------------------------------------------------------------

def test_forced_live_star():
    # Star centred at 0, seed s = 1, p = 1e-9 (T = 4).  Edge {0,v} has key v,
    # so h = fmix32(1 ^ v) and X_r = fmix32(1 + r).  Because fmix32 is a
    # bijection, h == X_r exactly when 1 ^ v == 1 + r, and then h ^ X_r = 0 < T:
    # even v -> r = v, odd v >= 3 -> r = v - 2.
    n, R = 200, 128
    g = star_graph(n)
    s = oracle.Sampler("hash", p=1e-9, R=R, seed=1)
    _, labels, _ = oracle.label_all(g, s, want_labels=True)
    for v in range(2, R, 2):
        assert labels[v, v] == 0
    for v in range(3, R + 2, 2):
        assert labels[v, v - 2] == 0


# ---------------------------------------------------------------------------
# P9: the worked example of Fig. 4
# ---------------------------------------------------------------------------

def test_fig4_worked_example():
    with open(os.path.join(GOLDEN, "fig4_worked_example.json")) as f:
        fx = json.load(f)
    names = fx["vertices"]
    idx = {a: i for i, a in enumerate(names)}
    n = len(names)
    pairs = list(itertools.combinations(range(n), 2))
    g = from_edge_list(n, np.array([p[0] for p in pairs]), np.array([p[1] for p in pairs]))
    und = [tuple(e) for e in g.undirected_edges().tolist()]
    assert len(und) == 10
    table = np.zeros((2, len(und)), dtype=np.uint8)
    for r, live in enumerate(fx["live"]):
        for a, b in live:
            e = und.index(tuple(sorted((idx[a], idx[b]))))
            table[r, e] = 1
    s = oracle.Sampler("table", R=2, table=table)
    _, labels, _ = oracle.label_all(g, s, want_labels=True)
    for r in range(2):
        assert [names[x] for x in labels[:, r]] == fx["expected_labels"][r]


# ---------------------------------------------------------------------------
# P1: exhaustive enumeration of live-edge worlds (every world once)
# ---------------------------------------------------------------------------

def _closure_reach(n, edges, mask, S):
    """|vertices reachable from S| in world `mask`, by Boolean matrix closure."""
    a = np.eye(n, dtype=bool)
    for e, (u, v) in enumerate(edges):
        if (mask >> e) & 1:
            a[u, v] = a[v, u] = True
    for _ in range(max(1, math.ceil(math.log2(max(n, 2))))):
        a = (a.astype(np.int64) @ a.astype(np.int64)) > 0
    if len(S) == 0:
        return 0
    return int(a[list(S)].any(axis=0).sum())


def _closure_components(n, edges, mask):
    a = np.eye(n, dtype=bool)
    for e, (u, v) in enumerate(edges):
        if (mask >> e) & 1:
            a[u, v] = a[v, u] = True
    for _ in range(max(1, math.ceil(math.log2(max(n, 2))))):
        a = (a.astype(np.int64) @ a.astype(np.int64)) > 0
    return np.array([int(np.argmax(a[v])) for v in range(n)], dtype=np.int32)


@pytest.mark.parametrize("n,m,seed", [(6, 8, 1), (7, 10, 2), (5, 10, 3), (8, 9, 4)])
def test_exhaustive_worlds(n, m, seed):
    g = random_small_graph(n, m, seed)
    edges = [tuple(e) for e in g.undirected_edges().tolist()]
    assert len(edges) == m
    R = 1 << m
    s = oracle.Sampler("enum", R=R)
    g0, labels, _ = oracle.label_all(g, s, want_labels=True)
    # every per-world partition equals the closure's (min-id) partition
    for mask in range(R):
        assert np.array_equal(labels[:, mask], _closure_components(n, edges, mask))

    # counts: f(S) = sum over worlds |reach(S)| = 2^m * exact IC sigma at p = 1/2
    def f(S):
        return sum(_closure_reach(n, edges, w, S) for w in range(R))

    for S in [(0,), (1, 2), (0, n - 1), tuple(range(n))]:
        assert oracle.sigma_count(g, s, S) == f(S)
    # initial gains = f({v})
    assert [int(x) for x in g0] == [f((v,)) for v in range(n)]
    # lazy greedy (CELF) == plain greedy on the exact function, lowest id on ties
    K = min(4, n)
    seeds, marg, cover, _ = oracle.celf(g, s, K, g0)
    S, fS = [], 0
    for k in range(K):
        best, arg = -1, -1
        for v in range(n):
            if v in S:
                continue
            gv = f(tuple(S + [v])) - fS
            if gv > best:
                best, arg = gv, v
        S.append(arg)
        assert seeds[k] == arg
        assert marg[k] == best
        fS += best
    assert cover == fS


# ---------------------------------------------------------------------------
# P2: hash worlds against scipy's connected components
# ---------------------------------------------------------------------------

def _hash_live_matrix(g, p, R, seed):
    und = g.undirected_edges()
    h = np.array([oracle.edge_hash(seed, int(u), int(v), g.n) for u, v in und], dtype=np.uint64)
    x = np.array([oracle.sample_value(seed, r) for r in range(R)], dtype=np.uint64)
    t = oracle.threshold(p)
    return und, (h[:, None] ^ x[None, :]) < np.uint64(t)


@pytest.mark.parametrize("p,R", [(0.05, 64), (0.3, 16), (0.002, 64)])
def test_hash_worlds_match_scipy_components(p, R):
    g = chung_lu(600, 2400, 2.5, 11)
    s = oracle.Sampler("hash", p=p, R=R, seed=11)
    _, labels, _ = oracle.label_all(g, s, want_labels=True)
    und, live = _hash_live_matrix(g, p, R, 11)
    for r in range(R):
        sel = live[:, r]
        want = min_id_labels(g.n, und[sel, 0], und[sel, 1])
        assert np.array_equal(labels[:, r], want), r


def test_label_range_matches_label_all():
    g = chung_lu(500, 1500, 2.5, 5)
    s = oracle.Sampler("hash", p=0.1, R=40, seed=5)
    _, labels, _ = oracle.label_all(g, s, want_labels=True, threads=3)
    part = oracle.label_range(g, s, 13, 9)
    assert np.array_equal(part, labels[:, 13:22])


# ---------------------------------------------------------------------------
# P5: special cases
# ---------------------------------------------------------------------------

def test_p_zero_all_singletons():
    g = chung_lu(300, 900, 2.5, 3)
    R, K = 32, 7
    s = oracle.Sampler("hash", p=0.0, R=R, seed=3)
    res = oracle.run(g, s, K, want_labels=True)
    assert np.array_equal(res["labels"], np.repeat(np.arange(g.n, dtype=np.int32)[:, None], R, 1))
    assert np.all(res["g0"] == R)
    assert list(res["seeds"]) == list(range(K))
    assert np.all(res["marginal"] == R)
    assert oracle.sigma_count(g, s, [4, 9, 9, 100]) == 3 * R


def test_p_one_every_sample_is_the_graph():
    g = chung_lu(400, 500, 2.5, 8)  # several components
    R, K = 8, 0
    und = g.undirected_edges()
    comp = min_id_labels(g.n, und[:, 0], und[:, 1])
    s = oracle.Sampler("hash", p=1.0, R=R, seed=8)
    g0, labels, _ = oracle.label_all(g, s, want_labels=True)
    assert np.all(labels == comp[:, None])
    sizes = np.bincount(comp, minlength=g.n)
    assert np.array_equal(g0, R * sizes[comp])
    # seeds: component minima by decreasing size (ties: smaller minimum),
    # then the lowest unselected ids at gain 0
    roots = np.unique(comp)
    order = sorted(roots, key=lambda c: (-sizes[c], c))
    K = len(order) + 5
    seeds, marg, cover, _ = oracle.celf(g, s, K, g0)
    assert list(seeds[:len(order)]) == [int(c) for c in order]
    assert list(marg[:len(order)]) == [int(R * sizes[c]) for c in order]
    rest = [v for v in range(g.n) if v not in set(order)][:5]
    assert list(seeds[len(order):]) == rest
    assert np.all(marg[len(order):] == 0)
    assert cover == R * g.n


# ---------------------------------------------------------------------------
# P4 / P10: invariants of the memo and of the coverage function
# ---------------------------------------------------------------------------

def _memo_gain(labels, u, S):
    """Memo formula of Section III-C: sum_r [l_u[r] not in {l_s[r]}] * size."""
    n, R = labels.shape
    tot = 0
    for r in range(R):
        col = labels[:, r]
        lu = col[u]
        if any(col[s] == lu for s in S):
            continue
        tot += int((col == lu).sum())
    return tot


def test_invariants_on_small_config():
    g = chung_lu(2000, 8000, 2.5, 1)
    R, K, p = 64, 8, 0.05
    s = oracle.Sampler("hash", p=p, R=R, seed=1)
    res = oracle.run(g, s, K, want_labels=True, threads=4)
    L = res["labels"]
    v = np.arange(g.n)
    assert np.all(L <= v[:, None])  # label is a vertex of the component <= v
    for r in range(R):
        col = L[:, r]
        assert np.array_equal(col[col], col)  # the label's own label is itself
        sizes = np.bincount(col, minlength=g.n)
        assert sizes.sum() == g.n
    # maximality: no live edge joins different labels
    und, live = _hash_live_matrix(g, p, R, 1)
    for r in range(R):
        e = und[live[:, r]]
        assert np.all(L[e[:, 0], r] == L[e[:, 1], r])
    # g0 = sum_r |C_r(v)| from the labels; sum_v g0 = sum_r sum_c |c|^2
    g0_from_labels = np.zeros(g.n, dtype=np.int64)
    sq = 0
    for r in range(R):
        sizes = np.bincount(L[:, r], minlength=g.n)
        g0_from_labels += sizes[L[:, r]]
        sq += int((sizes.astype(np.int64) ** 2).sum())
    assert np.array_equal(res["g0"], g0_from_labels)
    assert int(res["g0"].sum()) == sq
    # sigma({v}) = g0[v]
    for vv in (0, 3, 1999):
        assert oracle.sigma_count(g, s, [vv]) == res["g0"][vv]
    # marginals: non-increasing (submodular), equal to the memo formula and to
    # RandCas differences on the same samples; cover = sum of marginals
    seeds, marg = [int(x) for x in res["seeds"]], [int(x) for x in res["marginal"]]
    assert all(a >= b for a, b in zip(marg, marg[1:]))
    prev = 0
    for k in range(K):
        S = seeds[:k]
        assert marg[k] == _memo_gain(L, seeds[k], S)
        cur = oracle.sigma_count(g, s, seeds[:k + 1])
        assert cur - prev == marg[k]
        assert cur >= prev  # monotone
        prev = cur
    assert res["cover"] == sum(marg) == prev


def test_lazy_equals_plain_greedy():
    g = chung_lu(250, 700, 2.5, 21)
    R, K = 32, 6
    s = oracle.Sampler("hash", p=0.08, R=R, seed=21)
    res = oracle.run(g, s, K, want_labels=True)
    L = res["labels"]
    S = []
    for k in range(K):
        gains = [(-1 if v in S else _memo_gain(L, v, S)) for v in range(g.n)]
        best = max(gains)
        arg = gains.index(best)  # lowest id among maxima
        assert res["seeds"][k] == arg and res["marginal"][k] == best
        S.append(arg)


def test_gain_equals_randcas_difference():
    g = chung_lu(400, 1600, 2.5, 4)
    s = oracle.Sampler("hash", p=0.1, R=24, seed=4)
    S = [0, 5, 17]
    base = oracle.sigma_count(g, s, S)
    for u in (1, 2, 33, 399):
        assert oracle.gain(g, s, u, S) == oracle.sigma_count(g, s, S + [u]) - base


def test_threads_do_not_change_results():
    g = chung_lu(1500, 6000, 2.5, 9)
    s = oracle.Sampler("hash", p=0.05, R=48, seed=9)
    a = oracle.run(g, s, 5, want_labels=True, threads=1)
    b = oracle.run(g, s, 5, want_labels=True, threads=7)
    assert np.array_equal(a["labels"], b["labels"])
    assert np.array_equal(a["g0"], b["g0"])
    assert np.array_equal(a["seeds"], b["seeds"])
    assert np.array_equal(a["marginal"], b["marginal"])


def test_k_greater_than_n_rejected():
    g = star_graph(5)
    s = oracle.Sampler("hash", p=0.5, R=4, seed=1)
    g0, _, _ = oracle.label_all(g, s)
    with pytest.raises(ValueError):
        oracle.celf(g, s, 6, g0)


# ---------------------------------------------------------------------------
# P7: marginal behaviour of the hash sampler (Fig. 2)
# ---------------------------------------------------------------------------

def test_per_edge_live_frequency_binomial():
    g = chung_lu(2000, 8000, 2.5, 1)
    p, R = 0.05, 4096
    _, live = _hash_live_matrix(g, p, R, 1)
    q = oracle.threshold(p) / 2.0 ** 32
    cnt = live.sum(axis=1)
    sd = math.sqrt(R * q * (1 - q))
    assert np.all(np.abs(cnt - R * q) <= 6 * sd)


def test_sampling_probability_cdf_is_uniform():
    from scipy import stats

    g = chung_lu(2000, 8000, 2.5, 1)
    und = g.undirected_edges()
    h = np.array([oracle.edge_hash(1, int(u), int(v), g.n) for u, v in und], dtype=np.uint64)
    x = np.array([oracle.sample_value(1, r) for r in range(256)], dtype=np.uint64)
    rho = ((h[:, None] ^ x[None, :]).astype(np.float64) / 2.0 ** 32).ravel()
    d = stats.kstest(rho, "uniform").statistic
    assert d < 0.005  # maximum bias well below 0.5%


# ---------------------------------------------------------------------------
# P3: the sampler's own exact expectation, over all 2^32 values of X
# ---------------------------------------------------------------------------

def _exact_world_counts(h, T):
    """Number of X in [0, 2^32) producing each live-edge mask, computed by
    splitting the X range on its bits (each edge is live on h ^ [0, T))."""
    counts = {}
    m = len(h)

    def rec(prefix, depth, fixed_mask, open_edges):
        width = 1 << (32 - depth)
        if not open_edges:
            counts[fixed_mask] = counts.get(fixed_mask, 0) + width
            return
        for bit in (0, 1):
            pre = (prefix << 1) | bit
            d = depth + 1
            w = 1 << (32 - d)
            mask, still = fixed_mask, []
            for e in open_edges:
                base = (pre ^ (h[e] >> (32 - d))) << (32 - d)  # block of h ^ X values
                if base + w <= T:
                    mask |= 1 << e
                elif base >= T:
                    pass
                else:
                    still.append(e)
            rec(pre, d, mask, still)

    rec(0, 0, 0, list(range(m)))
    assert sum(counts.values()) == 1 << 32
    return counts


def test_hash_sampler_matches_its_exact_expectation():
    g = random_small_graph(6, 7, 12)
    edges = [tuple(e) for e in g.undirected_edges().tolist()]
    seed, p = 77, 0.3
    T = oracle.threshold(p)
    h = [oracle.edge_hash(seed, u, v, g.n) for u, v in edges]
    counts = _exact_world_counts(h, T)
    for S in [(0,), (2, 5)]:
        vals = {mask: _closure_reach(g.n, edges, mask, S) for mask in counts}
        mean = sum(c * vals[k] for k, c in counts.items()) / 2.0 ** 32
        var = sum(c * (vals[k] - mean) ** 2 for k, c in counts.items()) / 2.0 ** 32
        R = 1 << 14
        s = oracle.Sampler("hash", p=p, R=R, seed=seed)
        est = oracle.sigma_count(g, s, S) / R
        assert abs(est - mean) <= 5 * math.sqrt(var / R) + 1e-12


# ---------------------------------------------------------------------------
# The memo-formula CELF (Algorithm 7's evaluation from stored labels and
# sizes) against the RandCas CELF (Algorithm 3's re-simulation) on the same
# samples: identical seeds and marginals
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,m,p,R,K,seed", [(600, 2400, 0.05, 64, 12, 2), (1500, 4000, 0.2, 32, 9, 3),
                                            (300, 1500, 0.01, 200, 20, 4), (80, 200, 1.0, 8, 30, 5),
                                            (50, 120, 0.0, 16, 50, 6), (400, 1600, 0.3, 24, 400, 7)])
def test_memo_celf_equals_randcas_celf(n, m, p, R, K, seed):
    g = chung_lu(n, m, 2.4, seed)
    s = oracle.Sampler("hash", p=p, R=R, seed=seed)
    a = oracle.run(g, s, K, threads=2)
    b = oracle.run_memo(g, s, K, threads=2, keep_arrays=True)
    assert np.array_equal(a["g0"], b["g0"])
    assert list(a["seeds"]) == list(b["seeds"])
    assert list(a["marginal"]) == list(b["marginal"])
    assert a["cover"] == b["cover"]
    # sizes are the per-vertex component sizes of the labels
    L, Z = b["labels"], b["sizes"]
    for r in range(R):
        cnt = np.bincount(L[:, r], minlength=n)
        assert np.array_equal(Z[:, r], cnt[L[:, r]])
