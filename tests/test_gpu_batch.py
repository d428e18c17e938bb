"""Batched memo construction (im_batch_select): the memos built together,
one launch per labelling phase over all graphs, must be the memos of the
single-graph path, element by element against the oracle: labels, component
sizes and initial gains of every graph, then the seeds.

The batch mixes what the per-graph descriptors must carry: uniform and
per-edge probabilities, vertices with more than 64 neighbours (hub kernels),
a ragged R, an R above the batched set-up's single-workgroup sort (sorted
beforehand), p = 0 (nothing live), a one-vertex graph, K = 0, and a graph
whose memo is already resident (not rebuilt).
"""

import numpy as np
import pytest

import oracle
import paper_2008_03095_amd as P
from tests.conftest import announce
from tests.helpers import hub_mix_graph
from workloads import chung_lu, from_edge_list, star_graph, trivalency_p, uniform_p

pytestmark = pytest.mark.gpu


def _sizes_from_labels(L):
    out = np.empty_like(L)
    for r in range(L.shape[1]):
        cnt = np.bincount(L[:, r], minlength=L.shape[0])
        out[:, r] = cnt[L[:, r]]
    return out


def _specs():
    g_tri = chung_lu(1200, 5000, 2.2, 81)
    g_tri.p_slot = trivalency_p(g_tri, 81)
    g_uni = chung_lu(900, 4000, 2.1, 82)
    g_uni.p_slot = uniform_p(g_uni, 82)
    g_hub_tri = hub_mix_graph(88)
    g_hub_tri.p_slot = trivalency_p(g_hub_tri, 88)
    return [
        # (graph, p, R, hash seed, K)
        (chung_lu(1500, 7000, 2.1, 80), 0.06, 512, 80, 15),   # hubs, uniform p
        (g_tri, 0.0, 300, 81, 9),                             # per-edge p, ragged R
        (g_uni, 0.0, 1024, 82, 0),                            # per-edge p, K = 0
        (star_graph(300), 0.2, 256, 83, 5),                   # one hub of 299 neighbours
        (chung_lu(600, 2000, 2.5, 84), 0.04, 5000, 84, 7),    # R above the set-up sort's size
        (chung_lu(500, 1500, 2.5, 85), 0.0, 256, 85, 4),      # p = 0: all singletons
        (from_edge_list(1, [], []), 0.3, 64, 86, 1),          # one vertex, no edge
        (hub_mix_graph(89), 0.02, 1024, 89, 6),               # hub rows of 100 to 5,000 slots
        (g_hub_tri, 0.0, 300, 88, 6),                         # the same, per-edge p, ragged R
        (chung_lu(700, 2500, 2.3, 90), 0.05, 9000, 90, 5),    # 36 tiles: two mask words per vertex
    ]


def test_batched_memos_equal_the_oracle(gpu_ctx):
    specs = _specs()
    announce(f"batched construction of {len(specs)} memos")
    Gs = []
    try:
        for g, p, R, s, K in specs:
            G = P.Graph.from_csr(gpu_ctx, g)
            G.set_params(p, R, s)
            Gs.append(G)
        Gs[3].build_memo()  # resident before the call: found, not rebuilt
        res = P.batch_select(gpu_ctx, Gs, [K for *_, K in specs])
        for (g, p, R, s, K), G, (seeds, marg, cover) in zip(specs, Gs, res):
            samp = oracle.Sampler("hash", p=p, R=R, seed=s)
            g0, L, _ = oracle.label_all(g, samp, want_labels=True, threads=4)
            assert np.array_equal(G.labels(), L), (g.n, R)
            assert np.array_equal(G.sizes(), _sizes_from_labels(L)), (g.n, R)
            assert np.array_equal(G.gains0(), g0), (g.n, R)
            if K == 0:
                assert len(seeds) == 0 and cover == 0
                continue
            ref = oracle.run_memo(g, samp, K, threads=4)
            assert list(seeds) == list(ref["seeds"]), (g.n, R, K)
            assert list(marg) == list(ref["marginal"])
            assert cover == ref["cover"]
    finally:
        for G in Gs:
            G.free()


def test_batch_rejects_a_repeated_graph(gpu_ctx):
    g = chung_lu(300, 900, 2.5, 87)
    G = P.Graph.from_csr(gpu_ctx, g)
    try:
        G.set_params(0.05, 256, 87)
        with pytest.raises(P.InfuseError) as e:
            P.batch_select(gpu_ctx, [G, G], [3, 3])
        assert e.value.status == 1
    finally:
        G.free()


def test_batch_more_selections_than_workgroups(gpu_ctx):
    # 640 selections: more than the persistent grid's workgroups, so each
    # workgroup runs several selections one after the other
    from workloads import random_small_graph
    specs = [(random_small_graph(12 + i % 20, 20 + i % 37, 500 + i), 0.3, 64, 500 + i, 1 + i % 4)
             for i in range(640)]
    announce(f"batch_select of {len(specs)} small graphs")
    Gs = []
    try:
        for g, p, R, s, K in specs:
            G = P.Graph.from_csr(gpu_ctx, g)
            G.set_params(p, R, s)
            Gs.append(G)
        res = P.batch_select(gpu_ctx, Gs, [K for *_, K in specs])
        for (g, p, R, s, K), (seeds, marg, cover) in zip(specs, res):
            ref = oracle.run_memo(g, oracle.Sampler("hash", p=p, R=R, seed=s), K, threads=1)
            assert list(seeds) == list(ref["seeds"]), (g.n, K, s)
            assert list(marg) == list(ref["marginal"])
            assert cover == ref["cover"]
    finally:
        for G in Gs:
            G.free()
