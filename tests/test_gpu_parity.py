"""GPU parity: the HIP library against the CPU oracle, element by element.

Labels, component sizes, initial gains, seeds, marginal counts, cover counts
and sigma counts are integers and must be identical.
"""

import numpy as np
import pytest

import oracle
import paper_2008_03095_amd as P
from tests.conftest import announce
from tests.helpers import digest_weights, hub_mix_graph, label_digests
from workloads import (chung_lu, from_edge_list, make_config, normal_p, path_graph, random_small_graph,
                       star_graph, trivalency_p, uniform_p)

pytestmark = pytest.mark.gpu


def _sizes_from_labels(L):
    out = np.empty_like(L)
    for r in range(L.shape[1]):
        cnt = np.bincount(L[:, r], minlength=L.shape[0])
        out[:, r] = cnt[L[:, r]]
    return out


def _full_check(ctx, g, p, R, seed, K, sigma_sets=(), name=""):
    announce(f"{name} n={g.n} m={g.m} p={p} R={R} s={seed} K={K}")
    s = oracle.Sampler("hash", p=p, R=R, seed=seed)
    ref = oracle.run(g, s, K, want_labels=True, threads=4)
    G = P.Graph.from_csr(ctx, g)
    try:
        G.set_params(p, R, seed)
        seeds, marg, cover = G.select_seeds(K)
        L = G.labels()
        assert np.array_equal(L, ref["labels"]), "labels differ"
        assert np.array_equal(G.sizes(), _sizes_from_labels(ref["labels"])), "sizes differ"
        assert np.array_equal(G.gains0(), ref["g0"]), "initial gains differ"
        assert list(seeds) == list(ref["seeds"]), (list(seeds), list(ref["seeds"]))
        assert list(marg) == list(ref["marginal"])
        assert cover == ref["cover"]
        for S in sigma_sets:
            S = [x for x in S if x < g.n]
            cnt, sig = G.estimate_sigma(S)
            want = oracle.sigma_count(g, s, S) if len(S) else 0
            assert cnt == want, (S, cnt, want)
            assert sig == pytest.approx(want / R)
    finally:
        G.free()


def test_c1_full(gpu_ctx):
    w = make_config("c1")
    g = w.graphs[0]
    _full_check(gpu_ctx, g, w.p, w.R, w.seeds[0], w.K,
                sigma_sets=[[0], [0, 3, 2], list(range(0, 2000, 37)), [5, 5, 5, 1999]], name="c1")


SMALL_GRAPHS = {
    "rand9x14": lambda: random_small_graph(9, 14, 3),
    "star40": lambda: star_graph(40),
    "path50": lambda: path_graph(50),
    "empty7": lambda: from_edge_list(7, np.empty(0, np.int64), np.empty(0, np.int64)),
    "single": lambda: from_edge_list(1, np.empty(0, np.int64), np.empty(0, np.int64)),
    "cl300": lambda: chung_lu(300, 1200, 2.3, 17),
}


@pytest.mark.parametrize("gname", list(SMALL_GRAPHS))
@pytest.mark.parametrize("R", [1, 63, 64, 65, 100, 256, 300])
def test_small_graphs_ragged_R(gpu_ctx, gname, R):
    g = SMALL_GRAPHS[gname]()
    K = min(5, g.n)
    _full_check(gpu_ctx, g, 0.3, R, 7, K, sigma_sets=[[0], [0, 1, 2]], name=f"{gname} R={R}")


@pytest.mark.parametrize("p", [0.0, 2.0 ** -32, 0.01, 0.5, 1.0])
def test_probability_extremes(gpu_ctx, p):
    g = chung_lu(400, 1500, 2.5, 23)
    _full_check(gpu_ctx, g, p, 130, 23, 6, sigma_sets=[[1, 2, 3]], name=f"p={p}")


def test_forced_live_star(gpu_ctx):
    # same closed form as the oracle pin: edge {0,v} is live in column v
    # (even v) and v - 2 (odd v >= 3) for s = 1 and T = 4
    announce("forced-live star")
    g = star_graph(200)
    G = P.Graph.from_csr(gpu_ctx, g)
    try:
        G.set_params(1e-9, 128, 1)
        L = G.labels()
        for v in range(2, 128, 2):
            assert L[v, v] == 0
        for v in range(3, 130, 2):
            assert L[v, v - 2] == 0
    finally:
        G.free()


def test_per_slot_probabilities(gpu_ctx):
    g = chung_lu(3000, 15000, 2.5, 101)
    g.p_slot = trivalency_p(g, 101)
    _full_check(gpu_ctx, g, 0.0, 512, 101, 8, sigma_sets=[[0, 1], [10, 20, 30]], name="trivalency")


@pytest.mark.parametrize("setting", ["uniform", "normal"])
def test_weight_settings(gpu_ctx, setting):
    # the paper's other weight settings as per-slot probabilities: U[0, 0.1]
    # and N(0.05, 0.025) clipped; a graph with hubs (degree > 64) and ragged R
    g = chung_lu(4000, 30000, 2.1, 7)
    assert int((g.degrees() > 64).sum()) > 0
    g.p_slot = uniform_p(g, 7) if setting == "uniform" else normal_p(g, 7)
    _full_check(gpu_ctx, g, 0.0, 600, 7, 15, sigma_sets=[[0, 5, 9], list(range(0, 4000, 97))],
                name=f"weights {setting}")


def test_per_slot_zero_and_one(gpu_ctx):
    g = chung_lu(500, 2000, 2.5, 5)
    vals = np.array([0.0, 1.0, 0.05, 0.5])
    und_key = {}
    rows = np.repeat(np.arange(g.n), g.degrees())
    ps = np.empty(g.nnz)
    for j, (u, v) in enumerate(zip(rows, g.col)):
        k = (min(u, v), max(u, v))
        if k not in und_key:
            und_key[k] = vals[len(und_key) % 4]
        ps[j] = und_key[k]
    g.p_slot = ps
    _full_check(gpu_ctx, g, 0.0, 200, 9, 5, sigma_sets=[[0, 1]], name="p_slot {0,1,...}")


@pytest.mark.parametrize("probs", ["uniform", "trivalency"])
@pytest.mark.parametrize("R", [300, 1024])
def test_hub_rows_of_several_lengths(gpu_ctx, probs, R):
    g = hub_mix_graph(91)
    deg = g.degrees()
    assert deg.max() >= 5000 and int(((deg > 64) & (deg < 1000)).sum()) > 10
    p = 0.02
    if probs == "trivalency":
        g.p_slot = trivalency_p(g, 91)
        p = 0.0
    _full_check(gpu_ctx, g, p, R, 91, 10, sigma_sets=[[g.n - 1, 3], [0, 1, 4500]],
                name=f"hub mix {probs} R={R}")


@pytest.mark.parametrize("R", [8448, 9000, 20000])
def test_more_than_32_tiles(gpu_ctx, R):
    # R above 8,192 columns: more than one tile-mask word per vertex (33, 36
    # and 79 tiles; the last two ragged)
    g = chung_lu(800, 3000, 2.3, 55)
    _full_check(gpu_ctx, g, 0.05, R, 55, 10, sigma_sets=[[0, 1, 2], list(range(0, 800, 7))], name=f"R={R}")


def test_c2_full(gpu_ctx):
    w = make_config("c2")
    g = w.graphs[0]
    announce("c2")
    s = oracle.Sampler("hash", p=w.p, R=w.R, seed=w.seeds[0])
    dw = digest_weights(g.n)
    ref = oracle.run(g, s, w.K, digest_w=dw, threads=8)
    G = P.Graph.from_csr(gpu_ctx, g)
    try:
        G.set_params(w.p, w.R, w.seeds[0])
        seeds, marg, cover = G.select_seeds(w.K)
        assert np.array_equal(G.gains0(), ref["g0"])
        assert list(seeds) == list(ref["seeds"])
        assert list(marg) == list(ref["marginal"])
        assert cover == ref["cover"]
        for r0 in range(0, w.R, 512):
            L = G.labels(r0, 512)
            assert np.array_equal(label_digests(L, dw), ref["digests"][r0:r0 + 512])
        for S in ([0], [1, 2, 3], list(range(0, 15000, 301))):
            assert G.estimate_sigma(S)[0] == oracle.sigma_count(g, s, S, threads=8)
    finally:
        G.free()


def test_k_zero_and_k_n(gpu_ctx):
    g = chung_lu(60, 150, 2.5, 2)
    announce("K=0 and K=n")
    s = oracle.Sampler("hash", p=0.2, R=64, seed=2)
    ref = oracle.run(g, s, g.n)
    G = P.Graph.from_csr(gpu_ctx, g)
    try:
        G.set_params(0.2, 64, 2)
        seeds, marg, cover = G.select_seeds(0)
        assert len(seeds) == 0 and cover == 0
        seeds, marg, cover = G.select_seeds(g.n)
        assert list(seeds) == list(ref["seeds"]) and list(marg) == list(ref["marginal"])
        assert sorted(seeds) == list(range(g.n))
        assert cover == g.n * 64
        with pytest.raises(P.InfuseError):
            G.select_seeds(g.n + 1)
        with pytest.raises(P.InfuseError):
            G.estimate_sigma([g.n])
        assert G.estimate_sigma([]) == (0, 0.0)
    finally:
        G.free()


def test_large_seed_set_sigma(gpu_ctx):
    # more seeds than the pairwise kernel handles: the bitmap kernel runs
    g = chung_lu(3000, 9000, 2.5, 31)
    announce("sigma |S| = 400")
    s = oracle.Sampler("hash", p=0.05, R=300, seed=31)
    S = list(range(0, 3000, 7))[:400] + [0, 7]
    G = P.Graph.from_csr(gpu_ctx, g)
    try:
        G.set_params(0.05, 300, 31)
        assert G.estimate_sigma(S)[0] == oracle.sigma_count(g, s, S, threads=4)
    finally:
        G.free()


def test_invalid_graphs_rejected(gpu_ctx):
    announce("invalid graphs")
    ok = star_graph(4)
    bad_rows = [
        (4, np.array([0, 1, 2, 3, 3], np.uint64), np.array([1, 0, 0, 0], np.uint32)),  # asymmetric
        (3, np.array([0, 1, 2, 2], np.uint64), np.array([0, 0], np.uint32)),  # self loop
        (3, np.array([0, 2, 3, 4], np.uint64), np.array([1, 1, 0, 0], np.uint32)),  # duplicate
        (2, np.array([0, 1, 2], np.uint64), np.array([5, 0], np.uint32)),  # id >= n
    ]
    for n, rp, col in bad_rows:
        with pytest.raises(P.InfuseError) as e:
            P.Graph(gpu_ctx, n, rp, col)
        assert e.value.status == 2
    with pytest.raises(P.InfuseError):
        P.Graph(gpu_ctx, ok.n, ok.row_ptr, ok.col, p_slot=np.full(ok.nnz, 1.5))
    G = P.Graph.from_csr(gpu_ctx, ok)
    try:
        with pytest.raises(P.InfuseError):
            G.set_params(0.1, 0, 1)
        with pytest.raises(P.InfuseError):
            G.set_params(float("nan"), 10, 1)
    finally:
        G.free()


def test_tuning_variants_and_repeats_identical(gpu_ctx):
    # race check: repeated builds and every launch shape give the same bytes
    g = chung_lu(5000, 30000, 2.3, 77)
    announce("determinism across tunings")
    G = P.Graph.from_csr(gpu_ctx, g)
    old = gpu_ctx.tuning()
    try:
        G.set_params(0.08, 1024, 77)
        base = G.labels()
        base_sel = G.select_seeds(12)
        for chunk in (256, 512, 1024, 4096, 8192):
            for width in (1, 4, 33):
                gpu_ctx.set_tuning(cc_chunk=chunk, celf_width=width)
                G.drop_memo()
                assert np.array_equal(G.labels(), base)
                sel = G.select_seeds(12)
                assert list(sel[0]) == list(base_sel[0]) and list(sel[1]) == list(base_sel[1])
    finally:
        gpu_ctx.set_tuning(cc_chunk=old["cc_chunk"], celf_width=old["celf_width"])
        G.free()


CELF_CASES = {
    # more seeds than the persistent kernel's candidate pool: repeated pool rebuilds
    "cl5000_K2500": (lambda: chung_lu(5000, 20000, 2.3, 5), 0.03, 512, 5, 2500),
    # every vertex selected; the pool holds the whole graph
    "cl300_Kn": (lambda: chung_lu(300, 1200, 2.3, 17), 0.1, 64, 17, 300),
    # long path, large components, few tiles
    "path3000": (lambda: path_graph(3000), 0.9, 256, 9, 40),
    # ragged R (last tile partly used), zero-gain rounds towards the end
    "star500_R300": (lambda: star_graph(500), 0.3, 300, 4, 499),
    # 36 tiles: two tile-mask words per vertex (the bulk pass's dense path)
    "cl800_R9000": (lambda: chung_lu(800, 3000, 2.3, 56), 0.05, 9000, 56, 12),
}


CELF_VARIANTS = {
    "persistent": (P.Context.CELF_PERSISTENT, 0, False),
    # one candidate in a step's first round: many rounds, pool refills and bulk passes
    "persistent_round1": (P.Context.CELF_PERSISTENT, 1, False),
    "per_step": (P.Context.CELF_PER_STEP, 0, False),
    # the per-step launches captured into one hipGraph
    "per_step_graph": (P.Context.CELF_PER_STEP, 0, True),
}


@pytest.mark.parametrize("variant", list(CELF_VARIANTS))
@pytest.mark.parametrize("case", list(CELF_CASES))
def test_celf_modes(gpu_ctx, case, variant):
    mode, round0, graphs = CELF_VARIANTS[variant]
    make, p, R, seed, K = CELF_CASES[case]
    g = make()
    announce(f"CELF {variant} {case} n={g.n} K={K}")
    ref = oracle.run_memo(g, oracle.Sampler("hash", p=p, R=R, seed=seed), K, threads=4)
    old = gpu_ctx.tuning()
    G = P.Graph.from_csr(gpu_ctx, g)
    try:
        gpu_ctx.set_tuning(celf_mode=mode, celf_round0=round0, use_graphs=graphs)
        G.set_params(p, R, seed)
        seeds, marg, cover = G.select_seeds(K)
        assert list(seeds) == list(ref["seeds"])
        assert list(marg) == list(ref["marginal"])
        assert cover == ref["cover"]
    finally:
        gpu_ctx.set_tuning(celf_mode=old["celf_mode"], celf_round0=old["celf_round0"],
                           use_graphs=old["use_graphs"])
        G.free()


@pytest.mark.parametrize("variant", ["persistent", "per_step"])
def test_batch_select_mixed(gpu_ctx, variant):
    # graphs of different sizes and parameters in one call; K = 0, K = n and
    # more graphs than one workgroup each would get with equal groups
    mode, round0, _ = CELF_VARIANTS[variant]
    specs = [
        (chung_lu(400, 1600, 2.5, 41), 0.05, 256, 41, 0),
        (chung_lu(900, 3000, 2.3, 42), 0.02, 512, 42, 12),
        (star_graph(150), 0.3, 300, 43, 150),
        (path_graph(700), 0.9, 256, 44, 25),
        (chung_lu(2500, 9000, 2.5, 45), 0.03, 1024, 45, 40),
    ] + [(chung_lu(200 + 37 * i, 800 + 90 * i, 2.5, 60 + i), 0.05, 256, 60 + i, 3 + i % 7) for i in range(40)]
    announce(f"batch_select {variant} {len(specs)} graphs")
    old = gpu_ctx.tuning()
    Gs = []
    try:
        gpu_ctx.set_tuning(celf_mode=mode, celf_round0=round0)
        for g, p, R, s, K in specs:
            G = P.Graph.from_csr(gpu_ctx, g)
            G.set_params(p, R, s)
            Gs.append(G)
        res = P.batch_select(gpu_ctx, Gs, [K for *_, K in specs])
        for (g, p, R, s, K), (seeds, marg, cover) in zip(specs, res):
            if K == 0:
                assert len(seeds) == 0 and cover == 0
                continue
            ref = oracle.run_memo(g, oracle.Sampler("hash", p=p, R=R, seed=s), K, threads=4)
            assert list(seeds) == list(ref["seeds"]), (g.n, K)
            assert list(marg) == list(ref["marginal"])
            assert cover == ref["cover"]
    finally:
        gpu_ctx.set_tuning(celf_mode=old["celf_mode"], celf_round0=old["celf_round0"])
        for G in Gs:
            G.free()


def test_autotune_picks_a_shape_and_keeps_results(gpu_ctx, tmp_path):
    g = chung_lu(3000, 20000, 2.1, 8)
    announce("autotune")
    old = gpu_ctx.tuning()
    G = P.Graph.from_csr(gpu_ctx, g)
    try:
        G.set_params(0.04, 512, 8)
        cache = str(tmp_path / "tuning.json")
        t = gpu_ctx.autotune(G, 12, reps=1, cache=cache)
        assert t["cc_chunk"] in (256, 512, 1024)
        assert t["list_blocks"] in (2048, 8192, 32768)
        if t["celf_mode"] == P.Context.CELF_PERSISTENT:
            assert t["celf_round0"] in (8, 16, 32)
        again = gpu_ctx.autotune(G, 12, reps=1, cache=cache)  # from the cache
        assert again["cc_chunk"] == t["cc_chunk"] and again["celf_round0"] == t["celf_round0"]
        assert again["list_blocks"] == t["list_blocks"]
        ref = oracle.run_memo(g, oracle.Sampler("hash", p=0.04, R=512, seed=8), 12, threads=4)
        seeds, marg, cover = G.select_seeds(12)
        assert list(seeds) == list(ref["seeds"]) and cover == ref["cover"]
    finally:
        gpu_ctx.set_tuning(cc_chunk=old["cc_chunk"], celf_mode=old["celf_mode"], celf_round0=old["celf_round0"],
                           list_blocks=old["list_blocks"])
        G.free()


DIRECT_CASES = {
    "c1": (lambda: make_config("c1").graphs[0], 0.05, 256, 1, None),
    "star300_R300": (lambda: star_graph(300), 0.2, 300, 3, None),
    "path400_dense": (lambda: path_graph(400), 0.97, 128, 5, None),
    "empty7": (lambda: from_edge_list(7, np.empty(0, np.int64), np.empty(0, np.int64)), 0.5, 64, 1, None),
    "p0": (lambda: chung_lu(500, 2000, 2.5, 9), 0.0, 256, 9, None),
    "p1": (lambda: chung_lu(500, 2000, 2.5, 9), 1.0, 64, 9, None),
    "hubs_uniform_w": (lambda: chung_lu(4000, 30000, 2.1, 7), 0.0, 600, 7, "uniform"),
    "trivalency": (lambda: chung_lu(3000, 15000, 2.5, 101), 0.0, 512, 101, "trivalency"),
    # 36 tiles of samples: per-(vertex, tile) frontier items beyond one mask word
    "wide_R9000": (lambda: chung_lu(800, 3000, 2.3, 57), 0.05, 9000, 57, None),
}


@pytest.mark.parametrize("case", list(DIRECT_CASES))
def test_sigma_without_memo(gpu_ctx, case):
    make, p, R, seed, w = DIRECT_CASES[case]
    g = make()
    if w == "uniform":
        g.p_slot = uniform_p(g, seed)
    elif w == "trivalency":
        g.p_slot = trivalency_p(g, seed)
    announce(f"sigma without memo {case} n={g.n} R={R}")
    s = oracle.Sampler("hash", p=p, R=R, seed=seed)
    sets = [[0], [0, g.n - 1], list(range(0, g.n, max(1, g.n // 37))), [1, 1, 2, 2, 3]]
    G = P.Graph.from_csr(gpu_ctx, g)
    try:
        G.set_params(p, R, seed)
        for S in sets:
            S = [x for x in S if x < g.n]
            cnt, sig, levels = G.estimate_sigma_direct(S)
            want = oracle.sigma_count(g, s, S, threads=4)
            assert cnt == want, (S[:5], cnt, want)
            assert sig == pytest.approx(want / R)
            if p == 0.0 and w is None:
                assert cnt == len(set(S)) * R
        assert G.estimate_sigma_direct([]) == (0, 0.0, 0)
        with pytest.raises(P.InfuseError):
            G.estimate_sigma_direct([g.n])
    finally:
        G.free()
