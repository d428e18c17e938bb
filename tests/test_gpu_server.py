"""Serving loop (im_server_*): every result is the same alone and in the mix.

Queries of both kinds, on several graphs and parameter sets, are first run
one at a time through the direct calls, then submitted together to a server
whose slots overlap them on the device; seeds, marginal counts and sigma
counts must be identical (integers).  A subset is also checked against the
oracle.  Cancellation, statistics and budget rejection are covered too.
"""

import numpy as np
import pytest

import oracle
import paper_2008_03095_amd as P
from tests.conftest import announce
from workloads import chung_lu, rmat

pytestmark = pytest.mark.gpu


def _graphs():
    return [
        chung_lu(2000, 8000, 2.5, 11),
        chung_lu(3000, 15000, 2.3, 12),
        rmat(12, 6, 0.57, 0.19, 0.19, 13),
    ]


def _queries(graphs, n_queries=48, seed=5):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_queries):
        gi = int(rng.integers(len(graphs)))
        p = float(rng.choice([0.01, 0.03, 0.08]))
        R = int(rng.choice([256, 300, 1024]))
        s = int(rng.choice([4, 9]))
        if rng.random() < 0.6:
            k = int(rng.integers(1, 40))
            S = rng.choice(graphs[gi].n, size=k, replace=False).astype(np.uint32)
            out.append(("sigma", gi, p, R, s, S))
        else:
            out.append(("select", gi, p, R, s, int(rng.choice([5, 20, 50]))))
    return out


def _alone(ctx, Gs, q):
    kind, gi, p, R, s, arg = q
    G = Gs[gi]
    G.set_params(p, R, s)
    if kind == "sigma":
        return G.estimate_sigma(arg)[0]
    seeds, marg, cover = G.select_seeds(arg)
    return (list(seeds), list(marg), cover)


@pytest.mark.parametrize("persistent_min_mwords", [0, 0xFFFFFFFF])
def test_server_results_alone_equal_mixed(gpu_ctx, persistent_min_mwords):
    # 0 (default): every selection runs the persistent kernel, which holds
    # back the other slots; 0xFFFFFFFF: every selection runs the per-step
    # kernels beside the other slots
    graphs = _graphs()
    qs = _queries(graphs)
    announce(f"server mix of {len(qs)} queries, persistent_min_mwords={persistent_min_mwords}")
    Gs = [P.Graph.from_csr(gpu_ctx, g) for g in graphs]
    try:
        alone = [_alone(gpu_ctx, Gs, q) for q in qs]
        for G in Gs:
            G.drop_memo()
        srv = P.Server(gpu_ctx, slots=4, persistent_min_mwords=persistent_min_mwords)
        try:
            tickets = []
            for kind, gi, p, R, s, arg in qs:
                if kind == "sigma":
                    tickets.append(srv.submit_sigma(Gs[gi], arg, p, R, s))
                else:
                    tickets.append(srv.submit_select(Gs[gi], arg, p, R, s))
            results = [srv.poll(t, wait_ms=120000) for t in tickets]
            stats = srv.stats()
        finally:
            srv.close()
        for q, a, r in zip(qs, alone, results):
            assert r is not None and r["status"] == 0, (q[:5], r)
            if q[0] == "sigma":
                assert r["count"] == a, (q[:5], r["count"], a)
                assert r["sigma"] == pytest.approx(a / q[3])
            else:
                assert list(r["seeds"]) == a[0], q[:5]
                assert list(r["marginal"]) == a[1], q[:5]
                assert r["count"] == a[2]
        assert stats["completed"] == len(qs)
        assert stats["admitted"] == len(qs) and stats["rejected"] == 0
        assert stats["memo_hits"] + stats["memo_builds"] == len(qs)
        assert stats["memo_hits"] > 0  # repeated (graph, p, R, s) reuse resident memos
        assert stats["peak_concurrent"] > 1  # queries overlapped on the device
        # a few of the mixed results against the oracle
        for (kind, gi, p, R, s, arg), a in list(zip(qs, alone))[:6]:
            samp = oracle.Sampler("hash", p=p, R=R, seed=s)
            if kind == "sigma":
                assert a == oracle.sigma_count(graphs[gi], samp, list(arg), threads=4)
            else:
                ref = oracle.run_memo(graphs[gi], samp, arg, threads=4)
                assert a[0] == list(ref["seeds"]) and a[1] == list(ref["marginal"])
    finally:
        for G in Gs:
            G.free()


def test_server_cancel_and_empty(gpu_ctx):
    g = chung_lu(1500, 6000, 2.5, 21)
    announce("server cancel")
    G = P.Graph.from_csr(gpu_ctx, g)
    srv = P.Server(gpu_ctx, slots=1)
    try:
        t1 = srv.submit_select(G, 30, 0.05, 512, 3)
        t2 = srv.submit_select(G, 30, 0.05, 1024, 3)
        srv.cancel(t2)
        r1 = srv.poll(t1, wait_ms=60000)
        assert r1["status"] == 0 and len(r1["seeds"]) == 30
        with pytest.raises(P.InfuseError) as e:
            srv.poll(t2, wait_ms=60000)
        assert e.value.status == 7  # IM_ERR_CANCELLED (or finished before the cancel arrived)
        t3 = srv.submit_sigma(G, [], 0.05, 512, 3)
        r3 = srv.poll(t3, wait_ms=1000)
        assert r3["count"] == 0 and r3["status"] == 0
        with pytest.raises(P.InfuseError):
            srv.poll(123456789)
        srv.drain()
    finally:
        srv.close()
        G.free()


def test_server_budget_rejects_what_cannot_fit():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU device")
    announce("server budget")
    g = chung_lu(4000, 16000, 2.5, 31)
    # room for the graph and a R = 256 memo, not for a R = 8192 memo
    ctx = P.Context(device=0, hbm_budget=48 << 20)
    G = P.Graph.from_csr(ctx, g)
    srv = P.Server(ctx, slots=2)
    try:
        ok = srv.submit_sigma(G, [1, 2, 3], 0.05, 256, 7)
        big = srv.submit_select(G, 10, 0.05, 8192, 7)
        r_ok = srv.poll(ok, wait_ms=60000)
        assert r_ok["status"] == 0
        assert r_ok["count"] == oracle.sigma_count(g, oracle.Sampler("hash", p=0.05, R=256, seed=7), [1, 2, 3])
        r_big = srv.poll(big, wait_ms=60000)
        assert r_big["status"] == 5  # IM_ERR_BUDGET
        assert srv.stats()["rejected"] == 1
    finally:
        srv.close()
        G.free()
        ctx.close()
