"""Serving workload at its own scale against the oracle.

The four resident graphs of the serving configuration (Chung-Lu 15k/31k and
37k/175k, R-MAT scale 18 edge factor 5, R-MAT scale 20 edge factor 8) and the
first queries of its Poisson trace (seed 4) are replayed through the server
under a device-memory budget small enough that resident memos are evicted and
rebuilt while the trace runs.  Every query of the stored fixture (the first
query of each kind, graph and R in that prefix; selections on the R-MAT
scale-20 graph at R <= 1,024) must return the oracle's sigma count, or its
seeds, marginal counts and cover count, exactly: the memo gain equals RandCas
over the same samples (Algorithm 4, Section III-C).

The fixture is tests/golden/c5_oracle.json, written by
tests/golden/make_golden.py from the oracle and the generators only.
"""

import json
import os

import numpy as np
import pytest

import paper_2008_03095_amd as P
from tests.conftest import announce
from workloads import make_config, serving_trace

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "c5_oracle.json")

# Large enough for the biggest single query (R-MAT scale 20 at R = 8,192:
# a 34 GB memo and a 1 GB coverage bitmap), far too small for the trace's 64
# distinct (graph, p, R) memos: the server must evict to admit.
BUDGET = 48 << 30


@pytest.fixture(scope="module")
def c5():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU device")
    with open(GOLDEN) as f:
        gold = json.load(f)
    w = make_config("c5")
    trace = serving_trace([g.n for g in w.graphs], n_queries=gold["prefix"], rate=200.0, seed=4)
    return w, trace, gold


def test_c5_fixture_matches_trace(c5):
    """The stored queries are the trace's own (generator drift would make the
    comparison meaningless)."""
    w, trace, gold = c5
    assert [dict(n=g.n, m=g.m) for g in w.graphs] == gold["graphs"]
    for row in gold["queries"]:
        q = trace[row["index"]]
        assert (q.kind, q.graph, q.p, q.R) == (row["kind"], row["graph"], row["p"], row["R"])
        if q.kind == "sigma":
            assert [int(x) for x in q.S] == row["S"]
        else:
            assert q.K == row["K"]
    kinds = {(r["kind"], r["graph"], r["R"]) for r in gold["queries"]}
    for gi in range(4):
        for R in (256, 1024, 4096, 8192):
            assert ("sigma", gi, R) in kinds
    assert ("select", 3, 1024) in kinds and ("select", 2, 8192) in kinds


def test_c5_served_under_eviction_equals_oracle(c5):
    w, trace, gold = c5
    seed = gold["hash_seed"]
    announce(f"c5 trace prefix of {len(trace)} queries, budget {BUDGET >> 30} GiB")
    ctx = P.Context(device=0, hbm_budget=BUDGET)
    Gs = []
    try:
        Gs = [P.Graph.from_csr(ctx, g) for g in w.graphs]
        srv = P.Server(ctx, slots=4)
        try:
            tickets = []
            for q in trace:
                if q.kind == "sigma":
                    tickets.append(srv.submit_sigma(Gs[q.graph], q.S, q.p, q.R, seed))
                else:
                    tickets.append(srv.submit_select(Gs[q.graph], q.K, q.p, q.R, seed))
            results = [srv.poll(t, wait_ms=600000) for t in tickets]
            stats = srv.stats()
        finally:
            srv.close()
        assert all(r is not None and r["status"] == 0 for r in results), \
            [(i, r) for i, r in enumerate(results) if r is None or r["status"] != 0][:3]
        assert stats["completed"] == len(trace) and stats["rejected"] == 0
        assert stats["evictions"] > 0, stats  # memos were evicted and rebuilt
        assert stats["peak_concurrent"] > 1, stats
        for row in gold["queries"]:
            r = results[row["index"]]
            tag = (row["index"], row["kind"], row["graph"], row["p"], row["R"])
            if row["kind"] == "sigma":
                assert r["count"] == row["count"], (tag, r["count"], row["count"])
                assert r["sigma"] == pytest.approx(row["count"] / row["R"])
            else:
                assert [int(x) for x in r["seeds"]] == row["seeds"], tag
                assert [int(x) for x in r["marginal"]] == row["marginal"], tag
                assert r["count"] == row["cover"], tag
    finally:
        for G in Gs:
            G.free()
        ctx.close()
