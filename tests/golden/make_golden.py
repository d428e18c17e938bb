"""Writes the oracle's expected outputs for the workloads too large to
recompute inside a GPU test (c3: 64 graphs, c4: R-MAT scale 18 with 8,192
simulations, c5: spot queries of the serving trace on its four resident
graphs).  Calls only the oracle and the input generators.

    python tests/golden/make_golden.py [c3] [c4] [c5]

Outputs tests/golden/c3_oracle.json, c4_oracle.json and c5_oracle.json.
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from tests.helpers import combine_digests as combine  # noqa: E402
from tests.helpers import digest_weights  # noqa: E402
from tests.helpers import gains_checksum as g0_check  # noqa: E402
from workloads import make_config, serving_trace, splitmix64_stream  # noqa: E402

THREADS = os.cpu_count() or 8


def run_graph(g, p, R, seed, K, sigma_sets=()):
    s = oracle.Sampler("hash", p=p, R=R, seed=seed)
    dw = digest_weights(g.n)
    t = time.time()
    res = oracle.run_memo(g, s, K, digest_w=dw, threads=THREADS)
    out = dict(
        n=g.n, m=g.m, p=p, R=R, seed=seed, K=K,
        seeds=[int(x) for x in res["seeds"]],
        marginal=[int(x) for x in res["marginal"]],
        cover=int(res["cover"]),
        g0_sum=int(res["g0"].sum()),
        g0_check=g0_check(res["g0"]),
        label_check=combine(res["digests"]),
        oracle_seconds=round(time.time() - t, 2),
        oracle_threads=THREADS,
    )
    if sigma_sets:
        out["sigma"] = [dict(S=[int(x) for x in S], count=oracle.sigma_count(g, s, S, threads=THREADS))
                        for S in sigma_sets]
    return out, res


def make_c4():
    w = make_config("c4")
    g = w.graphs[0]
    rng_ids = [int(x % np.uint64(g.n)) for x in splitmix64_stream(44, 0, 256)]
    sigma_sets = [[0], [1, 2, 3, 4, 5], rng_ids[:20]]
    out, res = run_graph(g, w.p, w.R, w.seeds[0], w.K, sigma_sets)
    sample_ids = sorted(set(rng_ids + list(range(16))))
    out["g0_samples"] = {str(v): int(res["g0"][v]) for v in sample_ids}
    out["digest_every"] = 64
    out["digests"] = ["%016x" % int(x) for x in res["digests"][::64]]
    out["citation"] = ("oracle outputs for the R-MAT scale-18 workload (Amazon-sized stand-in, Table 3): "
                       "labels by BFS per sample (Algorithm 5's fixed point), CELF with the memo "
                       "formula of Section III-C; written by tests/golden/make_golden.py")
    with open(os.path.join(HERE, "c4_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


def make_c3():
    w = make_config("c3")
    graphs = []
    for g, seed in zip(w.graphs, w.seeds):
        o, _ = run_graph(g, 0.0, w.R, seed, w.K)
        graphs.append(o)
    out = dict(citation=("oracle outputs for the 64-graph batching workload (per-edge trivalency p); "
                         "written by tests/golden/make_golden.py"), graphs=graphs)
    with open(os.path.join(HERE, "c3_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


# Serving trace spot checks: the first C5_PREFIX queries of the trace are
# replayed by the GPU test; within them, the first query of every (kind,
# graph, R) class is checked against the values written here.  Selections on
# the R-MAT scale-20 graph are taken at R <= 1,024 only: the memo-formula CELF
# holds labels and sizes of every sample in host memory (8 bytes per vertex
# and sample).
C5_PREFIX = 300
C5_SELECT_MAX_R = {3: 1024}


def c5_golden_queries(trace, prefix=C5_PREFIX):
    """Indices (into the trace) of the queries the c5 fixture covers."""
    seen = set()
    out = []
    for i, q in enumerate(trace[:prefix]):
        if q.kind == "select" and q.R > C5_SELECT_MAX_R.get(q.graph, 1 << 30):
            continue
        key = (q.kind, q.graph, q.R)
        if key not in seen:
            seen.add(key)
            out.append(i)
    return out


def make_c5():
    w = make_config("c5")
    trace = serving_trace([g.n for g in w.graphs], n_queries=2000, rate=200.0, seed=4)
    seed = w.seeds[0]
    rows = []
    for i in c5_golden_queries(trace):
        q = trace[i]
        g = w.graphs[q.graph]
        s = oracle.Sampler("hash", p=q.p, R=q.R, seed=seed)
        t = time.time()
        row = dict(index=i, kind=q.kind, graph=q.graph, p=q.p, R=q.R)
        if q.kind == "sigma":
            row["S"] = [int(x) for x in q.S]
            row["count"] = oracle.sigma_count(g, s, q.S, threads=THREADS)
        else:
            res = oracle.run_memo(g, s, q.K, threads=THREADS)
            row.update(K=q.K, seeds=[int(x) for x in res["seeds"]],
                       marginal=[int(x) for x in res["marginal"]], cover=int(res["cover"]))
        row["oracle_seconds"] = round(time.time() - t, 2)
        rows.append(row)
        print(f"  c5 query {i}: {q.kind} graph {q.graph} p {q.p} R {q.R}: {row['oracle_seconds']} s", flush=True)
    out = dict(citation=("oracle outputs for spot queries of the serving trace (Poisson 200 queries/s, seed 4) "
                         "on its four resident graphs: sigma counts by multi-source BFS on the hashed samples "
                         "(RandCas, Algorithm 4), selections by CELF with the memo formula of Section III-C; "
                         "written by tests/golden/make_golden.py"),
               prefix=C5_PREFIX, hash_seed=seed, oracle_threads=THREADS,
               graphs=[dict(n=g.n, m=g.m) for g in w.graphs], queries=rows)
    with open(os.path.join(HERE, "c5_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c3", "c4", "c5"]
    for name in which:
        t = time.time()
        {"c3": make_c3, "c4": make_c4, "c5": make_c5}[name]()
        print(f"{name}: {time.time() - t:.1f}s", flush=True)
