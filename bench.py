#!/usr/bin/env python3
"""Benchmark of the whole hot path on one MI355X.

A step = one cold pass over the large single-graph workload (R-MAT scale 18,
edge factor 5, a/b/c/d = .57/.19/.19/.05, seed 3; p = 0.01, R = 8,192,
K = 100, hash seed 3): hash sampler set-up, fused multi-simulation connected
components, component-size memo and initial gains, 100 CELF steps on the
device, and sigma(S) of the selected seeds.  The graph is resident in HBM
before the timed region; the memo is dropped before every step.

Prints one JSON line.  value = m*R per second of whole steps (edge-samples/s).

    python bench.py [--steps K] [--warmup W] [--workload c4|c2|c1]
    python bench.py --calibrate-copy     # plain copy kernel for counter scaling
"""

from __future__ import annotations

import argparse
import hashlib
import json
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edge-samples/s (m·R/s), K-seed time; serving p50/p99 vs plain per-query launch"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "celf_persistent_c4_traffic.txt")
ROOF_SOURCES = [os.path.join(ROOT, "paper_2008_03095_amd", "csrc", f) for f in ("celf_persistent.hip", "common.h")]
# the labelling kernels of the memo construction (components phase)
CC_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cc_kernels_c4_traffic.txt")
CC_SOURCES = [os.path.join(ROOT, "paper_2008_03095_amd", "csrc", f) for f in ("cc.hip", "lists.h", "tile.h", "common.h")]
CC_KERNELS = ("hook", "hook_hubs", "lists", "link", "link_hubs", "flatten", "count")
# the memo-free search (directed workload): level kernel and its sources
BFS_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "bfs_level_d1_traffic.txt")
BFS_SOURCES = [os.path.join(ROOT, "paper_2008_03095_amd", "csrc", f)
               for f in ("direct.hip", "direct.h", "tile.h", "common.h")]

WORKLOADS = {
    "c4": "R-MAT scale 18, edge factor 5, a/b/c/d=.57/.19/.19/.05, seed 3; p=0.01, R=8192, K=100",
    "c2": "Chung-Lu n=15000, gamma 2.3, m=31000, seed 2; p=0.01, R=2048, K=50",
    "c1": "Chung-Lu n=2000, gamma 2.5, m=8000, seed 1; p=0.05, R=256, K=10",
}


def code_tokens(text: str) -> str:
    """The source text without comments and with whitespace runs folded, so
    that an edit of a comment does not count as a change of the kernel."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def roof_source_hash(sources=None) -> str:
    h = hashlib.sha256()
    for p in sources or ROOF_SOURCES:
        with open(p, encoding="utf-8") as f:
            h.update(code_tokens(f.read()).encode())
    return h.hexdigest()[:16]


def read_traffic(path=None, sources=None):
    """HBM bytes of the roofline kernel from a committed counter summary, or
    None when its sources changed since the counters were taken."""
    try:
        with open(path or TRAFFIC_FILE) as f:
            for line in f:
                if line.startswith("TRAFFIC_JSON "):
                    rec = json.loads(line[len("TRAFFIC_JSON "):])
                    if rec.get("source_hash") == roof_source_hash(sources):
                        return rec
    except OSError:
        pass
    return None


def bfs_algorithmic_bytes(stats: dict, per_arc_p: bool) -> int:
    """Bytes the memo-free search moves by its definition, from its work
    counts: per frontier item (vertex, 256-column tile) its four frontier
    words read and cleared and its row bounds (72 B); per arc scanned the
    target id and hash (8 B) and, with per-arc probabilities, the threshold
    (4 B); per (arc, item) pair live in a frontier column the target's four
    visited words read and or-ed and its four frontier words or-ed (96 B).
    The 1 KiB of sample values of a tile is shared by every item and left
    out."""
    return 72 * stats["items"] + (12 if per_arc_p else 8) * stats["arcs"] + 96 * stats["live_pairs"]


def celf_algorithmic_bytes(evals: int, K: int, mwords: int, listed_tiles: int, gathers: int) -> int:
    """Bytes the memo-formula gain moves by its definition on the sparse memo,
    from the CELF kernel's work counts: per evaluation (and per commit) the
    candidate's tile-mask words (4 B each); per listed (candidate, tile)
    pair its row of 256 labels (1 KiB); per column of a non-singleton
    component the component's size (4 B) and its coverage word (4 B).  A
    tile without its mask bit holds singletons only, counted in closed form
    (no bytes)."""
    return 4 * mwords * (evals + K) + 1024 * listed_tiles + 8 * gathers


def cc_algorithmic_bytes(work: dict, n: int, mwords: int, light_slots: int, hub_slots: int, listed: int,
                         link_tiles: int) -> dict:
    """Bytes each labelling kernel moves by its definition, from the work
    counts of one construction (Graph.memo_work) and the sizes of the lists:
      hook (light rows) : its rows' slots (neighbour + hash, 8 B) once, 1 KiB
                          per tile row written, the mask words of every vertex
      hook_hubs         : the hubs' slots once (8 B), 1 KiB per tile row written
      lists             : mask words read, one 4 B entry per listed and per
                          union tile, the initial gains set (8 B per vertex)
      link + link_hubs  : 1 KiB of hook parents per union tile, and per union
                          attempt the two entries read and one written (12 B)
      flatten           : 1 KiB read per listed tile, 4 B per entry rewritten
      count             : 1 KiB read per listed tile, 8 B per size decrement
                          made in device memory (read and write)
      gain0             : 1 KiB read per listed tile, 4 B per size gathered,
                          8 B per vertex (the gain)"""
    masks = 8 * mwords * n
    link = 1024 * link_tiles + 12 * work["union_attempts"]
    return {
        "hook": 8 * light_slots + 1024 * work["row_tiles"] + masks,
        "hook_hubs": 8 * hub_slots + 1024 * work["hub_tiles"],
        "lists": masks + 4 * (listed + link_tiles) + 8 * n,
        "link+link_hubs": link,
        "flatten": 1024 * listed + 4 * work["flatten_rewrites"],
        "count": 1024 * listed + 8 * work["count_atomics"],
        "gain0": 1024 * listed + 4 * work["gain_gathers"] + 8 * n,
    }


def cpu_baseline(workload, samples: int):
    """The oracle as it stands (labelling of every sample + memo-formula CELF)
    on the first `samples` simulations of the same graph and K."""
    import oracle

    g = workload.graphs[0]
    threads = len(os.sched_getaffinity(0))
    s = oracle.Sampler("hash", p=workload.p, R=samples, seed=workload.seeds[0])
    t = time.perf_counter()
    oracle.run_memo(g, s, workload.K, threads=threads)
    dt = time.perf_counter() - t
    return {
        "value": g.m * samples / dt,
        "unit": "edge-samples/s",
        "cores": threads,
        "kind": "oracle",
        "seconds": round(dt, 3),
        "sample": (f"same graph and K={workload.K}, first {samples} of {workload.R} simulations: "
                   f"BFS labelling of every sample + CELF on stored labels (m*{samples} "
                   f"edge-samples in {dt:.2f} s)"),
    }


def _pct(xs, q):
    import numpy as np

    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def serve_bench(args):
    """Serving workload: four resident graphs and a Poisson trace of sigma(S)
    and K-selection queries at 200 queries/s (seed 4), replayed in real time
    against the server, then run one query at a time from scratch (memo built
    for every query, no overlap) as the plain per-query baseline."""
    import numpy as np
    import torch

    import paper_2008_03095_amd as P
    from workloads import make_config, serving_trace

    w = make_config("c5")
    ctx = P.Context(device=0, hbm_budget=int(args.hbm_budget_gib * (1 << 30)))
    Gs = [P.Graph.from_csr(ctx, g) for g in w.graphs]
    trace = serving_trace([g.n for g in w.graphs], n_queries=args.queries, rate=200.0, seed=4)
    seed = w.seeds[0]

    def submit(srv, q):
        if q.kind == "sigma":
            return srv.submit_sigma(Gs[q.graph], q.S, q.p, q.R, seed)
        return srv.submit_select(Gs[q.graph], q.K, q.p, q.R, seed)

    # warm-up: one query of each kind (device code loading, allocator pools)
    def server():
        return P.Server(ctx, slots=args.slots, persistent_min_mwords=args.persistent_min_mwords)

    srv = server()
    for q in trace[:2]:
        srv.poll(submit(srv, q), wait_ms=600000)
    srv.close()
    for G in Gs:
        G.drop_memo()

    # served: real-time arrivals, continuous admission, memo reuse, overlap
    srv = server()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = []
    for q in trace:
        wait = q.t_arrival - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        tickets.append(submit(srv, q))
    served = [srv.poll(t, wait_ms=600000) for t in tickets]
    t_served = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    bad = [r for r in served if r is None or r["status"] != 0]
    if bad:
        raise RuntimeError(f"{len(bad)} served queries failed: {bad[:3]}")

    # saturated: the whole trace submitted at once, memos dropped first, so
    # the makespan measures the server's capacity rather than the arrival rate
    for G in Gs:
        G.drop_memo()
    srv = server()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = [submit(srv, q) for q in trace]
    burst = [srv.poll(t, wait_ms=600000) for t in tickets]
    t_burst = time.perf_counter() - t0
    burst_stats = srv.stats()
    srv.close()
    if any(r is None or r["status"] != 0 for r in burst):
        raise RuntimeError("saturated run: some queries failed")
    # results must not depend on the mix
    for r1, r2 in zip(served, burst):
        if r1["count"] != r2["count"]:
            raise RuntimeError("a query returned different results in the two serving runs")

    # plain per-query baseline: each query alone, its memo built from scratch
    service = []
    for q in trace:
        for G in Gs:
            G.drop_memo()
        G = Gs[q.graph]
        torch.cuda.synchronize()
        t = time.perf_counter()
        G.set_params(q.p, q.R, seed)
        if q.kind == "sigma":
            cnt, _ = G.estimate_sigma(q.S)
        else:
            G.select_seeds(q.K)
        service.append(time.perf_counter() - t)
    # the same arrivals queued in front of one-at-a-time execution
    plain_lat, clock = [], 0.0
    for q, sv in zip(trace, service):
        start = max(clock, q.t_arrival)
        clock = start + sv
        plain_lat.append((clock - q.t_arrival) * 1e3)
    t_plain = clock - trace[0].t_arrival
    for G in Gs:
        G.free()
    ctx.close()

    lat = [r["latency_ms"] for r in served]
    by_kind = {}
    for q, r in zip(trace, served):
        by_kind.setdefault(q.kind, []).append(r["latency_ms"])
    plain_kind = {}
    for q, l in zip(trace, plain_lat):
        plain_kind.setdefault(q.kind, []).append(l)
    rec = {
        "metric": "serving p50/p99 latency and throughput vs plain per-query launch",
        "value": len(trace) / t_served,
        "unit": "queries/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "c5: Chung-Lu 15k/31k, Chung-Lu 37k/175k, R-MAT 18 ef 5, R-MAT 20 ef 8; "
                               "Poisson 200 queries/s, seed 4, 70% sigma(S) |S| in 1..50, 30% selections; "
                               "p in {.005,.01,.02,.05}, R in {256,1024,4096,8192}, K in {10,50,100}",
                   "queries": len(trace), "slots": args.slots, "hbm_budget_gib": args.hbm_budget_gib,
                   "persistent_min_mwords": args.persistent_min_mwords},
        "served": {"throughput_qps": len(trace) / t_served, "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99),
                   "by_kind": {k: {"n": len(v), "p50_ms": _pct(v, 50), "p99_ms": _pct(v, 99)}
                               for k, v in by_kind.items()},
                   "stats": stats},
        "plain_per_query": {"throughput_qps": len(trace) / t_plain, "p50_ms": _pct(plain_lat, 50),
                            "p99_ms": _pct(plain_lat, 99),
                            "service_ms_mean": 1e3 * float(np.mean(service)),
                            "by_kind": {k: {"n": len(v), "p50_ms": _pct(v, 50), "p99_ms": _pct(v, 99)}
                                        for k, v in plain_kind.items()}},
    }
    rec["served_saturated"] = {"throughput_qps": len(trace) / t_burst, "makespan_s": t_burst,
                               "stats": burst_stats}
    rec["throughput_vs_plain"] = rec["served"]["throughput_qps"] / rec["plain_per_query"]["throughput_qps"]
    rec["capacity_vs_plain"] = rec["served_saturated"]["throughput_qps"] / rec["plain_per_query"]["throughput_qps"]
    print(json.dumps(rec), flush=True)


def directed_bench(args):
    """Directed graphs (a widening of the paper's undirected method): the
    spread of a seed set on a directed R-MAT (scale 18, edge factor 5, arcs
    not symmetrised, seed 3) under the weighted cascade (p(u -> v) =
    1 / in-degree(v)), R = 8,192, S = the 100 vertices of largest out-degree.
    One step = the memo-free search (sampler set-up, level-synchronous
    reachability over all samples, count); value = arcs * R / step time."""
    import numpy as np
    import torch

    import oracle
    import paper_2008_03095_amd as P
    from workloads import rmat_directed, wc_p

    g = rmat_directed(18, 5, 0.57, 0.19, 0.19, 3)
    g.p_slot = wc_p(g)
    R, seed = 8192, 3
    deg = np.diff(g.row_ptr.astype(np.int64))
    S = [int(v) for v in np.argsort(-deg, kind="stable")[:100]]
    ctx = P.Context(device=0)
    G = P.Graph.from_csr(ctx, g)
    G.set_params(0.0, R, seed)
    for _ in range(args.warmup):
        cnt, _, levels = G.estimate_sigma_direct(S)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cnt, _, levels = G.estimate_sigma_direct(S)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt * 1e3 / args.steps
    # one more call, untimed, with the kernel clock and the search's work
    # counts on (both perturb the kernels a little: the level times of this
    # call are the roofline's)
    ctx.set_profiling(2)
    ctx.reset_kernel_stats()
    G.estimate_sigma_direct(S)
    torch.cuda.synchronize()
    ctx.set_profiling(False)
    names = ["edge_hash", "x_sort", "sigma_direct", "bfs_level"]
    stats = {k: ctx.kernel_stats(k) for k in names}
    work = G.search_stats()
    lv_n, level_ms = stats["bfs_level"]
    alg = bfs_algorithmic_bytes(work, True)
    achieved = alg / (level_ms * 1e-3) / 1e9 if level_ms > 0 else None
    traffic = read_traffic(BFS_TRAFFIC_FILE, BFS_SOURCES)
    rec = {
        "metric": "arc-samples/s (arcs·R / spread time), directed spread under the weighted cascade",
        "value": g.nnz * R / (ms * 1e-3),
        "unit": "arc-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64 bitsets",
        "data": "synthetic",
        "config": {"workload": "d1: directed R-MAT scale 18, edge factor 5, seed 3, weighted cascade; R=8192, "
                               "|S|=100 (largest out-degree)", "n": g.n, "arcs": g.nnz, "R": R},
        "count": cnt,
        "levels": levels,
        "kernel_ms_profiled_call": {k: v[1] for k, v in stats.items()},
        "search_work": work,
        # roofline of the level kernel over one step: the step's algorithmic
        # bytes over the summed duration of its level launches
        "roofline": {
            "bound": "hbm",
            "kernel": "k_bfs_level",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": traffic["bytes_per_step"] if traffic else None,
            "algorithmic_bytes": alg,
            "launches_per_step": lv_n,
            "level_ms_per_step": level_ms,
        },
    }
    G.free()
    if args.no_selection:
        ctx.close()
        print(json.dumps(rec), flush=True)
        return
    # greedy selection on a smaller digraph (memo-free, candidates searched
    # side by side): directed R-MAT scale 14, weighted cascade, R = 1,024, K = 50
    gs = rmat_directed(14, 5, 0.57, 0.19, 0.19, 4)
    gs.p_slot = wc_p(gs)
    Gs = P.Graph.from_csr(ctx, gs)
    Gs.set_params(0.0, 1024, 4)
    Gs.select_seeds_direct(50)  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    sel_seeds, _, sel_cover = Gs.select_seeds_direct(50)
    torch.cuda.synchronize()
    sel_ms = (time.perf_counter() - t) * 1e3
    rec["selection"] = {"graph": "directed R-MAT scale 14, edge factor 5, seed 4, weighted cascade",
                        "n": gs.n, "arcs": gs.nnz, "R": 1024, "K": 50, "ms": sel_ms, "cover": sel_cover,
                        "evaluations": int(Gs._lib.im_last_celf_evals(Gs.handle))}
    Gs.free()
    ctx.close()
    if not args.no_cpu_baseline:
        t = time.perf_counter()
        ref = oracle.celf_arcs(gs, oracle.Sampler("hash", R=1024, seed=4), 50)
        rec["selection"]["oracle_s"] = time.perf_counter() - t
        rec["selection"]["oracle_equal"] = list(ref["seeds"]) == [int(x) for x in sel_seeds]
        # the oracle on the first samples of the same spread
        samples = min(args.cpu_samples, R)
        threads = len(os.sched_getaffinity(0))
        t = time.perf_counter()
        oracle.sigma_count(g, oracle.Sampler("hash", R=samples, seed=seed), S, threads=threads)
        dt_c = time.perf_counter() - t
        rec["cpu_baseline"] = {"value": g.nnz * samples / dt_c, "unit": "arc-samples/s", "cores": threads,
                               "kind": "oracle", "sample": f"same graph and S, first {samples} of {R} samples "
                               f"({dt_c:.2f} s)"}
    print(json.dumps(rec), flush=True)


def batch_bench(args):
    """Batching workload: 64 Chung-Lu graphs (seeds 100..163, n log-uniform in
    [1,000, 40,000], m uniform in [2n, 10n], per-edge trivalency p), R = 1,024,
    K = 20 each: one im_batch_select call for all graphs against 64 plain
    per-graph selections, every memo built from scratch in both."""
    import numpy as np
    import torch

    import paper_2008_03095_amd as P
    from workloads import make_config

    w = make_config("c3")
    ctx = P.Context(device=0)
    Gs = [P.Graph.from_csr(ctx, g) for g in w.graphs]
    for G, s in zip(Gs, w.seeds):
        G.set_params(0.0, w.R, s)  # p ignored: per-slot probabilities
    Ks = [w.K] * len(Gs)
    es = sum(g.m for g in w.graphs) * w.R

    def drop():
        for G in Gs:
            G.drop_memo()

    def plain():
        out = []
        for G in Gs:
            out.append(G.select_seeds(w.K))
        return out

    def batched():
        return P.batch_select(ctx, Gs, Ks)

    for _ in range(args.warmup):
        drop(); plain(); drop(); batched()
    tp, tb = [], []
    for _ in range(args.steps):
        drop()
        torch.cuda.synchronize()
        t = time.perf_counter()
        rp = plain()
        tp.append(time.perf_counter() - t)
        drop()
        torch.cuda.synchronize()
        t = time.perf_counter()
        rb = batched()
        tb.append(time.perf_counter() - t)
        for a, b in zip(rp, rb):
            if list(a[0]) != list(b[0]) or a[2] != b[2]:
                raise RuntimeError("batched and plain selections differ")
    for G in Gs:
        G.free()
    ctx.close()
    t_plain, t_batch = float(np.median(tp)), float(np.median(tb))
    rec = {
        "metric": "batched vs plain per-graph K-seed selection (64 graphs)",
        "value": es / t_batch,
        "unit": "edge-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_batch * 1e3,
        "higher_is_better": True,
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "c3: 64 Chung-Lu graphs, gamma 2.5, seeds 100..163, n log-uniform in "
                               "[1000, 40000], m uniform in [2n, 10n], per-edge trivalency p "
                               "{0.1, 0.01, 0.001}; R=1024, K=20 each",
                   "graphs": len(w.graphs), "sum_m": sum(g.m for g in w.graphs), "R": w.R, "K": w.K},
        "batched_ms": t_batch * 1e3,
        "plain_ms": t_plain * 1e3,
        "speedup_vs_plain": t_plain / t_batch,
    }
    print(json.dumps(rec), flush=True)


def calibrate_copy(gib: int = 4, reps: int = 5):
    import torch

    n = gib << 28  # int32 elements
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read": n * 4, "bytes_written": n * 4,
                      "reps": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS) + ["c3", "c5", "d1"])
    ap.add_argument("--queries", type=int, default=2000, help="serving workload: queries of the trace")
    ap.add_argument("--persistent-min-mwords", type=int, default=0,
                    help="serving workload: memo size (2^20 words) below which selections run the per-step "
                         "kernels beside the other slots (0: every selection persistent)")
    ap.add_argument("--slots", type=int, default=4, help="serving workload: concurrent query slots")
    ap.add_argument("--hbm-budget-gib", type=float, default=224.0, help="serving workload: memo budget")
    ap.add_argument("--cpu-samples", type=int, default=8192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--no-selection", action="store_true", help="d1: the spread only")
    ap.add_argument("--weights", default="const", choices=["const", "uniform", "normal"],
                    help="edge probabilities: the workload's constant p, or per edge U[0,0.1] or "
                         "N(0.05,0.025) clipped (the paper's other weight settings)")
    ap.add_argument("--cc-chunk", type=int, default=0, help="columns per wavefront in labelling")
    ap.add_argument("--list-blocks", type=int, default=0, help="workgroups of the list-walking kernels")
    ap.add_argument("--celf-width", type=int, default=0, help="CELF candidates per round (per-step mode)")
    ap.add_argument("--celf-mode", type=int, default=0, help="1 persistent kernel, 2 per-step kernels")
    ap.add_argument("--celf-round0", type=int, default=None,
                    help="persistent CELF: candidates of a step's first round (0 = automatic)")
    ap.add_argument("--profile-celf", action="store_true",
                    help="also time every CELF launch (perturbs the step time)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: the multi-GPU path (R-sharding with one all-reduce of "
              "int64 gains) is designed, not implemented; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.workload == "c5":
        serve_bench(args)
        return
    if args.workload == "c3":
        batch_bench(args)
        return
    if args.workload == "d1":
        directed_bench(args)
        return

    import numpy as np
    import torch

    import paper_2008_03095_amd as P
    from workloads import make_config

    w = make_config(args.workload)
    g = w.graphs[0]
    p, R, K, seed = w.p, w.R, w.K, w.seeds[0]
    if args.weights != "const":
        from workloads import normal_p, uniform_p

        g.p_slot = uniform_p(g, seed) if args.weights == "uniform" else normal_p(g, seed)

    ctx = P.Context(device=0)
    ctx.set_tuning(cc_chunk=args.cc_chunk, celf_width=args.celf_width, celf_mode=args.celf_mode,
                   list_blocks=args.list_blocks,
                   celf_round0=args.celf_round0)
    G = P.Graph.from_csr(ctx, g)
    G.set_params(p, R, seed)

    def step():
        # cold memo: the selection builds it (no wait between construction
        # and selection)
        G.drop_memo()
        seeds, marg, cover = G.select_seeds(K)
        cnt, _ = G.estimate_sigma(seeds)
        if cnt != cover:
            raise RuntimeError("sigma of the selected seeds differs from the cover count")
        return seeds, cover

    for _ in range(args.warmup):
        step()
    # the timed steps record events around the persistent CELF launch only
    # (level 1), the roofline kernel; events around every kernel (level 2)
    # would add a few microseconds to each of a step's launches
    ctx.set_profiling(3 if args.profile_celf else 1)
    ctx.reset_kernel_stats()
    phases = np.zeros(4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        seeds, cover = step()
        phases += np.array(G.phase_ms())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.set_profiling(False)

    ms_per_step = dt * 1e3 / args.steps
    value = g.m * R * args.steps / dt
    roof_n, roof_ms = ctx.kernel_stats("celf")
    roof_avg = roof_ms / roof_n if roof_n else None
    phases /= args.steps
    t_cc = phases[1]
    names = ["edge_hash", "x_sort", "hook", "hook_hubs", "lists", "link", "link_hubs", "flatten", "count",
             "gain0",
             "sigma", "celf",
             "celf_topw", "celf_eval", "celf_bulk"]
    if args.profile_celf:
        names += ["celf.barrier", "celf.eval", "celf.commit", "celf.restale", "celf.prep", "celf.post",
                  "celf.rebuild", "celf.bulk", "celf.sort", "celf.move", "celf.lookahead_commits"]
    prof_steps = args.steps
    if not args.profile_celf:
        # every kernel's time from one more step, untimed, with events around
        # each launch (level 2)
        ctx.set_profiling(2)
        ctx.reset_kernel_stats()
        step()
        torch.cuda.synchronize()
        ctx.set_profiling(False)
        prof_steps = 1
    stats = {k: ctx.kernel_stats(k) for k in names}
    evals = G.celf_evals()
    memo_stats = G.memo_stats()

    # one more step, untimed, with every work count on (level 4: the
    # labelling kernels' counts and the CELF kernel's listed tiles and
    # gathers; they cost atomics, so the timed steps run without them)
    ctx.set_profiling(4)
    ctx.reset_kernel_stats()
    step()
    torch.cuda.synchronize()
    work = G.memo_work()
    celf_tiles = ctx.kernel_stats("celf.listed_tiles")[0]
    celf_gathers = ctx.kernel_stats("celf.gathers")[0]
    ctx.set_profiling(False)

    mwords = (((R + 255) // 256) + 31) // 32
    deg = np.diff(g.row_ptr.astype(np.int64))
    light_slots = int(deg[deg <= 64].sum())
    hub_slots = int(deg[deg > 64].sum())
    cc_alg = cc_algorithmic_bytes(work, g.n, mwords, light_slots, hub_slots, memo_stats["listed_tiles"],
                                  memo_stats["link_tiles"])
    cc_phase_alg = sum(v for k, v in cc_alg.items() if k != "gain0")
    cc_traffic = read_traffic(CC_TRAFFIC_FILE, CC_SOURCES)
    if cc_traffic and (cc_traffic.get("workload") != args.workload or args.weights != "const"):
        cc_traffic = None

    # roofline kernel: the persistent CELF kernel (one launch per step, the
    # largest single kernel of the step), at the sparse memo's own bytes
    alg_bytes = celf_algorithmic_bytes(evals, K, mwords, celf_tiles, celf_gathers)
    dense_bytes = (8 * R + R // 8) * (evals + K)
    achieved = alg_bytes / (roof_avg * 1e-3) / 1e9 if roof_avg else None
    traffic = read_traffic()
    if traffic and (traffic.get("workload") != args.workload or args.weights != "const"):
        traffic = None  # the counters were taken on another workload
    # components phase (hook ... count): the labelling kernels' algorithmic
    # bytes over the phase's device time; beside it a dense-memo
    # floor (every label written once, both endpoint labels of every live
    # edge-sample read) over the same time, as a model
    cc_ach = cc_phase_alg / (t_cc * 1e-3) / 1e9 if t_cc > 0 else None
    dense_floor = 4 * g.n * R + 8 * work["live_pairs"]
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "edge-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "n": g.n, "m": g.m,
                   "R": R, "K": K, "p": p if args.weights == "const" else args.weights,
                   "hash_seed": seed, "tuning": ctx.tuning()},
        "k_seed_ms": ms_per_step,
        "phase_ms": {"sampler_prep": phases[0], "components": phases[1], "gains0": phases[2],
                     "celf": phases[3]},
        "edge_samples_per_s_components": g.m * R / (t_cc * 1e-3) if t_cc > 0 else None,
        "celf_evals": evals,
        "cover_count": cover,
        "kernel_avg_ms": {k: (v[1] / v[0] if v[0] else None) for k, v in stats.items()},
        "kernel_launches_per_step": {k: v[0] / prof_steps for k, v in stats.items()},
        "kernel_total_ms_per_step": {k: v[1] / prof_steps for k, v in stats.items()},
        "roofline": {
            "bound": "hbm",
            "kernel": "k_celf_persistent",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": traffic["bytes_per_launch"] if traffic else None,
            "algorithmic_bytes": alg_bytes,
            "work": {"evaluations": evals, "commits": K, "listed_tiles": celf_tiles, "gathers": celf_gathers},
            "avg_launch_ms": roof_avg,
            "dense_model_bytes": dense_bytes,
        },
        "roofline_components": {
            "bound": "hbm",
            "kernels": list(CC_KERNELS),
            "achieved": cc_ach,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": cc_ach / HBM_PEAK_GBS if cc_ach else None,
            "algorithmic_bytes": cc_phase_alg,
            "phase_ms": t_cc,
            "traffic": cc_traffic["bytes_components"] if cc_traffic else None,
            "traffic_frac": (cc_traffic["bytes_components"] / (t_cc * 1e-3) / 1e9 / HBM_PEAK_GBS
                             if cc_traffic and t_cc > 0 else None),
            "dense_floor_bytes": dense_floor,
            "dense_floor_frac": dense_floor / (t_cc * 1e-3) / 1e9 / HBM_PEAK_GBS if t_cc > 0 else None,
            "per_kernel_algorithmic_bytes": cc_alg,
            "per_kernel_traffic": cc_traffic["per_kernel_bytes"] if cc_traffic else None,
            "work": work,
        },
        "cpu_baseline": None,
    }
    rec["memo_stats"] = memo_stats
    # sigma of the selected seeds without a memo (search over all samples),
    # outside the timed steps
    t_direct = []
    for _ in range(2):
        torch.cuda.synchronize()
        t = time.perf_counter()
        cnt_d, _, levels = G.estimate_sigma_direct(seeds)
        t_direct.append(time.perf_counter() - t)
        if cnt_d != cover:
            raise RuntimeError("memo-free sigma differs from the cover count")
    rec["sigma_without_memo"] = {"ms": 1e3 * min(t_direct), "levels": levels, "count": cnt_d}
    G.free()
    ctx.close()
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w, min(args.cpu_samples, R))
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
