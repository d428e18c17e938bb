"""The five workload configurations, as seeded synthetic stand-ins.

The paper evaluates on SNAP networks (Table 3) that are not available here;
these graphs reproduce their shapes (vertex/edge counts, power-law degrees):

  c1  tiny Chung-Lu n=2,000, gamma 2.5, m=8,000 (seed 1); p=0.05, R=256, K=10
  c2  Chung-Lu n=15,000, gamma 2.3, m=31,000 (NetHEP-sized, seed 2);
      p=0.01, R=2,048, K=50
  c3  64 Chung-Lu graphs, gamma 2.5, seeds 100..163, n log-uniform in
      [1,000, 40,000], m uniform integer in [2n, 10n]; per-edge trivalency
      p in {0.1, 0.01, 0.001}; R=1,024, K=20 each
  c4  R-MAT scale 18, edge factor 5, a/b/c/d = .57/.19/.19/.05 (Amazon-sized,
      seed 3); p=0.01, R=8,192, K=100
  c5  serving: four resident graphs (Chung-Lu 15k/31k, Chung-Lu 37k/175k,
      R-MAT 18 ef 5, R-MAT 20 ef 8) and a Poisson query trace (seed 4)

The hash seed s of a workload is its generator seed (c1: 1, c2: 2, c4: 3,
c3: the graph's own seed, c5: 4).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .graphs import Graph, chung_lu, rmat, splitmix64_stream, trivalency_p, uniform01


@dataclass
class Workload:
    name: str
    graphs: List[Graph]
    p: Optional[float]  # uniform p, or None when graphs carry per-slot p
    R: int
    K: int
    seeds: List[int]  # hash seed per graph
    notes: dict = field(default_factory=dict)


def _c3_graph(g_seed: int) -> Graph:
    # n log-uniform in [1000, 40000] and m uniform integer in [2n, 10n], drawn
    # from the first two outputs of the graph's own SplitMix64 stream.
    u = uniform01(g_seed, 0, 2)
    n = int(round(math.exp(math.log(1000.0) + u[0] * (math.log(40000.0) - math.log(1000.0)))))
    n = min(max(n, 1000), 40000)
    m = 2 * n + int(u[1] * (8 * n + 1))
    g = chung_lu(n, m, 2.5, g_seed, stream_offset=2, name=f"c3/g{g_seed}")
    g.p_slot = trivalency_p(g, g_seed)
    return g


def make_config(name: str) -> Workload:
    if name == "c1":
        g = chung_lu(2000, 8000, 2.5, 1, name="c1 chung_lu n=2000 m=8000")
        return Workload("c1", [g], 0.05, 256, 10, [1])
    if name == "c2":
        g = chung_lu(15000, 31000, 2.3, 2, name="c2 chung_lu n=15000 m=31000")
        return Workload("c2", [g], 0.01, 2048, 50, [2])
    if name == "c3":
        gs = [_c3_graph(s) for s in range(100, 164)]
        return Workload("c3", gs, None, 1024, 20, list(range(100, 164)))
    if name == "c4":
        g = rmat(18, 5, 0.57, 0.19, 0.19, 3, name="c4 rmat scale=18 ef=5")
        return Workload("c4", [g], 0.01, 8192, 100, [3])
    if name == "c5":
        gs = [
            chung_lu(15000, 31000, 2.3, 4, name="c5/chung_lu 15k/31k"),
            chung_lu(37151, 175000, 2.3, 4, stream_offset=1 << 40, name="c5/chung_lu 37k/175k"),
            rmat(18, 5, 0.57, 0.19, 0.19, 4, name="c5/rmat18 ef5"),
            rmat(20, 8, 0.57, 0.19, 0.19, 4 + (1 << 32), name="c5/rmat20 ef8"),
        ]
        return Workload("c5", gs, None, 0, 0, [4, 4, 4, 4])
    raise KeyError(name)


def config_graphs(name: str) -> List[Graph]:
    return make_config(name).graphs


CONFIGS = ("c1", "c2", "c3", "c4", "c5")


@dataclass
class Query:
    t_arrival: float  # seconds from trace start
    kind: str  # "sigma" or "select"
    graph: int
    p: float
    R: int
    K: int = 0
    S: Optional[np.ndarray] = None


def serving_trace(graph_sizes: List[int], n_queries: int = 2000, rate: float = 200.0,
                  seed: int = 4) -> List[Query]:
    """Poisson arrivals; 70% sigma(S) with |S| ~ U{1..50}, 30% K-selections.

    (p, R) for both kinds is drawn from {0.005, 0.01, 0.02, 0.05} x
    {256, 1024, 4096, 8192}; K from {10, 50, 100}; the graph uniformly.
    """
    ps = (0.005, 0.01, 0.02, 0.05)
    Rs = (256, 1024, 4096, 8192)
    Ks = (10, 50, 100)
    out: List[Query] = []
    t = 0.0
    pos = 0
    for _ in range(n_queries):
        u = uniform01(seed, pos, 7)
        pos += 7
        t += -math.log(1.0 - u[0]) / rate
        gi = min(int(u[1] * len(graph_sizes)), len(graph_sizes) - 1)
        p = ps[min(int(u[3] * 4), 3)]
        R = Rs[min(int(u[4] * 4), 3)]
        if u[2] < 0.7:
            k = 1 + min(int(u[5] * 50), 49)
            raw = splitmix64_stream(seed ^ 0x5EED, pos, 4 * k + 64)
            pos += 4 * k + 64
            picks = []
            seen = set()
            for x in raw:
                vtx = int(x % np.uint64(graph_sizes[gi]))
                if vtx not in seen:
                    seen.add(vtx)
                    picks.append(vtx)
                if len(picks) == k:
                    break
            out.append(Query(t, "sigma", gi, p, R, S=np.array(picks, dtype=np.uint32)))
        else:
            K = Ks[min(int(u[6] * 3), 2)]
            out.append(Query(t, "select", gi, p, R, K=K))
    return out
