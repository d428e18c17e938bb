"""Deterministic undirected graph generators (numpy, no method arithmetic).

Every generator draws from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): output k of a stream seeded
with s is mix(s + (k+1)*0x9E3779B97F4A7C15), where mix is the published
two-multiply xor-shift finaliser.  Uniform doubles take the top 53 bits.

Graphs are returned as a symmetric CSR (both orientations stored, rows sorted,
no duplicates, no self-loops), which is the input format of Section III-D of
the paper (xadj/adj).  Vertex ids are uint32, row offsets uint64.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def splitmix64_stream(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs start..start+count-1 of the SplitMix64 stream seeded with `seed`."""
    k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GAMMA
        return _mix64(z)


def uniform01(seed: int, start: int, count: int) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of SplitMix64 outputs."""
    return (splitmix64_stream(seed, start, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


@dataclass
class Graph:
    """Graph in CSR form: symmetric (undirected, both orientations of every
    edge) or, with directed=True, the out-arcs of every vertex."""

    n: int
    row_ptr: np.ndarray  # uint64 [n+1]
    col: np.ndarray  # uint32 [2m] (undirected) or [m] (directed)
    p_slot: Optional[np.ndarray] = None  # float64 per slot or None (uniform p)
    name: str = ""
    meta: dict = field(default_factory=dict)
    directed: bool = False

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        """Edges (undirected) or arcs (directed)."""
        return self.nnz if self.directed else self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def undirected_edges(self) -> np.ndarray:
        """(u, v) pairs with u < v, in CSR order of the smaller endpoint."""
        rows = np.repeat(np.arange(self.n, dtype=np.uint32), self.degrees())
        keep = rows < self.col
        return np.stack([rows[keep], self.col[keep]], axis=1)


def from_edge_list(n: int, u: np.ndarray, v: np.ndarray, name: str = "",
                   p_und: Optional[np.ndarray] = None) -> Graph:
    """Symmetric, sorted, deduplicated, loop-free CSR from undirected pairs.

    If `p_und` is given it holds one probability per input pair (after the
    first occurrence of each unordered pair wins) and is written to both
    orientations of the edge.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    keep = lo != hi
    lo, hi = lo[keep], hi[keep]
    pk = None if p_und is None else np.asarray(p_und, dtype=np.float64)[keep]
    key = lo * n + hi
    _, first = np.unique(key, return_index=True)
    first.sort()
    lo, hi = lo[first], hi[first]
    if pk is not None:
        pk = pk[first]
    src = np.concatenate([lo, hi])
    dst = np.concatenate([hi, lo])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    row_ptr = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(np.bincount(src, minlength=n), out=row_ptr[1:])
    p_slot = None
    if pk is not None:
        p_slot = np.concatenate([pk, pk])[order]
    return Graph(n=n, row_ptr=row_ptr, col=dst.astype(np.uint32), p_slot=p_slot, name=name)


def from_arc_list(n: int, u: np.ndarray, v: np.ndarray, name: str = "") -> Graph:
    """Directed CSR (out-arcs, rows sorted) from arcs u -> v; duplicate arcs
    and self-loops are dropped."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    key = np.unique(u * n + v)
    src, dst = key // n, key % n
    row_ptr = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(np.bincount(src, minlength=n), out=row_ptr[1:])
    return Graph(n=n, row_ptr=row_ptr, col=dst.astype(np.uint32), name=name, directed=True)


def chung_lu(n: int, m: int, gamma: float, seed: int, stream_offset: int = 0,
             name: str = "") -> Graph:
    """Chung-Lu power-law graph with exactly `m` unique undirected edges.

    Vertex i gets weight w_i proportional to (i+1)^(-1/(gamma-1)), so the
    expected degree sequence follows a power law with exponent `gamma`.
    Endpoint pairs are drawn independently proportional to w (inverse-CDF
    on uniform doubles); self-loops and repeated pairs are dropped, in draw
    order, until exactly m distinct pairs are kept.
    """
    if m > n * (n - 1) // 2:
        raise ValueError("m exceeds the number of vertex pairs")
    w = np.power(np.arange(1, n + 1, dtype=np.float64), -1.0 / (gamma - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    kept = np.empty(0, dtype=np.int64)
    pos = stream_offset
    while kept.size < m:
        need = m - kept.size
        batch = max(1024, int(need * 1.3) + 64)
        uu = uniform01(seed, pos, 2 * batch)
        pos += 2 * batch
        a = np.minimum(np.searchsorted(cdf, uu[0::2], side="right"), n - 1)
        b = np.minimum(np.searchsorted(cdf, uu[1::2], side="right"), n - 1)
        lo = np.minimum(a, b)
        hi = np.maximum(a, b)
        ok = lo != hi
        key = (lo * n + hi)[ok]
        _, first = np.unique(key, return_index=True)
        first.sort()
        key = key[first]
        key = key[~np.isin(key, kept)]
        kept = np.concatenate([kept, key[:need]])
    u = kept // n
    v = kept % n
    g = from_edge_list(n, u, v, name=name or f"chung_lu(n={n},m={m},gamma={gamma},seed={seed})")
    g.meta.update(kind="chung_lu", gamma=gamma, seed=seed, m_target=m)
    return g


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int,
         name: str = "", chunk: int = 1 << 21) -> Graph:
    """R-MAT graph (Chakrabarti, Zhan & Faloutsos 2004), symmetrised.

    edge_factor * 2^scale draws; each picks one of four quadrants per level
    with probabilities a, b, c, d = 1-a-b-c (no noise), most significant bit
    first.  Pairs are symmetrised, deduplicated and self-loops dropped; ids are
    not permuted.
    """
    n = 1 << scale
    draws = edge_factor * n
    us, vs = [], []
    pos = 0
    t_ab, t_abc = a + b, a + b + c
    for start in range(0, draws, chunk):
        cnt = min(chunk, draws - start)
        uu = uniform01(seed, pos, cnt * scale).reshape(cnt, scale)
        pos += cnt * scale
        row_bit = (uu >= t_ab).astype(np.int64)
        col_bit = (((uu >= a) & (uu < t_ab)) | (uu >= t_abc)).astype(np.int64)
        weights = (1 << np.arange(scale - 1, -1, -1, dtype=np.int64))
        us.append(row_bit @ weights)
        vs.append(col_bit @ weights)
    u = np.concatenate(us)
    v = np.concatenate(vs)
    g = from_edge_list(n, u, v, name=name or f"rmat(scale={scale},ef={edge_factor},seed={seed})")
    g.meta.update(kind="rmat", scale=scale, edge_factor=edge_factor, seed=seed)
    return g


def rmat_directed(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int,
                  name: str = "", chunk: int = 1 << 21) -> Graph:
    """R-MAT digraph: the draws of rmat() taken as arcs row -> column (not
    symmetrised), deduplicated, self-loops dropped."""
    n = 1 << scale
    draws = edge_factor * n
    us, vs = [], []
    pos = 0
    t_ab, t_abc = a + b, a + b + c
    for start in range(0, draws, chunk):
        cnt = min(chunk, draws - start)
        uu = uniform01(seed, pos, cnt * scale).reshape(cnt, scale)
        pos += cnt * scale
        row_bit = (uu >= t_ab).astype(np.int64)
        col_bit = (((uu >= a) & (uu < t_ab)) | (uu >= t_abc)).astype(np.int64)
        weights = (1 << np.arange(scale - 1, -1, -1, dtype=np.int64))
        us.append(row_bit @ weights)
        vs.append(col_bit @ weights)
    g = from_arc_list(n, np.concatenate(us), np.concatenate(vs),
                      name=name or f"rmat_dir(scale={scale},ef={edge_factor},seed={seed})")
    g.meta.update(kind="rmat_directed", scale=scale, edge_factor=edge_factor, seed=seed)
    return g


def wc_p(g: Graph) -> np.ndarray:
    """Weighted-cascade probabilities of a digraph: arc u -> v gets
    1 / in-degree(v), so the arcs into a vertex sum to one."""
    if not g.directed:
        raise ValueError("the weighted cascade is defined on arcs")
    indeg = np.bincount(g.col.astype(np.int64), minlength=g.n)
    return 1.0 / indeg[g.col.astype(np.int64)].astype(np.float64)


def random_small_digraph(n: int, m: int, seed: int) -> Graph:
    """Uniform random simple digraph with n vertices and m arcs (m <= n(n-1))."""
    arcs = [(i, j) for i in range(n) for j in range(n) if i != j]
    if m > len(arcs):
        raise ValueError("too many arcs")
    keys = splitmix64_stream(seed, 0, len(arcs))
    sel = np.array([arcs[i] for i in sorted(np.argsort(keys, kind="stable")[:m])], dtype=np.int64).reshape(-1, 2)
    return from_arc_list(n, sel[:, 0], sel[:, 1], name=f"drand({n},{m},{seed})")


def trivalency_p(g: Graph, graph_seed: int, values=(0.1, 0.01, 0.001)) -> np.ndarray:
    """Per-slot probabilities drawn from `values` by a hash of the edge.

    The class of undirected edge {u<v} is SplitMix64's finaliser applied to
    (graph_seed << 40) ^ (u * n + v), reduced mod len(values); both slots of
    the edge receive the same value.  This is input data: the library and the
    oracle both read the resulting array.
    """
    rows = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    cols = g.col.astype(np.int64)
    lo = np.minimum(rows, cols)
    hi = np.maximum(rows, cols)
    key = (lo * g.n + hi).astype(np.uint64) ^ (np.uint64(graph_seed) << np.uint64(40))
    cls = (_mix64(key) % np.uint64(len(values))).astype(np.int64)
    return np.asarray(values, dtype=np.float64)[cls]


def _edge_uniforms(g: Graph, seed: int, stream: int) -> np.ndarray:
    """One uniform double in [0, 1) per slot, equal on both slots of an edge:
    the SplitMix64 finaliser of (seed << 40) ^ (stream << 36) ^ (u * n + v),
    u < v, top 53 bits."""
    rows = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    cols = g.col.astype(np.int64)
    lo = np.minimum(rows, cols)
    hi = np.maximum(rows, cols)
    key = (lo * g.n + hi).astype(np.uint64) ^ (np.uint64(seed) << np.uint64(40)) ^ (
        np.uint64(stream) << np.uint64(36))
    return (_mix64(key) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def uniform_p(g: Graph, seed: int, lo: float = 0.0, hi: float = 0.1) -> np.ndarray:
    """Per-slot probabilities drawn uniformly from [lo, hi) per undirected
    edge (the paper's third weight setting, U[0, 0.1])."""
    return lo + (hi - lo) * _edge_uniforms(g, seed, 1)


def normal_p(g: Graph, seed: int, mean: float = 0.05, sd: float = 0.025) -> np.ndarray:
    """Per-slot probabilities from N(mean, sd) per undirected edge (Box-Muller
    on two edge uniforms), clipped to [0, 1] (the paper's second weight
    setting, N(0.05, 0.025))."""
    u1 = _edge_uniforms(g, seed, 2)
    u2 = _edge_uniforms(g, seed, 3)
    z = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
    return np.clip(mean + sd * z, 0.0, 1.0)


def star_graph(n: int) -> Graph:
    """Star centred at vertex 0 with leaves 1..n-1."""
    leaves = np.arange(1, n, dtype=np.int64)
    return from_edge_list(n, np.zeros_like(leaves), leaves, name=f"star({n})")


def path_graph(n: int) -> Graph:
    a = np.arange(n - 1, dtype=np.int64)
    return from_edge_list(n, a, a + 1, name=f"path({n})")


def random_small_graph(n: int, m: int, seed: int) -> Graph:
    """Uniform random simple graph with n vertices and m edges (m <= n(n-1)/2)."""
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    if m > len(pairs):
        raise ValueError("too many edges")
    keys = splitmix64_stream(seed, 0, len(pairs))
    order = np.argsort(keys, kind="stable")[:m]
    sel = np.array([pairs[i] for i in sorted(order)], dtype=np.int64).reshape(-1, 2)
    if m == 0:
        return from_edge_list(n, np.empty(0, np.int64), np.empty(0, np.int64), name=f"rand({n},{m},{seed})")
    return from_edge_list(n, sel[:, 0], sel[:, 1], name=f"rand({n},{m},{seed})")
