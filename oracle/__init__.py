"""Python access to the plain CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this
package and this package never imports the GPU library.

The oracle follows the paper's definitions directly (see oracle.c): hash
liveness of Eq. 1-2, per-sample BFS components with minimum-id labels, initial
gains of Algorithm 5, CELF of Algorithm 7 with RandCas re-evaluation
(Algorithm 4) on the same samples, and sigma counts.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODE_HASH, MODE_ENUM, MODE_TABLE = 0, 1, 2

_lib = None


def build(force: bool = True) -> str:
    """Compiles oracle.c into liboracle.so with gcc (no intrinsics, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp,
                               _SRC, "-lpthread", "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = C.CDLL(_LIB)
    u32, u64, i32, i64, dbl = C.c_uint32, C.c_uint64, C.c_int32, C.c_int64, C.c_double
    vp = C.c_void_p
    lib.orc_fmix32.argtypes = [u32]
    lib.orc_fmix32.restype = u32
    lib.orc_edge_key.argtypes = [u32, u32, u32]
    lib.orc_edge_key.restype = u32
    lib.orc_edge_hash.argtypes = [u32, u32, u32, u32]
    lib.orc_edge_hash.restype = u32
    lib.orc_sample_value.argtypes = [u32, u32]
    lib.orc_sample_value.restype = u32
    lib.orc_threshold.argtypes = [dbl]
    lib.orc_threshold.restype = u64
    lib.orc_is_live.argtypes = [u32, u32, u64]
    lib.orc_is_live.restype = C.c_int
    common = [u32, vp, vp, C.c_int, dbl, vp, u32, u32, vp]
    lib.orc_label_all.argtypes = common + [vp, vp, vp, vp, vp, C.c_int]
    lib.orc_label_all.restype = C.c_int
    lib.orc_label_range.argtypes = common + [u32, u32, vp]
    lib.orc_label_range.restype = C.c_int
    lib.orc_sigma_count.argtypes = common + [vp, u32, C.c_int]
    lib.orc_sigma_count.restype = i64
    lib.orc_gain.argtypes = common + [u32, vp, C.c_int]
    lib.orc_gain.restype = i64
    lib.orc_celf.argtypes = common + [vp, u32, vp, vp, vp, vp, C.c_int]
    lib.orc_celf.restype = C.c_int
    lib.orc_celf_memo.argtypes = [u32, u32, vp, vp, vp, u32, vp, vp, vp, vp]
    lib.orc_celf_memo.restype = C.c_int
    lib.orc_arc_key.argtypes = [u32, u32, u32]
    lib.orc_arc_key.restype = u32
    lib.orc_arc_hash.argtypes = [u32, u32, u32, u32]
    lib.orc_arc_hash.restype = u32
    lib.orc_sigma_count_arcs.argtypes = [u32, vp, vp, dbl, vp, u32, u32, vp, u32, C.c_int]
    lib.orc_sigma_count_arcs.restype = i64
    lib.orc_celf_arcs.argtypes = [u32, vp, vp, dbl, vp, u32, u32, u32, vp, vp, vp, vp]
    lib.orc_celf_arcs.restype = C.c_int
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Sampler:
    """Which liveness rule the oracle applies.

    mode 'hash'  : Eq. 1-2 with uniform p (or the graph's per-slot p)
    mode 'enum'  : sample r is the world whose live undirected edges are the
                   set bits of r (edge ids in CSR order of the smaller end)
    mode 'table' : explicit table[r, e] of live flags
    """

    def __init__(self, mode: str = "hash", p: float = 0.0, R: int = 1, seed: int = 0,
                 table: Optional[np.ndarray] = None, p_slot: Optional[np.ndarray] = None):
        self.mode = {"hash": MODE_HASH, "enum": MODE_ENUM, "table": MODE_TABLE}[mode]
        self.p = float(p)
        self.R = int(R)
        self.seed = int(seed) & 0xFFFFFFFF
        self.table = None if table is None else np.ascontiguousarray(table, dtype=np.uint8)
        self.p_slot = None if p_slot is None else np.ascontiguousarray(p_slot, dtype=np.float64)
        if self.R < 1:
            raise ValueError("R must be >= 1")


def _args(g, s: Sampler):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.uint64)
    col = np.ascontiguousarray(g.col, dtype=np.uint32)
    p_slot = s.p_slot if s.p_slot is not None else (
        None if g.p_slot is None or s.mode != MODE_HASH else np.ascontiguousarray(g.p_slot, np.float64))
    keep = (rp, col, p_slot, s.table)
    return keep, [g.n, _ptr(rp), _ptr(col), s.mode, s.p, _ptr(p_slot), s.R, s.seed, _ptr(s.table)]


def fmix32(x: int) -> int:
    return _load().orc_fmix32(x & 0xFFFFFFFF)


def edge_key(u: int, v: int, n: int) -> int:
    return _load().orc_edge_key(u, v, n)


def edge_hash(seed: int, u: int, v: int, n: int) -> int:
    return _load().orc_edge_hash(seed & 0xFFFFFFFF, u, v, n)


def sample_value(seed: int, r: int) -> int:
    return _load().orc_sample_value(seed & 0xFFFFFFFF, r & 0xFFFFFFFF)


def threshold(p: float) -> int:
    return _load().orc_threshold(float(p))


def is_live(h: int, x: int, t: int) -> bool:
    return bool(_load().orc_is_live(h, x, t))


def label_all(g, s: Sampler, want_labels: bool = False, digest_w: Optional[np.ndarray] = None,
              threads: int = 1, want_sizes: bool = False):
    """Returns (g0 int64[n], labels int32[n][R] or None, digests uint64[R] or None),
    plus sizes uint32[n][R] as a fourth item when want_sizes is set."""
    lib = _load()
    keep, a = _args(g, s)
    g0 = np.zeros(g.n, dtype=np.int64)
    labels = np.empty((g.n, s.R), dtype=np.int32) if want_labels else None
    sizes = np.empty((g.n, s.R), dtype=np.uint32) if want_sizes else None
    dig = None
    dw = None
    if digest_w is not None:
        dw = np.ascontiguousarray(digest_w, dtype=np.uint64)
        dig = np.zeros(s.R, dtype=np.uint64)
    rc = lib.orc_label_all(*a, _ptr(g0), _ptr(labels), _ptr(sizes), _ptr(dig), _ptr(dw), int(threads))
    if rc != 0:
        raise RuntimeError("oracle: allocation failure")
    del keep
    if want_sizes:
        return g0, labels, dig, sizes
    return g0, labels, dig


def label_range(g, s: Sampler, r0: int, cnt: int) -> np.ndarray:
    lib = _load()
    keep, a = _args(g, s)
    out = np.empty((g.n, cnt), dtype=np.int32)
    if lib.orc_label_range(*a, r0, cnt, _ptr(out)) != 0:
        raise RuntimeError("oracle: allocation failure")
    del keep
    return out


def arc_key(u: int, v: int, n: int) -> int:
    return _load().orc_arc_key(u, v, n)


def arc_hash(seed: int, u: int, v: int, n: int) -> int:
    return _load().orc_arc_hash(seed & 0xFFFFFFFF, u, v, n)


def sigma_count(g, s: Sampler, S, threads: int = 1) -> int:
    """sum_r |vertices reachable from S in sample r|.  On a directed graph
    (g.directed) reachability follows the out-arcs, each arc hashed from its
    ordered pair (hash sampling only)."""
    lib = _load()
    S = np.ascontiguousarray(np.asarray(S, dtype=np.uint32))
    if getattr(g, "directed", False):
        if s.mode != MODE_HASH:
            raise ValueError("directed graphs use hash sampling")
        rp = np.ascontiguousarray(g.row_ptr, dtype=np.uint64)
        col = np.ascontiguousarray(g.col, dtype=np.uint32)
        p_slot = s.p_slot if s.p_slot is not None else (
            None if g.p_slot is None else np.ascontiguousarray(g.p_slot, np.float64))
        r = lib.orc_sigma_count_arcs(g.n, _ptr(rp), _ptr(col), s.p, _ptr(p_slot), s.R, s.seed, _ptr(S),
                                     int(S.size), int(threads))
        del rp, col, p_slot
        return int(r)
    keep, a = _args(g, s)
    r = lib.orc_sigma_count(*a, _ptr(S), int(S.size), int(threads))
    del keep
    return int(r)


def celf_arcs(g, s: Sampler, K: int) -> dict:
    """Lazy greedy on a digraph (hash sampling): seeds, marginal counts,
    cover count and the number of evaluations."""
    if not getattr(g, "directed", False) or s.mode != MODE_HASH:
        raise ValueError("celf_arcs takes a digraph and hash sampling")
    lib = _load()
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.uint64)
    col = np.ascontiguousarray(g.col, dtype=np.uint32)
    p_slot = s.p_slot if s.p_slot is not None else (
        None if g.p_slot is None else np.ascontiguousarray(g.p_slot, np.float64))
    seeds = np.zeros(max(K, 1), dtype=np.uint32)
    marg = np.zeros(max(K, 1), dtype=np.int64)
    cover = C.c_int64()
    evals = C.c_uint64()
    rc = lib.orc_celf_arcs(g.n, _ptr(rp), _ptr(col), s.p, _ptr(p_slot), s.R, s.seed, int(K), _ptr(seeds),
                           _ptr(marg), C.byref(cover), C.byref(evals))
    if rc == -2:
        raise ValueError("K > n")
    if rc != 0:
        raise RuntimeError("oracle: allocation failure")
    return {"seeds": seeds[:K], "marginal": marg[:K], "cover": int(cover.value), "evals": int(evals.value)}


def gain(g, s: Sampler, u: int, seed_set=(), threads: int = 1) -> int:
    lib = _load()
    keep, a = _args(g, s)
    is_seed = np.zeros(max(g.n, 1), dtype=np.uint8)
    for x in seed_set:
        is_seed[int(x)] = 1
    r = lib.orc_gain(*a, int(u), _ptr(is_seed), int(threads))
    del keep
    return int(r)


def celf(g, s: Sampler, K: int, g0: np.ndarray, threads: int = 1):
    """Returns (seeds uint32[K], marginal int64[K], cover_count, n_evals)."""
    lib = _load()
    keep, a = _args(g, s)
    g0 = np.ascontiguousarray(g0, dtype=np.int64)
    seeds = np.zeros(K, dtype=np.uint32)
    marg = np.zeros(K, dtype=np.int64)
    cover = C.c_int64(0)
    evals = C.c_uint64(0)
    rc = lib.orc_celf(*a, _ptr(g0), int(K), _ptr(seeds), _ptr(marg), C.byref(cover),
                      C.byref(evals), int(threads))
    del keep
    if rc == -2:
        raise ValueError("K > n")
    if rc != 0:
        raise RuntimeError("oracle: allocation failure")
    return seeds, marg, int(cover.value), int(evals.value)


def run(g, s: Sampler, K: int, want_labels: bool = False, digest_w=None, threads: int = 1) -> dict:
    """Whole method on the oracle: labels/g0, then CELF."""
    g0, labels, dig = label_all(g, s, want_labels=want_labels, digest_w=digest_w, threads=threads)
    seeds, marg, cover, evals = celf(g, s, K, g0, threads=threads)
    return dict(g0=g0, labels=labels, digests=dig, seeds=seeds, marginal=marg, cover=cover,
                evals=evals)


def celf_memo(labels: np.ndarray, sizes: np.ndarray, g0: np.ndarray, K: int):
    """CELF evaluating gains from stored labels and sizes (memo formula).
    Returns (seeds, marginal, cover, n_evals)."""
    lib = _load()
    n, R = labels.shape
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    sizes = np.ascontiguousarray(sizes, dtype=np.uint32)
    g0 = np.ascontiguousarray(g0, dtype=np.int64)
    seeds = np.zeros(K, dtype=np.uint32)
    marg = np.zeros(K, dtype=np.int64)
    cover = C.c_int64(0)
    evals = C.c_uint64(0)
    rc = lib.orc_celf_memo(n, R, _ptr(labels), _ptr(sizes), _ptr(g0), int(K), _ptr(seeds),
                           _ptr(marg), C.byref(cover), C.byref(evals))
    if rc == -2:
        raise ValueError("K > n")
    if rc != 0:
        raise RuntimeError("oracle: allocation failure")
    return seeds, marg, int(cover.value), int(evals.value)


def run_memo(g, s: Sampler, K: int, digest_w=None, threads: int = 1, keep_arrays: bool = False) -> dict:
    """Whole method with the memo-formula CELF (Algorithm 7's evaluation)."""
    g0, labels, dig, sizes = label_all(g, s, want_labels=True, digest_w=digest_w, threads=threads,
                                       want_sizes=True)
    seeds, marg, cover, evals = celf_memo(labels, sizes, g0, K)
    out = dict(g0=g0, digests=dig, seeds=seeds, marginal=marg, cover=cover, evals=evals)
    if keep_arrays:
        out.update(labels=labels, sizes=sizes)
    return out
