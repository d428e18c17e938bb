"""Test helpers shared by oracle pins and GPU parity tests (no method arithmetic)."""

import numpy as np

from workloads import chung_lu, from_edge_list, splitmix64_stream


def digest_weights(n: int) -> np.ndarray:
    """Random odd 64-bit weights for the per-sample label digest."""
    return splitmix64_stream(0xD16E57, 0, n) | np.uint64(1)


def label_digests(labels_chunk: np.ndarray, w: np.ndarray) -> np.ndarray:
    """sum_v (label[v] + 1) * w[v] mod 2^64 for every column of a [n][c] chunk."""
    x = (labels_chunk.astype(np.int64) + 1).astype(np.uint64)
    with np.errstate(over="ignore"):
        return (x * w[:, None]).sum(axis=0, dtype=np.uint64)


def min_id_labels(n: int, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Connected components of (range(n), {u_i, v_i}) via scipy, relabelled to min id."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    a = sp.coo_matrix((np.ones(len(u)), (np.asarray(u, np.int64), np.asarray(v, np.int64))),
                      shape=(n, n))
    _, comp = connected_components(a, directed=False)
    mins = np.full(comp.max() + 1 if n else 0, n, dtype=np.int64)
    np.minimum.at(mins, comp, np.arange(n))
    return mins[comp].astype(np.int32)


def combine_digests(digests: np.ndarray) -> str:
    """Checksum of all per-sample digests (weights independent of the label weights)."""
    w = splitmix64_stream(0xC0FFEE, 0, digests.size) | np.uint64(1)
    with np.errstate(over="ignore"):
        return "%016x" % int((digests.astype(np.uint64) * w).sum(dtype=np.uint64))


def gains_checksum(g0: np.ndarray) -> str:
    w = splitmix64_stream(0x6A1, 0, g0.size) | np.uint64(1)
    with np.errstate(over="ignore"):
        return "%016x" % int((g0.astype(np.uint64) * w).sum(dtype=np.uint64))


def hub_mix_graph(seed):
    """Hub rows of very different lengths in one graph: vertex n-1 joined to
    0 .. 4,999 (a row of 5,000 slots, nearly all of them smaller neighbours:
    thousands of unions per column), vertex 3 to 1,000 .. 3,999 (3,000 slots,
    nearly all larger), vertex 4,500 to 100 random vertices, over a Chung-Lu
    background (its own hubs of a few hundred slots)."""
    n = 6000
    bg = chung_lu(n, 15000, 2.2, seed)
    rows = np.repeat(np.arange(n), bg.degrees())
    rng = np.random.default_rng(seed)
    us = [rows, np.full(5000, n - 1), np.full(3000, 3), np.full(100, 4500)]
    vs = [bg.col.astype(np.int64), np.arange(5000), np.arange(1000, 4000), rng.integers(0, n, 100)]
    return from_edge_list(n, np.concatenate(us), np.concatenate(vs))
