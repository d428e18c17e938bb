"""Python binding of libinfuse (include/infuse.h): argument marshalling only.

Every step of the method runs in the HIP library; this module converts numpy
arrays to pointers, hands PyTorch's caching allocator and a torch stream to
the library, and converts results back.  There is no CPU fallback: without
the built library every call raises.
"""

from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence, Tuple

import numpy as np

from ._lib import (ALLOC_FN, FREE_FN, InfuseError, check, im_allocator, im_query, im_result,
                   im_server_config, im_tuning, load)

__all__ = ["Context", "Graph", "Server", "InfuseError", "batch_select", "load"]


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Context:
    """Device, stream and allocator binding (im_ctx_create).

    By default device memory comes from PyTorch's caching allocator and work
    runs on a dedicated torch stream of the device.
    """

    def __init__(self, device: int = 0, hbm_budget: int = 0, torch_memory: bool = True,
                 stream=None, allocator=None):
        """allocator: optional (alloc(nbytes) -> device pointer or None,
        free(ptr)) pair of callables used as the context's allocator
        callbacks instead of PyTorch's caching allocator."""
        self._lib = load()
        self._cb = None
        self.device = device
        alloc_p = None
        handle = None
        try:
            import torch
            have_torch = torch.cuda.is_available()
        except Exception:  # pragma: no cover - torch is part of the image
            have_torch = False
        if have_torch:
            if stream is None:
                stream = torch.cuda.Stream(device=device)
            self._stream = stream
            handle = stream.cuda_stream
        else:
            self._stream = None
        if allocator is not None:
            user_alloc, user_free = allocator

            def _alloc(user, nbytes, s):
                try:
                    return user_alloc(int(nbytes))
                except Exception:
                    return None

            def _free(user, ptr, s):
                user_free(ptr)

            self._cb = (ALLOC_FN(_alloc), FREE_FN(_free))
            self._alloc_struct = im_allocator(self._cb[0], self._cb[1], None)
            alloc_p = C.byref(self._alloc_struct)
        elif have_torch and torch_memory:
            dev = device
            st = handle

            def _alloc(user, nbytes, s):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, st)
                except Exception:
                    return None

            def _free(user, ptr, s):
                torch.cuda.caching_allocator_delete(ptr)

            self._cb = (ALLOC_FN(_alloc), FREE_FN(_free))
            self._alloc_struct = im_allocator(self._cb[0], self._cb[1], None)
            alloc_p = C.byref(self._alloc_struct)
        out = C.c_void_p()
        check(self._lib.im_ctx_create(device, C.c_void_p(handle) if handle else None, alloc_p,
                                      int(hbm_budget), C.byref(out)))
        self.handle = out

    @property
    def stream(self):
        return self._stream

    def close(self):
        if getattr(self, "handle", None):
            self._lib.im_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bytes_in_use(self) -> int:
        return int(self._lib.im_ctx_bytes_in_use(self.handle))

    CELF_PERSISTENT, CELF_PER_STEP = 1, 2

    def set_tuning(self, cc_chunk: int = 0, celf_width: int = 0, use_graphs: Optional[bool] = None,
                   celf_mode: int = 0, celf_round0: Optional[int] = None, list_blocks: int = 0):
        t = im_tuning()
        t.cc_chunk = cc_chunk
        t.list_blocks = list_blocks
        t.celf_width = celf_width
        t.use_graphs = 0 if use_graphs is None else (1 if use_graphs else 2)
        t.celf_mode = celf_mode
        # celf_round0: None keeps the current value, 0 selects automatic
        t.celf_round0 = 0xFFFFFFFF if celf_round0 is None else int(celf_round0)
        check(self._lib.im_set_tuning(self.handle, C.byref(t)))

    def tuning(self) -> dict:
        t = im_tuning()
        check(self._lib.im_get_tuning(self.handle, C.byref(t)))
        return dict(cc_chunk=t.cc_chunk, celf_width=t.celf_width, use_graphs=bool(t.use_graphs),
                    celf_mode=t.celf_mode, celf_round0=t.celf_round0, list_blocks=t.list_blocks)

    def autotune(self, graph: "Graph", K: int, reps: int = 2, cache: Optional[str] = None) -> dict:
        """Launch shapes for `graph` (im_autotune), applied to this context.

        With `cache` (a JSON file), a shape found before for a graph of the
        same size class (n, slots, R, hubs) is applied without timing, and a
        new one is stored."""
        import json
        import os

        key = None
        if cache:
            rp = np.diff(np.asarray(graph._row_ptr, dtype=np.int64)) if graph._row_ptr is not None else None
            hubs = int((rp > 64).sum()) if rp is not None else -1
            key = f"n={graph.n},nnz={graph.nnz},R={graph.R},hubs={hubs},mode={self.tuning()['celf_mode']}"
            if os.path.exists(cache):
                with open(cache) as f:
                    known = json.load(f)
                if key in known:
                    self.set_tuning(cc_chunk=known[key]["cc_chunk"], celf_round0=known[key]["celf_round0"],
                                    list_blocks=known[key].get("list_blocks", 0))
                    return self.tuning()
        t = im_tuning()
        check(self._lib.im_autotune(graph.handle, int(K), int(reps), C.byref(t)))
        out = self.tuning()
        if cache:
            known = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    known = json.load(f)
            known[key] = out
            with open(cache, "w") as f:
                json.dump(known, f, indent=1, sort_keys=True)
        return out

    def set_profiling(self, level):
        """0/False: off; 1/True: per-build kernels; 2: also every CELF launch and
        the persistent CELF phase clock; 3: also memo-construction work counts."""
        check(self._lib.im_set_profiling(self.handle, int(level)))

    def reset_kernel_stats(self):
        check(self._lib.im_reset_kernel_stats(self.handle))

    def kernel_stats(self, name: str) -> Tuple[int, float]:
        n = C.c_uint64()
        ms = C.c_double()
        check(self._lib.im_kernel_stats(self.handle, name.encode(), C.byref(n), C.byref(ms)))
        return int(n.value), float(ms.value)


class Graph:
    """A CSR graph resident on the device: undirected (im_graph_load_csr) or,
    with directed=True, the out-arcs of every vertex (im_graph_load_arcs)."""

    def __init__(self, ctx: Context, n: int, row_ptr: np.ndarray, col: np.ndarray,
                 p_slot: Optional[np.ndarray] = None, directed: bool = False):
        self._lib = ctx._lib
        self.ctx = ctx
        self.n = int(n)
        rp = np.ascontiguousarray(row_ptr, dtype=np.uint64)
        cl = np.ascontiguousarray(col, dtype=np.uint32)
        ps = None if p_slot is None else np.ascontiguousarray(p_slot, dtype=np.float64)
        out = C.c_void_p()
        load = self._lib.im_graph_load_arcs if directed else self._lib.im_graph_load_csr
        check(load(ctx.handle, self.n, int(rp[-1]) if rp.size else 0, _ptr(rp), _ptr(cl), _ptr(ps),
                   C.byref(out)))
        self.directed = bool(directed)
        self.handle = out
        self.R = 0
        self.nnz = int(rp[-1]) if rp.size else 0
        self._row_ptr = rp

    @classmethod
    def from_csr(cls, ctx: Context, g) -> "Graph":
        """From any object with n, row_ptr, col and optional p_slot and
        directed."""
        return cls(ctx, g.n, g.row_ptr, g.col, getattr(g, "p_slot", None), bool(getattr(g, "directed", False)))

    def free(self):
        if getattr(self, "handle", None):
            self._lib.im_graph_free(self.handle)
            self.handle = None

    def set_params(self, p: float, R: int, seed: int):
        check(self._lib.im_set_params(self.handle, float(p), int(R), int(seed) & 0xFFFFFFFF))
        self.R = int(R)

    def build_memo(self):
        check(self._lib.im_build_memo(self.handle))

    def drop_memo(self):
        check(self._lib.im_drop_memo(self.handle))

    def select_seeds(self, K: int):
        seeds = np.zeros(max(K, 1), dtype=np.uint32)
        marg = np.zeros(max(K, 1), dtype=np.int64)
        cover = C.c_int64()
        check(self._lib.im_select_seeds(self.handle, int(K), _ptr(seeds), _ptr(marg), C.byref(cover)))
        return seeds[:K], marg[:K], int(cover.value)

    def estimate_sigma(self, S: Sequence[int]):
        arr = np.ascontiguousarray(np.asarray(S, dtype=np.uint32))
        cnt = C.c_int64()
        sig = C.c_double()
        check(self._lib.im_estimate_sigma(self.handle, _ptr(arr) if arr.size else None, int(arr.size),
                                          C.byref(cnt), C.byref(sig)))
        return int(cnt.value), float(sig.value)

    def estimate_sigma_noalloc(self, S: Sequence[int]):
        """sigma(S) on the resident memo without device allocation
        (im_estimate_sigma_noalloc): (count, sigma)."""
        arr = np.ascontiguousarray(np.asarray(S, dtype=np.uint32))
        cnt = C.c_int64()
        sig = C.c_double()
        check(self._lib.im_estimate_sigma_noalloc(self.handle, _ptr(arr) if arr.size else None, int(arr.size),
                                                  C.byref(cnt), C.byref(sig)))
        return int(cnt.value), float(sig.value)

    def select_seeds_direct(self, K: int):
        """Greedy selection without a memo (im_select_seeds_direct), also for
        directed graphs: (seeds, marginal, cover)."""
        seeds = np.zeros(max(K, 1), dtype=np.uint32)
        marg = np.zeros(max(K, 1), dtype=np.int64)
        cover = C.c_int64()
        check(self._lib.im_select_seeds_direct(self.handle, int(K), _ptr(seeds), _ptr(marg), C.byref(cover)))
        return seeds[:K], marg[:K], int(cover.value)

    def estimate_sigma_direct(self, S: Sequence[int]):
        """sigma(S) without a memo (im_estimate_sigma_direct): (count, sigma, levels)."""
        arr = np.ascontiguousarray(np.asarray(S, dtype=np.uint32))
        cnt = C.c_int64()
        sig = C.c_double()
        lv = C.c_uint32()
        check(self._lib.im_estimate_sigma_direct(self.handle, _ptr(arr) if arr.size else None, int(arr.size),
                                                 C.byref(cnt), C.byref(sig), C.byref(lv)))
        return int(cnt.value), float(sig.value), int(lv.value)

    def labels(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        count = self.R - first if count is None else count
        out = np.empty((self.n, count), dtype=np.int32)
        check(self._lib.im_copy_labels(self.handle, _ptr(out), int(first), int(count)))
        return out

    def sizes(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        count = self.R - first if count is None else count
        out = np.empty((self.n, count), dtype=np.int32)
        check(self._lib.im_copy_sizes(self.handle, _ptr(out), int(first), int(count)))
        return out

    def gains0(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int64)
        check(self._lib.im_copy_gains0(self.handle, _ptr(out)))
        return out

    def phase_ms(self) -> List[float]:
        a = (C.c_double * 4)()
        check(self._lib.im_last_phase_ms(self.handle, a))
        return [float(x) for x in a]

    def celf_evals(self) -> int:
        return int(self._lib.im_last_celf_evals(self.handle))

    def search_stats(self) -> dict:
        """Work counts of the last memo-free call on this graph."""
        a = (C.c_uint64 * 4)()
        check(self._lib.im_last_search_stats(self.handle, a))
        return dict(levels=int(a[0]), items=int(a[1]), arcs=int(a[2]), live_pairs=int(a[3]))

    WORK_KEYS = ("live_pairs", "union_attempts", "flatten_rewrites", "count_atomics", "row_tiles", "hub_tiles",
                 "gain_gathers", "hub_link_waves")

    def memo_work(self) -> dict:
        """Work counts of the resident memo's construction (built while the
        context's profiling level was 4)."""
        a = (C.c_uint64 * len(self.WORK_KEYS))()
        check(self._lib.im_memo_work(self.handle, a, len(self.WORK_KEYS)))
        return {k: int(v) for k, v in zip(self.WORK_KEYS, a)}

    def memo_stats(self) -> dict:
        a = (C.c_uint64 * 4)()
        check(self._lib.im_memo_stats(self.handle, a))
        return dict(listed_tiles=int(a[0]), link_tiles=int(a[1]), hubs=int(a[2]), memo_bytes=int(a[3]))


def batch_select(ctx: Context, graphs: Sequence[Graph], Ks: Sequence[int]):
    """im_batch_select: every graph's memo and selection in batched launches."""
    lib = ctx._lib
    ng = len(graphs)
    kv = np.ascontiguousarray(np.asarray(Ks, dtype=np.uint32).reshape(-1))
    kmax = max(1, int(kv.max())) if ng else 1
    # one block per output kind, row i for graph i; the pointer tables are
    # built with numpy (a ctypes object per graph would cost more than the
    # call's device work for many small graphs)
    seeds = np.zeros((ng, kmax), dtype=np.uint32)
    margs = np.zeros((ng, kmax), dtype=np.int64)
    rows = np.arange(ng, dtype=np.uint64)
    sp = np.uint64(seeds.ctypes.data) + rows * np.uint64(seeds.strides[0])
    mp = np.uint64(margs.ctypes.data) + rows * np.uint64(margs.strides[0])
    hv = np.array([g.handle.value for g in graphs], dtype=np.uint64)
    cov = np.zeros(ng, dtype=np.int64)
    check(lib.im_batch_select(ctx.handle, ng, hv.ctypes.data_as(C.POINTER(C.c_void_p)),
                              kv.ctypes.data_as(C.POINTER(C.c_uint32)),
                              sp.ctypes.data_as(C.POINTER(C.POINTER(C.c_uint32))),
                              mp.ctypes.data_as(C.POINTER(C.POINTER(C.c_int64))),
                              cov.ctypes.data_as(C.POINTER(C.c_int64))))
    return [(seeds[i, :kv[i]], margs[i, :kv[i]], int(cov[i])) for i in range(ng)]


class Server:
    """Serving loop (im_server_*): admission by HBM budget, resident memos,
    overlapping queries on per-slot streams."""

    SIGMA, SELECT = 0, 1

    def __init__(self, ctx: Context, slots: int = 4, persistent_min_mwords: int = 0):
        self._lib = ctx._lib
        self.ctx = ctx
        cfg = im_server_config()
        cfg.slots = slots
        cfg.persistent_min_mwords = persistent_min_mwords
        out = C.c_void_p()
        check(self._lib.im_server_create(ctx.handle, C.byref(cfg), C.byref(out)))
        self.handle = out
        self._kept = {}

    def submit_sigma(self, g: Graph, S, p: float, R: int, seed: int) -> int:
        arr = np.ascontiguousarray(np.asarray(S, dtype=np.uint32))
        q = im_query(0, 0, float(p), int(R), int(seed) & 0xFFFFFFFF,
                     arr.ctypes.data_as(C.POINTER(C.c_uint32)), int(arr.size))
        t = C.c_uint64()
        check(self._lib.im_server_submit(self.handle, g.handle, C.byref(q), C.byref(t)))
        return int(t.value)

    def submit_select(self, g: Graph, K: int, p: float, R: int, seed: int) -> int:
        q = im_query(1, int(K), float(p), int(R), int(seed) & 0xFFFFFFFF, None, 0)
        t = C.c_uint64()
        check(self._lib.im_server_submit(self.handle, g.handle, C.byref(q), C.byref(t)))
        self._kept[int(t.value)] = int(K)
        return int(t.value)

    def poll(self, ticket: int, wait_ms: int = 0):
        """Returns None while running, else a dict (seeds/marginal for selections)."""
        res = im_result()
        K = self._kept.get(ticket, 0)
        seeds = np.zeros(max(K, 1), dtype=np.uint32)
        marg = np.zeros(max(K, 1), dtype=np.int64)
        st = self._lib.im_server_poll(self.handle, int(ticket), int(wait_ms), C.byref(res),
                                      _ptr(seeds), _ptr(marg))
        if st == 6:  # IM_ERR_NOT_READY
            return None
        check(st)
        self._kept.pop(ticket, None)
        out = dict(status=int(res.status), count=int(res.count), sigma=float(res.sigma),
                   latency_ms=float(res.latency_ms), queue_ms=float(res.queue_ms),
                   memo_hit=bool(res.memo_hit))
        if K:
            out["seeds"] = seeds[:K]
            out["marginal"] = marg[:K]
        return out

    def cancel(self, ticket: int):
        check(self._lib.im_server_cancel(self.handle, int(ticket)))

    def drain(self):
        check(self._lib.im_server_drain(self.handle))

    def stats(self) -> dict:
        a = (C.c_uint64 * 7)()
        check(self._lib.im_server_stats(self.handle, a))
        keys = ["admitted", "completed", "rejected", "memo_hits", "memo_builds", "evictions",
                "peak_concurrent"]
        return {k: int(v) for k, v in zip(keys, a)}

    def close(self):
        if getattr(self, "handle", None):
            self._lib.im_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
