"""ctypes declarations of the C ABI in include/infuse.h (marshalling only)."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libinfuse.so")

IM_OK = 0
STATUS_NAMES = {
    0: "IM_OK", 1: "IM_ERR_INVALID_ARG", 2: "IM_ERR_INVALID_GRAPH", 3: "IM_ERR_OUT_OF_MEMORY",
    4: "IM_ERR_DEVICE", 5: "IM_ERR_BUDGET", 6: "IM_ERR_NOT_READY", 7: "IM_ERR_CANCELLED",
    8: "IM_ERR_NOT_FOUND",
}


class InfuseError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class im_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class im_tuning(C.Structure):
    _fields_ = [("cc_chunk", C.c_uint32), ("celf_width", C.c_uint32), ("use_graphs", C.c_uint32),
                ("celf_mode", C.c_uint32), ("celf_round0", C.c_uint32), ("list_blocks", C.c_uint32),
                ("reserved", C.c_uint32 * 2)]


class im_server_config(C.Structure):
    _fields_ = [("slots", C.c_uint32), ("persistent_min_mwords", C.c_uint32), ("reserved", C.c_uint32 * 6)]


class im_query(C.Structure):
    _fields_ = [("kind", C.c_int32), ("K", C.c_uint32), ("p", C.c_double), ("R", C.c_uint32),
                ("hash_seed", C.c_uint32), ("S", C.POINTER(C.c_uint32)), ("s_len", C.c_uint32)]


class im_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("count", C.c_int64), ("sigma", C.c_double),
                ("latency_ms", C.c_double), ("queue_ms", C.c_double), ("memo_hit", C.c_uint32),
                ("reserved", C.c_uint32)]


# name -> (restype, argtypes); every name here is declared in include/infuse.h
vp, u32, u64, i32, i64, dbl = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32, C.c_int64, C.c_double
P = C.POINTER
SIGNATURES = {
    "im_last_error": (C.c_char_p, []),
    "im_version": (C.c_char_p, []),
    "im_ctx_create": (C.c_int, [C.c_int, vp, P(im_allocator), u64, P(vp)]),
    "im_ctx_destroy": (None, [vp]),
    "im_ctx_bytes_in_use": (u64, [vp]),
    "im_graph_load_csr": (C.c_int, [vp, u32, u64, vp, vp, vp, P(vp)]),
    "im_graph_load_arcs": (C.c_int, [vp, u32, u64, vp, vp, vp, P(vp)]),
    "im_graph_free": (None, [vp]),
    "im_set_params": (C.c_int, [vp, dbl, u32, u32]),
    "im_build_memo": (C.c_int, [vp]),
    "im_drop_memo": (C.c_int, [vp]),
    "im_select_seeds": (C.c_int, [vp, u32, vp, vp, P(i64)]),
    "im_estimate_sigma": (C.c_int, [vp, vp, u32, P(i64), P(dbl)]),
    "im_estimate_sigma_direct": (C.c_int, [vp, vp, u32, P(i64), P(dbl), P(u32)]),
    "im_estimate_sigma_noalloc": (C.c_int, [vp, vp, u32, P(i64), P(dbl)]),
    "im_select_seeds_direct": (C.c_int, [vp, u32, vp, vp, P(i64)]),
    "im_copy_labels": (C.c_int, [vp, vp, u64, u32]),
    "im_copy_sizes": (C.c_int, [vp, vp, u64, u32]),
    "im_copy_gains0": (C.c_int, [vp, vp]),
    "im_graph_n": (u32, [vp]),
    "im_graph_nnz": (u64, [vp]),
    "im_set_tuning": (C.c_int, [vp, P(im_tuning)]),
    "im_get_tuning": (C.c_int, [vp, P(im_tuning)]),
    "im_autotune": (C.c_int, [vp, u32, u32, P(im_tuning)]),
    "im_set_profiling": (C.c_int, [vp, C.c_int]),
    "im_reset_kernel_stats": (C.c_int, [vp]),
    "im_kernel_stats": (C.c_int, [vp, C.c_char_p, P(u64), P(dbl)]),
    "im_last_phase_ms": (C.c_int, [vp, P(dbl)]),
    "im_last_celf_evals": (u64, [vp]),
    "im_last_search_stats": (C.c_int, [vp, P(u64)]),
    "im_memo_stats": (C.c_int, [vp, P(u64)]),
    "im_memo_work": (C.c_int, [vp, P(u64), u32]),
    "im_batch_select": (C.c_int, [vp, u32, P(vp), P(u32), P(P(u32)), P(P(i64)), P(i64)]),
    "im_server_create": (C.c_int, [vp, P(im_server_config), P(vp)]),
    "im_server_submit": (C.c_int, [vp, vp, P(im_query), P(u64)]),
    "im_server_poll": (C.c_int, [vp, u64, u32, P(im_result), vp, vp]),
    "im_server_cancel": (C.c_int, [vp, u64]),
    "im_server_drain": (C.c_int, [vp]),
    "im_server_stats": (C.c_int, [vp, P(u64)]),
    "im_server_destroy": (None, [vp]),
}

_lib = None


def load() -> C.CDLL:
    """Loads libinfuse.so; fails loudly when the HIP library is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2008_03095_amd.build`")
    # PyTorch ships its own HIP/HSA runtime.  Loading it first makes this
    # library's libamdhip64.so.7 / libhsa-runtime64.so.1 dependencies bind to
    # the already-loaded copies (same SONAME), so one runtime serves both and
    # torch streams and allocations are valid here.
    import torch  # noqa: F401

    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int):
    if status != IM_OK:
        msg = load().im_last_error()
        raise InfuseError(status, msg.decode() if msg else "")
