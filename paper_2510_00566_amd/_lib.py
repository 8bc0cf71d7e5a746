"""ctypes binding of libpanorama.so: the C ABI under the same names.

Only argument marshalling lives here: every step of the search runs in the
HIP library.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpanorama.so")

PANO_OK, PANO_EINVAL, PANO_ENOMEM, PANO_EDEVICE, PANO_EUNSUPPORTED, PANO_EBUSY = range(6)
PANO_F32, PANO_BF16 = 0, 1
PANO_SEARCH_STATS = 1
PANO_SEARCH_EAGER = 2
PANO_SEARCH_TIMING = 4
PANO_SEARCH_ASYNC = 8
PANO_PQ_BRUTE = 16


class SearchParams(C.Structure):
    _fields_ = [("group", C.c_int32), ("blocks_per_item", C.c_int32), ("seed_pool", C.c_int32),
                ("seed_count", C.c_int32), ("grid", C.c_int32), ("use_bf16", C.c_int32),
                ("reserved", C.c_int32 * 6)]


class IndexInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int32), ("d_pad", C.c_int32), ("nlist", C.c_int32),
                ("L", C.c_int32), ("block", C.c_int32), ("has_bf16", C.c_int32), ("nblocks", C.c_int64),
                ("max_list_len", C.c_int64), ("bytes_levels", C.c_int64), ("bytes_levels_bf16", C.c_int64),
                ("bytes_tails", C.c_int64), ("bytes_ids", C.c_int64), ("bytes_raw", C.c_int64),
                ("transform_err_max", C.c_double), ("sigma_ratio", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("nq", C.c_int64), ("candidates", C.c_int64), ("dims_read", C.c_int64),
                ("level_reads", C.c_int64 * 64), ("items", C.c_int64), ("committed", C.c_int64),
                ("band", C.c_int64), ("fallback_queries", C.c_int64), ("ms_total", C.c_double),
                ("ms_scan", C.c_double), ("ms_merge", C.c_double), ("ms_prep", C.c_double),
                ("scan_bytes", C.c_int64), ("scan_cycles", C.c_int64 * 6)]


class PanoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pano status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(python -m paper_2510_00566_amd.build)")
    L = C.CDLL(LIB_PATH)
    P, i32, i64, u32, u64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_float
    PP = C.POINTER(C.c_void_p)
    sig = {
        "pano_last_error": (C.c_char_p, []),
        "pano_version": (C.c_char_p, []),
        "pano_ctx_create": (C.c_int, [C.c_int, PP]),
        "pano_ctx_destroy": (None, [P]),
        "pano_ctx_scratch_bytes": (C.c_int, [P, P]),
        "pano_ctx_trim": (C.c_int, [P]),
        "pano_ctx_status": (C.c_int, [P, P]),
        "pano_build_transform": (C.c_int, [P, i64, i32, i64, u64, PP]),
        "pano_transform_identity": (C.c_int, [i32, PP]),
        "pano_transform_from": (C.c_int, [i32, P, P, PP]),
        "pano_transform_get": (C.c_int, [P, P, P, P, P, P]),
        "pano_transform_free": (None, [P]),
        "pano_ivf_assign": (C.c_int, [P, P, i64, i32, i32, i32, u64, P, P, P]),
        "pano_build_levels": (C.c_int, [P, P, P, i64, i32, P, P, i32, P, i32, i32, C.c_int, PP, P]),
        "pano_search": (C.c_int, [P, P, i64, i32, P, i32, f32, P, P, P, u32, P]),
        "pano_search_ctx": (C.c_int, [P, P, P, i64, i32, P, i32, f32, P, P, P, u32, P]),
        "pano_search_scratch_bytes": (C.c_int, [P, i64, i32, i32, i32, P, P]),
        "pano_search_noalloc": (C.c_int, [P, P, i64, i32, P, i32, f32, P, P, P, P]),
        "pano_refine": (C.c_int, [P, P, i64, i32, P, i32, f32, P, P, P]),
        "pano_audit_bounds": (C.c_int, [P, P, i64, P, P, i64, i32, P, P, P]),
        "pano_search_bruteforce": (C.c_int, [P, P, i64, i32, P, i32, P, P, P, u32, P]),
        "pano_index_info": (C.c_int, [P, P]),
        "pano_index_layout": (C.c_int, [P, P, P]),
        "pano_stats_get": (C.c_int, [P, P]),
        "pano_index_free": (None, [P]),
        "pano_shape_plan": (C.c_int, [P, i32, P, i32, C.c_double, P, i32, P]),
        "pano_transform_shape": (C.c_int, [P, P, i32, C.c_double, i32, u64, PP]),
        "pano_pq_build": (C.c_int, [P, P, P, i64, i32, P, P, i32, P, i32, i32, i32, i64, u64, PP, P]),
        "pano_pq_search": (C.c_int, [P, P, P, i64, i32, P, i32, f32, P, P, u32, P]),
        "pano_pq_stats": (C.c_int, [P, P, P]),
        "pano_pq_export": (C.c_int, [P, P, P, P, P]),
        "pano_pq_free": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(status: int):
    if status != PANO_OK:
        msg = lib().pano_last_error().decode(errors="replace")
        raise PanoError(status, msg)


def exported_symbols():
    return ["pano_last_error", "pano_version", "pano_ctx_create", "pano_ctx_destroy",
            "pano_ctx_scratch_bytes", "pano_ctx_trim", "pano_ctx_status",
            "pano_build_transform", "pano_transform_identity", "pano_transform_from",
            "pano_transform_get", "pano_transform_free", "pano_ivf_assign", "pano_build_levels",
            "pano_search", "pano_search_ctx", "pano_search_scratch_bytes", "pano_search_noalloc", "pano_refine", "pano_audit_bounds", "pano_search_bruteforce", "pano_index_info", "pano_index_layout",
            "pano_stats_get", "pano_index_free", "pano_shape_plan", "pano_transform_shape", "pano_pq_build",
            "pano_pq_search", "pano_pq_stats", "pano_pq_export", "pano_pq_free"]
