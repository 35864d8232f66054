"""ctypes declarations of the C ABI in include/pk.h (libpk.so, built in-tree)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpk.so")

c_i64 = ctypes.c_int64
c_i32 = ctypes.c_int32
c_f32 = ctypes.c_float
c_vp = ctypes.c_void_p
c_sz = ctypes.c_size_t
c_st = ctypes.c_int   # pk_status

# (name, restype, argtypes) for every exported entry point
SIGNATURES = [
    ("pk_status_string", ctypes.c_char_p, [c_st]),
    ("pk_last_error", ctypes.c_char_p, []),
    ("pk_abi_version", ctypes.c_int, []),
    ("pk_context_create", c_st, [ctypes.c_int, ctypes.POINTER(c_vp)]),
    ("pk_context_destroy", None, [c_vp]),
    ("pk_context_set_checks", c_st, [c_vp, ctypes.c_int]),
    ("pk_workspace_bytes", c_st, [ctypes.c_int, ctypes.POINTER(c_i64), ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(c_sz)]),
    ("pk_sgemm", c_st, [c_vp, ctypes.c_int, c_i64, c_i64, c_i64, c_f32, c_vp, c_i64, c_vp, c_i64,
                        c_f32, c_vp, c_i64, c_vp]),
    ("pk_sgemm_ws", c_st, [c_vp, ctypes.c_int, c_i64, c_i64, c_i64, c_f32, c_vp, c_i64, c_vp, c_i64,
                           c_f32, c_vp, c_i64, c_vp, c_sz, c_vp]),
    ("pk_sgemm3", c_st, [c_vp, ctypes.c_int, c_i64, c_i64, c_i64, c_i64, c_f32, c_vp, c_i64, c_vp,
                         c_i64, c_vp, c_i64, c_f32, c_vp, c_i64, c_vp, c_sz, c_vp]),
    ("pk_sgemv", c_st, [c_vp, c_i64, c_i64, c_vp, c_i64, c_vp, c_vp, c_vp]),
    ("pk_sgemv_t", c_st, [c_vp, c_i64, c_i64, c_vp, c_i64, c_vp, c_vp, c_vp, c_sz, c_vp]),
    ("pk_sgemv_pair", c_st, [c_vp, c_i64, c_i64, c_vp, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz,
                             c_vp]),
    ("pk_conv2d_3x3", c_st, [c_vp, c_i64, c_i64, ctypes.POINTER(c_f32), c_vp, c_i64, c_vp, c_i64,
                             c_vp]),
    ("pk_conv3d_3x3x3", c_st, [c_vp, c_i64, c_i64, c_i64, ctypes.POINTER(c_f32), c_vp, c_vp, c_vp]),
    ("pk_colstats", c_st, [c_vp, c_i64, c_i64, c_vp, c_i64, c_f32, c_vp, c_vp, c_vp, c_sz, c_vp]),
    ("pk_corr", c_st, [c_vp, ctypes.c_int, c_i64, c_i64, c_vp, c_i64, c_f32, c_vp, c_vp, c_vp, c_i64,
                       c_vp, c_sz, c_vp]),
    ("pk_corr_noalloc", c_st, [c_vp, ctypes.c_int, c_i64, c_i64, c_vp, c_i64, c_f32, c_vp, c_vp, c_vp, c_i64,
                               c_vp]),
    ("pk_convert_bf16", c_st, [c_vp, c_i64, c_vp, c_vp, c_vp, c_vp]),
    ("pk_covar", c_st, [c_vp, ctypes.c_int, c_i64, c_i64, c_vp, c_i64, c_vp, c_vp, c_i64, c_vp, c_sz, c_vp]),
    ("pk_ssyrk", c_st, [c_vp, c_i64, c_i64, c_f32, c_vp, c_i64, c_f32, c_vp, c_i64, c_vp]),
    ("pk_ssyr2k", c_st, [c_vp, c_i64, c_i64, c_f32, c_vp, c_i64, c_vp, c_i64, c_f32, c_vp, c_i64, c_vp]),
    ("pk_sgesummv", c_st, [c_vp, c_i64, c_f32, c_vp, c_i64, c_f32, c_vp, c_i64, c_vp, c_vp, c_vp]),
    ("pk_smvt", c_st, [c_vp, c_i64, c_vp, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    ("pk_fdtd2d", c_st, [c_vp, c_i64, c_i64, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp]),
    ("pk_variant_load", c_st, [c_vp, ctypes.c_char_p, c_sz, ctypes.POINTER(c_i32)]),
    ("pk_variant_unload", c_st, [c_vp, c_i32]),
    ("pk_variant_info", c_st, [c_vp, c_i32, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32),
                               ctypes.POINTER(ctypes.c_uint64)]),
    ("pk_variant_default", c_st, [c_vp, c_i32, ctypes.POINTER(c_i32)]),
    ("pk_variant_select", c_st, [c_vp, c_i32, c_i32]),
    ("pk_variant_set_best", c_st, [c_vp, c_i32, c_i32, c_i32]),
    ("pk_size_bucket", c_i32, [c_i64]),
    ("pk_graph_begin", c_st, [c_vp, c_vp]),
    ("pk_graph_end", c_st, [c_vp, c_vp, ctypes.POINTER(c_vp)]),
    ("pk_graph_launch", c_st, [c_vp, c_vp]),
    ("pk_graph_destroy", None, [c_vp]),
    ("pk_timer_start", c_st, [c_vp, c_vp]),
    ("pk_timer_stop", c_st, [c_vp, c_vp, ctypes.POINTER(ctypes.c_double)]),
    ("pk_graph_time", c_st, [c_vp, c_vp, ctypes.c_int, c_vp, ctypes.POINTER(ctypes.c_double)]),
    ("pk_cache_flush", c_st, [c_vp, c_vp]),
    ("pk_stream_probe", c_st, [c_vp, ctypes.c_int, c_vp, c_vp, c_i64, c_vp]),
]

_lib = None


def load():
    """Load libpk.so; raises (never falls back) if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first "
                          "(python -m paper_1810_10496_amd.build or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
