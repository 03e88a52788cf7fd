"""ctypes declarations of the C ABI in include/detlsh.h.

Loading fails loudly when libdetlsh.so is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdetlsh.so")

OK, EINVAL, ENOMEM, EBUSY, EDEVICE, ECANCELED, EINTERNAL = range(7)
FP32, BF16_RERANK = 0, 1
RMIN_MAGIC, RMIN_FIXED = 0, 1
PROJ_GAUSSIAN, PROJ_PAA = 0, 1

STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EBUSY", 4: "EDEVICE", 5: "ECANCELED", 6: "EINTERNAL"}


class BuildOpts(C.Structure):
    _fields_ = [
        ("seed", C.c_uint64),
        ("max_leaf", C.c_int32),
        ("keep_bf16", C.c_int32),
        ("proj_bf16", C.c_int32),
        ("projection", C.c_int32),
        ("A", C.POINTER(C.c_float)),
        ("sample_ids", C.POINTER(C.c_int64)),
        ("borrow_x", C.c_int32),
    ]


class QueryOpts(C.Structure):
    _fields_ = [
        ("precision", C.c_int32),
        ("rerank_mult", C.c_int32),
        ("rmin_policy", C.c_int32),
        ("max_rounds", C.c_int32),
        ("r_min", C.c_double),
        ("workspace_bytes", C.c_size_t),
        ("verify", C.c_int32),
        ("granularity", C.c_int32),
        ("filter", C.c_int32),
    ]


class Info(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("d", C.c_int32), ("L", C.c_int32), ("K", C.c_int32), ("N_r", C.c_int32),
        ("n_s", C.c_int64),
        ("max_leaf", C.c_int32),
        ("has_bf16", C.c_int32),
        ("n_leaves", C.c_int64 * 8),
        ("device_bytes", C.c_size_t),
    ]


class RequestInfo(C.Structure):
    _fields_ = [
        ("t_submit", C.c_double),
        ("t_start", C.c_double),
        ("t_end", C.c_double),
        ("batches", C.c_int32),
        ("max_batch_requests", C.c_int32),
        ("max_batch_queries", C.c_int64),
    ]


# name -> (restype, argtypes); every symbol here is declared in include/detlsh.h
P = C.c_void_p
SIGNATURES = {
    "detlsh_build_index": (C.c_int, [P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                     C.POINTER(BuildOpts), P, C.POINTER(P)]),
    "detlsh_index_import": (C.c_int, [P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P, P,
                                      C.POINTER(BuildOpts), P, C.POINTER(P)]),
    "detlsh_index_info": (C.c_int, [P, C.POINTER(Info)]),
    "detlsh_export": (C.c_int, [P, P, P, P, P]),
    "detlsh_export_tree": (C.c_int, [P, C.c_int32, P, P, P, P, C.c_int64]),
    "detlsh_project": (C.c_int, [P, P, C.c_int64, P, P]),
    "detlsh_query": (C.c_int, [P, P, C.c_int64, C.c_int32, C.c_double, C.c_double, C.POINTER(QueryOpts), P, P,
                               P]),
    "detlsh_query_async": (C.c_int, [P, P, C.c_int64, C.c_int32, C.c_double, C.c_double, C.POINTER(QueryOpts),
                                     P, P, P, P]),
    "detlsh_query_debug": (C.c_int, [P, P, P, C.c_int64, C.c_int32, C.c_double, C.c_double,
                                     C.POINTER(QueryOpts), P, C.c_int64, P, P, P, P, P, P, P, P]),
    "detlsh_query_noalloc": (C.c_int, [P, P, C.c_int64, C.c_int32, C.c_double, C.c_double, C.POINTER(QueryOpts),
                                       P, P, P]),
    "detlsh_noalloc_scratch_bytes": (C.c_size_t, []),
    "detlsh_query_rc": (C.c_int, [P, P, C.c_int64, C.c_double, C.c_double, C.c_double, C.POINTER(QueryOpts), P,
                                  P, P]),
    "detlsh_insert": (C.c_int, [P, P, C.c_int64, P]),
    "detlsh_index_save": (C.c_int, [P, C.c_char_p]),
    "detlsh_index_load": (C.c_int, [C.c_char_p, P, C.POINTER(P)]),
    "detlsh_profile_enable": (C.c_int, [C.c_int32, C.c_int32]),
    "detlsh_profile_counters": (C.c_int, [C.POINTER(C.c_char_p), C.POINTER(C.c_int64), C.c_int32,
                                          C.POINTER(C.c_int32)]),
    "detlsh_profile_read": (C.c_int, [C.POINTER(C.c_char_p), C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                      C.c_int32, C.POINTER(C.c_int32)]),
    "detlsh_server_create": (C.c_int, [P, C.c_size_t, C.c_int32, C.c_int32, C.POINTER(P)]),
    "detlsh_server_submit": (C.c_int, [P, P, C.c_int64, C.c_int32, C.c_double, C.c_double, C.POINTER(QueryOpts),
                                       P, P, C.POINTER(C.c_uint64)]),
    "detlsh_server_wait": (C.c_int, [P, C.c_uint64, C.c_int64, C.POINTER(RequestInfo)]),
    "detlsh_server_cancel": (C.c_int, [P, C.c_uint64]),
    "detlsh_server_destroy": (None, [P]),
    "detlsh_probe_valu": (C.c_int, [C.c_int32, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "detlsh_free": (None, [P]),
    "detlsh_trim": (None, []),
    "detlsh_last_error": (C.c_char_p, []),
}

_lib = None


class DetlshError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2406_10938_amd.build` first")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != OK:
        raise DetlshError(status, lib().detlsh_last_error().decode())
