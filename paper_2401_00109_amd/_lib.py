"""ctypes declarations for libjabba.so (include/jabba.h).

Argument marshalling only.  The library must have been built (``build()`` in
``__graft_entry__`` or ``python -m paper_2401_00109_amd.build``); if it is
missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_build", "libjabba.so")

JABBA_OK = 0
JABBA_EINVAL = -1
JABBA_ENOMEM = -2
JABBA_EHIP = -3
JABBA_ECAPACITY = -4
JABBA_ENONFINITE = -5
JABBA_EOVERFLOW = -6
JABBA_ENODEV = -7
JABBA_ELIMIT = -8
JABBA_ENCODE_NOALLOC_MAX_CAPACITY = 65536

EXPORTS = [
    "jabba_abi_version", "jabba_status_str", "jabba_compress_workspace", "jabba_compress", "jabba_compress_plain",
    "jabba_digitize_workspace", "jabba_digitize", "jabba_encode_workspace", "jabba_encode", "jabba_reconstruct_workspace",
    "jabba_reconstruct_size", "jabba_reconstruct", "jabba_reconstruct_pieces", "jabba_workspace_status",
    "jabba_plan_create", "jabba_plan_tuning", "jabba_plan_run", "jabba_plan_destroy", "jabba_fp64_selftest",
    "jabba_timing_enable", "jabba_timing_get", "jabba_timing_names", "jabba_digitize_stats",
    "jabba_digitize_quality", "jabba_kmeans_workspace", "jabba_kmeans", "jabba_digitize_pca",
    "jabba_axis_tolerances", "jabba_aggregate_points", "jabba_compress_znorm", "jabba_encode_noalloc",
    "jabba_reconstruct_mse",
]


class Tuning(C.Structure):
    _fields_ = [("lanes_per_domain", C.c_int32), ("waves_per_block", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("stage1_waves", C.c_int32), ("segment_intervals", C.c_int32), ("reserved", C.c_int32 * 3)]


class Dict(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("params", C.c_void_p), ("k", C.c_void_p), ("center_len", C.c_void_p),
                ("center_inc", C.c_void_p), ("cx", C.c_void_p), ("cy", C.c_void_p), ("count", C.c_void_p)]


class PlanDesc(C.Structure):
    _fields_ = [
        ("values", C.c_void_p), ("series_off", C.c_void_p), ("n_series", C.c_int64), ("total_points", C.c_int64),
        ("D", C.c_int32), ("tol", C.c_double), ("max_len", C.c_int32), ("alpha", C.c_double), ("scl", C.c_double),
        ("B", C.c_int32), ("max_pieces", C.c_int64),
        ("len", C.c_void_p), ("inc", C.c_void_p), ("piece_off", C.c_void_p), ("n_pieces", C.c_void_p),
        ("symbols", C.c_void_p), ("dict", Dict),
        ("compress_ws", C.c_void_p), ("compress_ws_bytes", C.c_size_t),
        ("digitize_ws", C.c_void_p), ("digitize_ws_bytes", C.c_size_t),
        ("tuning", C.POINTER(Tuning)),
    ]


class JabbaError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})")


_lock = threading.Lock()
_lib = None
P = C.c_void_p
I64 = C.c_int64
I32 = C.c_int32
D = C.c_double
SZ = C.c_size_t


def lib() -> C.CDLL:
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"libjabba.so not built at {LIB_PATH}; run __graft_entry__.build() or "
                                  "python -m paper_2401_00109_amd.build")
            L = C.CDLL(LIB_PATH)
            L.jabba_abi_version.restype = C.c_int
            L.jabba_abi_version.argtypes = []
            L.jabba_status_str.restype = C.c_char_p
            L.jabba_status_str.argtypes = [C.c_int]
            L.jabba_compress_workspace.argtypes = [I64, I64, I32, C.POINTER(SZ)]
            L.jabba_compress.argtypes = [P, P, I64, I64, I32, D, I32, C.POINTER(Tuning), P, P, P, P, P, SZ, P]
            L.jabba_compress_znorm.argtypes = [P, P, I64, I64, I32, D, I32, C.POINTER(Tuning), P, P, P, P, P, P, P,
                                               SZ, P]
            L.jabba_compress_plain.argtypes = [P, P, P, I64, I32, D, I32, P, P, P, P, P, SZ, P]
            L.jabba_digitize_workspace.argtypes = [I64, I32, C.POINTER(SZ)]
            L.jabba_digitize.argtypes = [P, P, P, I64, D, D, I32, C.POINTER(Tuning), P, C.POINTER(Dict), P, SZ, P]
            L.jabba_digitize_pca.argtypes = [P, P, P, I64, D, D, I32, C.POINTER(Tuning), P, C.POINTER(Dict), P, P,
                                             SZ, P]
            L.jabba_axis_tolerances.argtypes = [D, D, D, C.POINTER(D), C.POINTER(D)]
            L.jabba_aggregate_points.argtypes = [P, P, P, I64, D, I32, P, I64, P, P, P, P, P, P, SZ, P]
            L.jabba_encode_workspace.argtypes = [I64, C.POINTER(SZ)]
            L.jabba_encode.argtypes = [P, P, P, I64, C.POINTER(Dict), P, P, SZ, P]
            L.jabba_encode_noalloc.argtypes = [P, P, P, I64, C.POINTER(Dict), P, P]
            L.jabba_reconstruct_workspace.argtypes = [I64, C.POINTER(SZ)]
            L.jabba_reconstruct_size.argtypes = [P, P, P, I64, C.POINTER(Dict), P, P, SZ, P]
            L.jabba_reconstruct.argtypes = [P, P, P, I64, P, C.POINTER(Dict), P, P, P, P, P, P, P, SZ, P]
            L.jabba_reconstruct_mse.argtypes = [P, P, I64, P, P]
            L.jabba_reconstruct_pieces.argtypes = [P, P, P, P, I64, P, P, P, P, SZ, P]
            L.jabba_workspace_status.argtypes = [P, P, C.POINTER(C.c_int32)]
            L.jabba_plan_create.argtypes = [C.POINTER(PlanDesc), C.POINTER(P)]
            L.jabba_plan_tuning.argtypes = [P, C.POINTER(Tuning)]
            L.jabba_plan_run.argtypes = [P, P]
            L.jabba_plan_destroy.argtypes = [P]
            L.jabba_fp64_selftest.argtypes = [P, P, P, P, I64, P]
            L.jabba_digitize_stats.argtypes = [P, I64, I32, P, C.POINTER(I64)]
            L.jabba_digitize_quality.argtypes = [P, P, P, I64, D, I32, C.POINTER(Dict), P, P, P, P, SZ, P]
            L.jabba_kmeans_workspace.argtypes = [I64, I64, C.POINTER(SZ)]
            L.jabba_kmeans.argtypes = [P, P, P, I64, I32, C.POINTER(Dict), P, P, P, SZ, P]
            L.jabba_timing_enable.argtypes = [C.c_int]
            L.jabba_timing_get.argtypes = [C.c_char_p, C.POINTER(C.c_double), C.POINTER(I64)]
            L.jabba_timing_names.argtypes = [C.c_char_p, SZ]
            for name in EXPORTS:
                if name != "jabba_status_str":
                    getattr(L, name).restype = C.c_int
            _lib = L
    return _lib


def status_str(status: int) -> str:
    try:
        return lib().jabba_status_str(int(status)).decode()
    except ImportError:
        return "unknown"


def check(rc: int, what: str) -> None:
    if rc != JABBA_OK:
        raise JabbaError(rc, what)
