"""ctypes declarations for libconvhull.so (include/convhull.h).

Argument marshalling only: every step of the hull path runs in the HIP
library. Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libconvhull.so")

CH_OK = 0
CH_E_INVALID_ARG = 1
CH_E_DOMAIN = 2
CH_E_CAPACITY = 3
CH_E_NOMEM = 4
CH_E_DEVICE = 5
CH_E_BUSY = 6
CH_E_TIMEOUT = 7
CH_E_CANCELLED = 8
CH_E_SHUTDOWN = 9
CH_E_NOT_FOUND = 10
CH_COUNT_DOMAIN_ERROR = 0xFFFFFFFF
CH_COUNT_INVALID = 0xFFFFFFFD
CH_MAX_POINTS = 0x7FFFFFFF
CH_FILTER_NOALLOC_MAX_POINTS = 1 << 22
CH_EXTREMES_FUSED = 0
CH_EXTREMES_TWO_KERNELS = 1

STATUS_NAMES = {
    0: "CH_OK", 1: "CH_E_INVALID_ARG", 2: "CH_E_DOMAIN", 3: "CH_E_CAPACITY", 4: "CH_E_NOMEM",
    5: "CH_E_DEVICE", 6: "CH_E_BUSY", 7: "CH_E_TIMEOUT", 8: "CH_E_CANCELLED",
    9: "CH_E_SHUTDOWN", 10: "CH_E_NOT_FOUND",
}


class Octagon(ctypes.Structure):
    _fields_ = [("kx", ctypes.c_int32 * 8), ("ky", ctypes.c_int32 * 8), ("idx", ctypes.c_uint32 * 8)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double)]


class BatchParams(ctypes.Structure):
    _fields_ = [("tile_points", ctypes.c_uint32), ("pass_blocks", ctypes.c_uint32),
                ("hull_blocks", ctypes.c_uint32), ("sample_min", ctypes.c_uint32)]


class HullInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("candidates", ctypes.c_uint32), ("survivors", ctypes.c_uint32),
                ("rounds", ctypes.c_uint32), ("large_path", ctypes.c_uint32), ("h", ctypes.c_uint32),
                ("single_read", ctypes.c_uint32), ("refined", ctypes.c_uint32)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("d_arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t),
                ("max_inflight", ctypes.c_uint32), ("n_streams", ctypes.c_int),
                ("max_batch_points", ctypes.c_uint64)]


# (name, restype, argtypes) for every entry point declared in include/convhull.h.
P = ctypes.c_void_p
U32 = ctypes.c_uint32
U64 = ctypes.c_uint64
I32 = ctypes.c_int
SZ = ctypes.c_size_t
SIGNATURES = {
    "ch_ctx_create": (I32, [I32, ctypes.c_char_p, ctypes.POINTER(P)]),
    "ch_ctx_destroy": (None, [P]),
    "ch_status_string": (ctypes.c_char_p, [I32]),
    "ch_last_error": (ctypes.c_char_p, [P]),
    "ch_filter_workspace_bytes": (SZ, [U32]),
    "ch_hull_workspace_bytes": (SZ, [U32]),
    "ch_filter": (I32, [P, P, U32, P, P, P, P, P, SZ, P]),
    "ch_filter_noalloc_scratch_bytes": (SZ, []),
    "ch_filter_noalloc": (I32, [P, P, U32, P, P, P, P, P]),
    "ch_hull": (I32, [P, P, U32, P, U32, ctypes.POINTER(U32), P, SZ, P]),
    "ch_gpufilter_workspace_bytes": (SZ, [U32]),
    "ch_hull_queues_workspace_bytes": (SZ, [U32]),
    "ch_gpufilter": (I32, [P, P, U32, I32, P, P, P, P, SZ, P]),
    "ch_hull_queues": (I32, [P, P, U32, I32, P, U32, ctypes.POINTER(U32), P, P, SZ, P]),
    "ch_diag_read_stream": (I32, [P, P, SZ, U32, P]),
    "ch_last_hull_info": (I32, [P, ctypes.POINTER(HullInfo)]),
    "ch_hull_batch_workspace_bytes": (SZ, [U32, U64]),
    "ch_hull_batch": (I32, [P, P, P, U32, U64, P, P, P, SZ, P]),
    "ch_batch_params_get": (I32, [P, U32, U64, ctypes.POINTER(BatchParams)]),
    "ch_batch_params_set": (I32, [P, ctypes.POINTER(BatchParams)]),
    "ch_tune_batch": (I32, [P, P, P, U32, U64, P, P, P, SZ, P, ctypes.POINTER(BatchParams)]),
    "ch_serve_max_request_points": (U64, [ctypes.POINTER(ServeConfig)]),
    "ch_serve_start": (I32, [P, ctypes.POINTER(ServeConfig), ctypes.POINTER(P)]),
    "ch_serve_submit": (I32, [P, P, U32, ctypes.POINTER(U64)]),
    "ch_serve_wait": (I32, [P, U64, ctypes.c_int64, P, U32, ctypes.POINTER(U32), P]),
    "ch_serve_stats": (I32, [P, ctypes.POINTER(U64), ctypes.POINTER(U64), ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "ch_serve_stop": (I32, [P]),
    "ch_profile_enable": (I32, [P, I32]),
    "ch_profile_reset": (I32, [P]),
    "ch_profile_read": (I32, [P, P, I32, ctypes.POINTER(I32)]),
}

_lib = None


class LibraryMissing(RuntimeError):
    pass


def load():
    """Load libconvhull.so (raises LibraryMissing if it was never built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
