"""ctypes binding of libknng.so (include/knng.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  If the shared library has not been built this module raises
at import time -- there is no fallback.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# KNNG_LIB selects another build of the same ABI (the profiling build,
# libknng_counters.so, counts the search's steps)
LIB_PATH = os.environ.get("KNNG_LIB") or os.path.join(HERE, "libknng.so")

KNNG_OK, KNNG_EINVAL, KNNG_ECAPACITY, KNNG_ENOMEM, KNNG_EDEVICE, KNNG_ESTATE = 0, -1, -2, -3, -4, -5
KNNG_EUNSUPPORTED = -6
KNNG_NUM_STEP_COUNTERS = 13
STEP_COUNTERS = ["searches", "evaluations", "window_steps", "scan_steps", "window_cands",
                 "scan_cands", "window_visited", "scan_visited", "window_committed",
                 "scan_committed", "restarts_taken", "moves", "window_kept"]
KNNG_U8, KNNG_F32 = 0, 1
KNNG_SCORE_EXACT, KNNG_SCORE_BF16, KNNG_SCORE_FP8, KNNG_SCORE_BF16_MFMA = 0, 1, 2, 3
KNNG_METRIC_L2, KNNG_METRIC_COSINE, KNNG_METRIC_INNER_PRODUCT = 0, 1, 2

STATUS_NAMES = {0: "KNNG_OK", -1: "KNNG_EINVAL", -2: "KNNG_ECAPACITY", -3: "KNNG_ENOMEM",
                -4: "KNNG_EDEVICE", -5: "KNNG_ESTATE", -6: "KNNG_EUNSUPPORTED"}

EXPORTED = [
    "knng_storage_bytes", "knng_workspace_bytes", "knng_build_exact", "knng_load",
    "knng_search", "knng_insert_batch", "knng_query", "knng_get_lists", "knng_get_points",
    "knng_size", "knng_budget", "knng_query_count", "knng_last_error", "knng_destroy",
    "knng_timing_enable", "knng_timing_read", "knng_row_bytes", "knng_get_rows",
    "knng_epoch", "knng_search_gnns", "knng_partition_scratch_bytes", "knng_partition",
    "knng_search_partitioned_scratch_bytes", "knng_search_partitioned",
    "knng_search_partitioned_noalloc", "knng_insert_exact", "knng_step_counters",
]

STAGES = ["ingest", "exact", "search", "peers", "update", "merge", "query"]


class knng_params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("k", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("score", ctypes.c_int32),
        ("capacity", ctypes.c_int64),
        ("max_batch", ctypes.c_int64),
        ("speedup", ctypes.c_int32),
        ("expansion_num", ctypes.c_int32),
        ("expansion_den", ctypes.c_int32),
        ("depth", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("metric", ctypes.c_int32),
    ]


class KnngError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1602_06819_amd.build` "
            "(the k-nn graph library has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.knng_storage_bytes.argtypes = [P(knng_params)]
    lib.knng_storage_bytes.restype = ctypes.c_size_t
    lib.knng_workspace_bytes.argtypes = [P(knng_params)]
    lib.knng_workspace_bytes.restype = ctypes.c_size_t
    lib.knng_build_exact.argtypes = [P(knng_params), vp, i64, vp, ctypes.c_size_t, vp,
                                     ctypes.c_size_t, vp, P(vp)]
    lib.knng_build_exact.restype = ctypes.c_int
    lib.knng_load.argtypes = [P(knng_params), vp, i64, vp, vp, vp, ctypes.c_size_t, vp,
                              ctypes.c_size_t, vp, P(vp)]
    lib.knng_load.restype = ctypes.c_int
    lib.knng_search.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, i64, vp]
    lib.knng_search.restype = ctypes.c_int
    lib.knng_insert_batch.argtypes = [vp, vp, i64, P(i64), vp, vp, vp]
    lib.knng_insert_batch.restype = ctypes.c_int
    lib.knng_insert_exact.argtypes = [vp, vp, i64, P(i64), vp]
    lib.knng_insert_exact.restype = ctypes.c_int
    lib.knng_query.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
    lib.knng_query.restype = ctypes.c_int
    lib.knng_get_lists.argtypes = [vp, i64, i64, vp, vp, vp]
    lib.knng_get_lists.restype = ctypes.c_int
    lib.knng_get_points.argtypes = [vp, i64, i64, vp, vp]
    lib.knng_get_points.restype = ctypes.c_int
    lib.knng_size.argtypes = [vp]
    lib.knng_size.restype = i64
    lib.knng_budget.argtypes = [vp, i64]
    lib.knng_budget.restype = i64
    lib.knng_query_count.argtypes = [vp]
    lib.knng_query_count.restype = i64
    lib.knng_last_error.argtypes = []
    lib.knng_last_error.restype = ctypes.c_char_p
    lib.knng_destroy.argtypes = [vp]
    lib.knng_destroy.restype = None
    lib.knng_timing_enable.argtypes = [vp, ctypes.c_int]
    lib.knng_timing_enable.restype = ctypes.c_int
    lib.knng_timing_read.argtypes = [vp, P(ctypes.c_double), P(i64)]
    lib.knng_timing_read.restype = ctypes.c_int
    lib.knng_row_bytes.argtypes = [vp]
    lib.knng_row_bytes.restype = ctypes.c_int32
    lib.knng_get_rows.argtypes = [vp, i64, i64, vp, vp, vp]
    lib.knng_get_rows.restype = ctypes.c_int
    lib.knng_epoch.argtypes = [vp, vp, i64, vp, i64, vp, vp, vp, vp, P(i64), vp, vp, vp]
    lib.knng_epoch.restype = ctypes.c_int
    lib.knng_search_gnns.argtypes = [vp, vp, i64, vp, ctypes.c_int32, vp, vp, vp, vp, i64, vp]
    lib.knng_search_gnns.restype = ctypes.c_int
    lib.knng_partition_scratch_bytes.argtypes = [vp, ctypes.c_int32]
    lib.knng_partition_scratch_bytes.restype = ctypes.c_size_t
    lib.knng_partition.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_uint64, vp, ctypes.c_size_t, vp, vp,
                                   vp]
    lib.knng_partition.restype = ctypes.c_int
    lib.knng_search_partitioned_scratch_bytes.argtypes = [vp, i64, ctypes.c_int32]
    lib.knng_search_partitioned_scratch_bytes.restype = ctypes.c_size_t
    lib.knng_search_partitioned.argtypes = [vp, vp, i64, vp, vp, ctypes.c_int32, vp,
                                            ctypes.c_size_t, vp, vp, vp, vp]
    lib.knng_search_partitioned.restype = ctypes.c_int
    lib.knng_search_partitioned_noalloc.argtypes = [vp, vp, i64, vp, vp, ctypes.c_int32, vp, vp,
                                                    vp, vp]
    lib.knng_search_partitioned_noalloc.restype = ctypes.c_int
    lib.knng_step_counters.argtypes = [vp, P(ctypes.c_uint64), ctypes.c_int]
    lib.knng_step_counters.restype = ctypes.c_int
    return lib


lib = _load()


def check(status: int) -> None:
    if status != KNNG_OK:
        raise KnngError(status, lib.knng_last_error().decode())


def last_error() -> str:
    return lib.knng_last_error().decode()
