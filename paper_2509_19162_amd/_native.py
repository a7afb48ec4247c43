"""ctypes declarations of libcayleygrowth.so (include/cayleygrowth.h and
include/cayleygrowth_testing.h). Argument marshalling only.

The library is loaded from this package's directory. There is no fallback:
if it is missing, every call raises.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcayleygrowth.so")

CG_OK = 0
CG_TRUNCATED = 1
CG_PENDING = 2
CG_E_INVAL = -1
CG_E_NOMEM = -2
CG_E_DEVICE = -3
CG_E_UNSUPPORTED = -4
CG_E_BUSY = -5
CG_E_CANCELLED = -6
CG_E_TIMEOUT = -7

CG_KEEP_ALL_LAYERS = 0x1
CG_ALLOW_DIRECTED = 0x2
CG_START_STATE = 0x4
CG_PROFILE = 0x8
CG_PACKED_SORT = 0x10
CG_BITMASK = 0x20
CG_SMALL_JOB = 0x40
CG_BINARY_STATE = 0x80

CG_KSTAT_MAX = 8

u8p = ctypes.POINTER(ctypes.c_uint8)
u64p = ctypes.POINTER(ctypes.c_uint64)


class CgJob(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int),
        ("gens", u8p),
        ("n_gens", ctypes.c_int),
        ("max_layers", ctypes.c_int),
        ("max_frontier", ctypes.c_uint64),
        ("flags", ctypes.c_uint32),
        ("start", u8p),
        ("layers_out", u8p),
        ("layers_out_cap", ctypes.c_uint64),
    ]


class CgKstat(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 32),
        ("launches", ctypes.c_uint64),
        ("total_ms", ctypes.c_double),
        ("alg_bytes", ctypes.c_double),
        ("items", ctypes.c_double),
    ]


class CgResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("num_layers", ctypes.c_int),
        ("layer_sizes", u64p),
        ("states_expanded", ctypes.c_uint64),
        ("candidates", ctypes.c_uint64),
        ("t_submit", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
        ("device_ms", ctypes.c_double),
        ("n_kstats", ctypes.c_int),
        ("kstats", CgKstat * CG_KSTAT_MAX),
    ]


class CgBatchOpts(ctypes.Structure):
    _fields_ = [
        ("stream", ctypes.c_void_p),
        ("max_active", ctypes.c_int),
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("tune", ctypes.c_int),
    ]


class CgBatchInfo(ctypes.Structure):
    _fields_ = [
        ("calls", ctypes.c_uint64),
        ("graph_builds", ctypes.c_uint64),
        ("graph_launches", ctypes.c_uint64),
        ("tuned_classes", ctypes.c_int),
        ("heavy_split", ctypes.c_double),
        ("tune_file_entries", ctypes.c_int),
    ]


class CgQueueOpts(ctypes.Structure):
    _fields_ = [
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("max_active", ctypes.c_int),
        ("max_queued", ctypes.c_int),
        ("large_lanes", ctypes.c_int),
        ("device", ctypes.c_int),
        ("stream", ctypes.c_void_p),
    ]


class CgQueueStats(ctypes.Structure):
    _fields_ = [
        ("budget_bytes", ctypes.c_uint64),
        ("charged_bytes", ctypes.c_uint64),
        ("peak_charged_bytes", ctypes.c_uint64),
        ("held_bytes", ctypes.c_uint64),
        ("peak_held_bytes", ctypes.c_uint64),
        ("running", ctypes.c_int),
        ("queued", ctypes.c_int),
        ("completed", ctypes.c_uint64),
        ("cancelled", ctypes.c_uint64),
        ("failed", ctypes.c_uint64),
        ("over_bound", ctypes.c_uint64),
    ]


class CgMemoryStats(ctypes.Structure):
    _fields_ = [
        ("held_bytes", ctypes.c_uint64),
        ("peak_held_bytes", ctypes.c_uint64),
        ("arena_bytes", ctypes.c_uint64),
    ]


class CgGrowthStats(ctypes.Structure):
    _fields_ = [
        ("total", ctypes.c_uint64),
        ("diameter", ctypes.c_int),
        ("mode", ctypes.c_int),
        ("max_layer", ctypes.c_uint64),
        ("antipodes", ctypes.c_uint64),
        ("mean", ctypes.c_double),
        ("variance", ctypes.c_double),
        ("skewness", ctypes.c_double),
        ("kurtosis", ctypes.c_double),
        ("gauss_mu", ctypes.c_double),
        ("gauss_sigma", ctypes.c_double),
        ("gauss_tv", ctypes.c_double),
        ("gumbel_mu", ctypes.c_double),
        ("gumbel_beta", ctypes.c_double),
        ("gumbel_tv", ctypes.c_double),
        ("gumbel_min", ctypes.c_int),
        ("best_fit", ctypes.c_int),
    ]


# (name, restype, argtypes) of every exported entry point
SIGNATURES = [
    ("cg_growth", ctypes.c_int, [ctypes.c_int, u8p, ctypes.c_int, ctypes.c_int, u64p]),
    ("cg_growth_ex", ctypes.c_int, [ctypes.POINTER(CgJob), ctypes.POINTER(CgResult), ctypes.c_void_p]),
    ("cg_engine_create", ctypes.c_void_p, [ctypes.c_void_p]),
    ("cg_engine_run", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CgJob), ctypes.POINTER(CgResult)]),
    ("cg_engine_destroy", None, [ctypes.c_void_p]),
    ("cg_growth_batch", ctypes.c_int,
     [ctypes.c_int, ctypes.POINTER(CgJob), ctypes.POINTER(CgResult), ctypes.POINTER(CgBatchOpts)]),
    ("cg_batch_info", ctypes.c_int, [ctypes.POINTER(CgBatchInfo)]),
    ("cg_growth_batch_noalloc", ctypes.c_int,
     [ctypes.c_int, ctypes.POINTER(CgJob), ctypes.POINTER(CgResult), ctypes.c_void_p]),
    ("cg_queue_create", ctypes.c_void_p, [ctypes.POINTER(CgQueueOpts)]),
    ("cg_queue_submit", ctypes.c_int,
     [ctypes.c_void_p, ctypes.POINTER(CgJob), ctypes.POINTER(CgResult), u64p]),
    ("cg_queue_poll", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    ("cg_queue_wait", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64]),
    ("cg_queue_cancel", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    ("cg_queue_destroy", None, [ctypes.c_void_p]),
    ("cg_queue_stats", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CgQueueStats)]),
    ("cg_memory_stats", ctypes.c_int, [ctypes.POINTER(CgMemoryStats), ctypes.c_int]),
    ("cg_release_cached_memory", None, []),
    ("cg_set_workspace", ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t]),
    ("cg_growth_stats", ctypes.c_int, [u64p, ctypes.c_int, ctypes.POINTER(CgGrowthStats)]),
    ("cg_strerror", ctypes.c_char_p, [ctypes.c_int]),
    ("cg_last_error", ctypes.c_char_p, []),
    ("cg_test_pack", ctypes.c_int, [ctypes.c_int, u8p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]),
    ("cg_test_unpack", ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, u8p, ctypes.c_void_p]),
    ("cg_test_expand", ctypes.c_int,
     [ctypes.c_int, u8p, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]),
    ("cg_test_sort", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    ("cg_test_sort_below", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p]),
    ("cg_test_sort32", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    ("cg_test_dedup", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
      ctypes.c_uint64, ctypes.c_void_p, u64p, ctypes.c_void_p]),
    ("cg_test_rank", ctypes.c_int,
     [ctypes.c_int, u64p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint32), ctypes.c_int, ctypes.c_void_p]),
    ("cg_test_unrank", ctypes.c_int,
     [ctypes.c_int, ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint64, u64p, ctypes.c_int, ctypes.c_void_p]),
    ("cg_test_rank64", ctypes.c_int,
     [ctypes.c_int, u64p, ctypes.c_uint64, u64p, ctypes.c_int, ctypes.c_void_p]),
    ("cg_test_unrank64", ctypes.c_int,
     [ctypes.c_int, u64p, ctypes.c_uint64, u64p, ctypes.c_int, ctypes.c_void_p]),
    ("cg_test_host_expand", ctypes.c_int, [ctypes.c_int, u8p, ctypes.c_int, u64p, ctypes.c_uint64, u64p]),
    ("cg_test_host_expand_bits", ctypes.c_int, [ctypes.c_int, u8p, ctypes.c_int, u64p, ctypes.c_uint64, u64p]),
    ("cg_test_copy", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p]),
    ("cg_test_layer_step", ctypes.c_int,
     [ctypes.c_int, u8p, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
      ctypes.c_uint64, ctypes.c_void_p, u64p, ctypes.c_void_p]),
]

_lib = None


class NativeLibraryMissing(RuntimeError):
    pass


def lib():
    """The loaded library (raises NativeLibraryMissing if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise NativeLibraryMissing(
                f"{LIB_PATH} is missing: build it with `python -m paper_2509_19162_amd.build` "
                "(there is no CPU fallback)"
            )
        h = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib
