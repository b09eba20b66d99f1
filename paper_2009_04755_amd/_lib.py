"""ctypes view of ``librocket.so`` (the C ABI declared in ``include/rocket.h``).

Argument marshalling only: every step of the all-pairs path runs in the HIP
library.  Loading fails loudly when the library has not been built; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librocket.so")

OK = 0
E_INVALID, E_UNSUPPORTED, E_OOM, E_HIP, E_KEYRANGE, E_UNSORTED, E_STATE = -1, -2, -3, -4, -5, -6, -7

NCC_FP32, NCC_BF16X3, NCC_BF16X6, GAUSS_OVERLAP, SPARSE_COSINE, GMM_L2, GMM_BHATTACHARYA, PCE = 1, 2, 3, 4, 5, 6, 7, 8
FN_BY_NAME = {"ncc_fp32": NCC_FP32, "ncc_bf16x3": NCC_BF16X3, "ncc_bf16x6": NCC_BF16X6,
              "gauss_overlap": GAUSS_OVERLAP, "sparse_cosine": SPARSE_COSINE, "gmm_l2": GMM_L2,
              "gmm_bhattacharya": GMM_BHATTACHARYA, "pce": PCE}

OPT = {"ncc_tile": 1, "ncc_kchunk": 2, "grid": 3, "queue_order": 4, "seed": 5, "ledger": 6, "ovl_block": 7,
       "ovl_variant": 8, "sp_lanes": 9, "sp_chunk": 10, "workspace_cap": 11, "autotune": 12, "timing": 13,
       "cache_slots": 14, "pce_radius": 15, "ncc_waves": 16, "pce_width": 17, "pce_batch": 18,
       "trace": 19}

# every symbol include/rocket.h declares
SYMBOLS = ["rocket_create", "rocket_destroy", "rocket_status_str", "rocket_last_error", "rocket_prepare",
           "rocket_compare", "rocket_allpairs_ex", "rocket_allpairs", "rocket_allpairs_host", "rocket_cv_build",
           "rocket_overlap_cost_grad",
           "rocket_set_option", "rocket_get_option", "rocket_get_stats", "rocket_get_ledger", "rocket_autotune",
           "rocket_plan_tiles", "rocket_pair_index", "rocket_allpairs_noalloc", "rocket_cost_grad",
           "rocket_set_tune_cache", "rocket_probe_valu", "rocket_get_trace"]
NOALLOC_SCRATCH_BYTES = 64 << 20  # ROCKET_NOALLOC_SCRATCH_BYTES


class TraceRec(ctypes.Structure):
    _fields_ = [("tile_i", ctypes.c_int32), ("tile_j", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("workgroup", ctypes.c_int32), ("start_ns", ctypes.c_int64), ("end_ns", ctypes.c_int64)]


class Items(ctypes.Structure):
    _fields_ = [("dense", ctypes.c_void_p), ("dim", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("xy", ctypes.c_void_p), ("sigma", ctypes.c_double),
                ("keys", ctypes.c_void_p), ("vals", ctypes.c_void_p), ("point_sigma", ctypes.c_void_p),
                ("point_cov", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in
                ("n", "pairs", "tiles", "work_items", "grid", "tile", "kchunk", "workspace_bytes", "variant",
                 "kernel_ns", "cache_slots", "cache_loads", "tune_us", "tune_cached")]


class RocketError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(message)
        self.status = status


_lib = None


def load():
    """The loaded library; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("librocket.so is not built (run __graft_entry__.build() or "
                           "python -m paper_2009_04755_amd.build); there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    PP = ctypes.POINTER(ctypes.c_void_p)
    IT = ctypes.POINTER(Items)
    L.rocket_create.argtypes = [PP, I32]
    L.rocket_create.restype = I32
    L.rocket_destroy.argtypes = [P]
    L.rocket_destroy.restype = None
    L.rocket_status_str.argtypes = [I32]
    L.rocket_status_str.restype = ctypes.c_char_p
    L.rocket_last_error.argtypes = [P]
    L.rocket_last_error.restype = ctypes.c_char_p
    L.rocket_prepare.argtypes = [P, IT, I64, I32, P]
    L.rocket_prepare.restype = I32
    L.rocket_compare.argtypes = [P, P, P, P]
    L.rocket_compare.restype = I32
    L.rocket_allpairs_ex.argtypes = [P, IT, I64, I32, P, P, P]
    L.rocket_allpairs_ex.restype = I32
    L.rocket_allpairs.argtypes = [IT, I64, I32, P]
    L.rocket_allpairs.restype = I32
    L.rocket_allpairs_noalloc.argtypes = [IT, I64, I32, P, P, P]
    L.rocket_allpairs_noalloc.restype = I32
    L.rocket_allpairs_host.argtypes = [P, P, I64, I64, I64, I32, P, P]
    L.rocket_allpairs_host.restype = I32
    L.rocket_cv_build.argtypes = [P, P, P, I64, I32, P, P, P, I64, P]
    L.rocket_cv_build.restype = I32
    L.rocket_overlap_cost_grad.argtypes = [P, IT, I64, P, P, P, P, P]
    L.rocket_overlap_cost_grad.restype = I32
    L.rocket_cost_grad.argtypes = [P, IT, I64, I32, P, P, P, P, P]
    L.rocket_cost_grad.restype = I32
    L.rocket_get_trace.argtypes = [P, P, I64, ctypes.POINTER(I64)]
    L.rocket_get_trace.restype = I32
    L.rocket_probe_valu.argtypes = [I32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
    L.rocket_probe_valu.restype = I32
    L.rocket_set_option.argtypes = [P, I32, I64]
    L.rocket_set_option.restype = I32
    L.rocket_get_option.argtypes = [P, I32, ctypes.POINTER(I64)]
    L.rocket_get_option.restype = I32
    L.rocket_get_stats.argtypes = [P, ctypes.POINTER(Stats)]
    L.rocket_get_stats.restype = I32
    L.rocket_get_ledger.argtypes = [P, P, I64, ctypes.POINTER(I64)]
    L.rocket_get_ledger.restype = I32
    L.rocket_autotune.argtypes = [P, P]
    L.rocket_autotune.restype = I32
    L.rocket_set_tune_cache.argtypes = [P, ctypes.c_char_p]
    L.rocket_set_tune_cache.restype = I32
    L.rocket_plan_tiles.argtypes = [I64, I64, P, P, I64]
    L.rocket_plan_tiles.restype = I64
    L.rocket_pair_index.argtypes = [I64, I64, I64]
    L.rocket_pair_index.restype = I64
    _lib = L
    return L


def check(status: int, ctx=None):
    if status != OK:
        L = load()
        msg = L.rocket_last_error(ctx).decode() if ctx is not None else L.rocket_last_error(None).decode()
        raise RocketError(status, msg or L.rocket_status_str(status).decode())
