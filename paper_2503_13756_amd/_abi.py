"""ctypes declarations of libswalign's C ABI (include/swalign.h).

Argument marshalling only: every computation runs in the HIP kernels of the
library.  Loading fails loudly when the library has not been built."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswalign.so")

SW_OK, SW_NOT_READY, SW_E_INVALID, SW_E_NOMEM, SW_E_DEVICE, SW_E_UNSUPPORTED, SW_E_BUSY = (
    0, 1, -1, -2, -3, -4, -5)
LEVELS_MIDPOINT, LEVELS_LEFT = 0, 1
MODE_ROT_TRANS, MODE_ROT_ONLY, MODE_MAX_SLICED = 0, 1, 2
PREC_FP32, PREC_BF16_SPLIT = 0, 1
FILTER_NONE, FILTER_RAMP = 0, 1
RESULT_OK, RESULT_ZERO_MASS, RESULT_NONFINITE = 0, 1, 2

STATUS_NAMES = {0: "SW_OK", 1: "SW_NOT_READY", -1: "SW_E_INVALID", -2: "SW_E_NOMEM",
                -3: "SW_E_DEVICE", -4: "SW_E_UNSUPPORTED", -5: "SW_E_BUSY"}


class sw_geom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("n_angles", ctypes.c_int32),
                ("n_quantiles", ctypes.c_int32), ("levels", ctypes.c_int32)]


class sw_result(ctypes.Structure):
    _fields_ = [("rot_index", ctypes.c_int32), ("theta_rad", ctypes.c_float),
                ("shift_px", ctypes.c_float * 2), ("sw2sq", ctypes.c_float),
                ("status", ctypes.c_int32)]


class sw_batch(ctypes.Structure):
    _fields_ = [("ref_qt", ctypes.c_void_p), ("ref_aux", ctypes.c_void_p),
                ("n_ref", ctypes.c_int64), ("img_qt", ctypes.c_void_p),
                ("img_aux", ctypes.c_void_p), ("n_img", ctypes.c_int64),
                ("pairs", ctypes.c_void_p), ("n_pairs", ctypes.c_int64),
                ("geom", sw_geom), ("mode", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("top_k", ctypes.c_int32), ("filter", ctypes.c_int32)]


class sw_stack(ctypes.Structure):
    _fields_ = [("ref_img", ctypes.c_void_p), ("imgs", ctypes.c_void_p), ("N", ctypes.c_int64),
                ("geom", sw_geom), ("ref_qt", ctypes.c_void_p), ("ref_aux", ctypes.c_void_p),
                ("qt", ctypes.c_void_p), ("aux", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class sw_serve_cfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("top_k", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("max_queue", ctypes.c_int32), ("use_graphs", ctypes.c_int32),
                ("max_per_step", ctypes.c_int32)]


class sw_request(ctypes.Structure):
    _fields_ = [("ref_img", ctypes.c_void_p), ("imgs", ctypes.c_void_p), ("N", ctypes.c_int64),
                ("geom", sw_geom), ("ref_key", ctypes.c_uint64)]


class sw_serve_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("submitted", "admitted", "completed", "cancelled",
                                               "failed", "steps", "graph_launches", "cache_hits",
                                               "evictions")] + \
               [("pending", ctypes.c_int64), ("in_flight", ctypes.c_int64),
                ("arena_used", ctypes.c_size_t), ("arena_peak", ctypes.c_size_t),
                ("arena_size", ctypes.c_size_t), ("waited_memory", ctypes.c_uint64),
                ("waited_slot", ctypes.c_uint64)]


class SwError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# (name, restype, argtypes) of every exported entry point
P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
SIGNATURES = [
    ("sw_ctx_create", I32, [ctypes.POINTER(ctypes.c_void_p), I32, ctypes.c_char_p]),
    ("sw_ctx_destroy", I32, [P]),
    ("sw_last_error", ctypes.c_char_p, []),
    ("sw_version", ctypes.c_char_p, []),
    ("sw_projection_plan", I32, [I32, I32, I32, P, P, P, ctypes.POINTER(ctypes.c_int32)]),
    ("sw_project", I32, [P, P, I64, ctypes.POINTER(sw_geom), P, P]),
    ("sw_quantiles", I32, [P, P, I64, ctypes.POINTER(sw_geom), P, P, P]),
    ("sw_tables", I32, [P, P, I64, ctypes.POINTER(sw_geom), P, P, P]),
    ("sw_ramp", I32, [P, P, I64, ctypes.POINTER(sw_geom), P, P]),
    ("sw_quantiles_rf", I32, [P, P, I64, ctypes.POINTER(sw_geom), P, P, P]),
    ("sw_tables_rf", I32, [P, P, I64, ctypes.POINTER(sw_geom), P, P, P]),
    ("sw_project_fourier", I32, [P, P, I64, ctypes.POINTER(sw_geom), P, P]),
    ("sw_tables_fourier", I32, [P, P, I64, ctypes.POINTER(sw_geom), P, P, P]),
    ("sw_project_fourier_at", I32, [P, P, I64, ctypes.POINTER(sw_geom), P, P, P]),
    ("sw_tables_fourier_at", I32, [P, P, I64, ctypes.POINTER(sw_geom), P, P, P, P]),
    ("sw_align_batch", I32, [P, ctypes.POINTER(sw_batch), P, P, P]),
    ("sw_align_batch_noalloc", I32, [P, ctypes.POINTER(sw_batch), P, P, P]),
    ("sw_align_stacks", I32, [P, ctypes.POINTER(sw_stack), I32, I32, I32, I32, P]),
    ("sw_autotune", I32, [P, ctypes.POINTER(ctypes.c_int32), I32, I64, ctypes.c_char_p]),
    ("sw_serve_start", I32, [P, ctypes.POINTER(sw_serve_cfg)]),
    ("sw_serve_submit", I32, [P, ctypes.POINTER(sw_request), ctypes.POINTER(ctypes.c_uint64)]),
    ("sw_serve_poll", I32, [P, ctypes.c_uint64, P]),
    ("sw_serve_cancel", I32, [P, ctypes.c_uint64]),
    ("sw_serve_stats_get", I32, [P, ctypes.POINTER(sw_serve_stats)]),
    ("sw_serve_stop", I32, [P]),
]

_lib = None


def load():
    """Load libswalign.so (built in-tree by paper_2503_13756_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2503_13756_amd.build` "
                "(there is no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def check(status):
    if status != SW_OK:
        raise SwError(status, load().sw_last_error().decode(errors="replace"))
    return status
