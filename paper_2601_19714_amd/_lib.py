"""ctypes declarations of the C ABI in include/wsimg.h (argument marshalling only)."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwsimg.so")

WSIMG_OK = 0
WSIMG_E_INVALID = -1
WSIMG_E_NOMEM = -2
WSIMG_E_HIP = -3
WSIMG_E_EMPTY = -4
WSIMG_E_CAPACITY = -5
WSIMG_E_UNSUPPORTED = -6
WSIMG_F32 = 1
WSIMG_F64 = 2
WSIMG_FIXED_WRANGE = 0x1
WSIMG_UNNORMALIZED = 0x2
WSIMG_FOLD_W = 0x4
WSIMG_PAD2 = 0x8
WSIMG_COMPLEX_OUT = 0x10
WSIMG_N_KERNELS = 8

# every symbol include/wsimg.h declares
EXPORTS = (
    "wsimg_plan_create", "wsimg_plan_create_batch", "wsimg_plan_destroy", "wsimg_plan_set_stream",
    "wsimg_plan_get_info", "wsimg_plan_query", "wsimg_image", "wsimg_image_batch", "wsimg_predict", "wsimg_grid", "wsimg_set_timing", "wsimg_read_timing", "wsimg_stage_name",
    "wsimg_status_string", "wsimg_last_error", "wsimg_version", "wsimg_image_noalloc",
)
WSIMG_NOALLOC_SCRATCH_BYTES = 64 << 20


class Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_wplanes", ctypes.c_int32), ("support", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("pixel_rad", ctypes.c_double), ("beta", ctypes.c_double),
                ("w_lo", ctypes.c_double), ("w_hi", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("w_support", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int64), ("n_gridded", ctypes.c_int64), ("n_dropped", ctypes.c_int64),
                ("sum_w", ctypes.c_double), ("w_lo", ctypes.c_double), ("w_hi", ctypes.c_double),
                ("n_strips_occupied", ctypes.c_int64), ("n_planes_occupied", ctypes.c_int64)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_wplanes", ctypes.c_int32), ("support", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("strip_rows", ctypes.c_int32), ("col_block", ctypes.c_int32),
                ("n_buckets", ctypes.c_int64), ("max_vis", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("max_channels", ctypes.c_int64), ("n_grid", ctypes.c_int64),
                ("grid_threads", ctypes.c_int32), ("stack_threads", ctypes.c_int32),
                ("stack_cols", ctypes.c_int32), ("stack_radix", ctypes.c_int32),
                ("lds_grid_bytes", ctypes.c_int64), ("lds_stack_bytes", ctypes.c_int64),
                ("record_bytes", ctypes.c_int64), ("row_capacity", ctypes.c_int64),
                ("list_capacity", ctypes.c_int64)]


class Timing(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_int64), ("ms", ctypes.c_double * WSIMG_N_KERNELS),
                ("ms_total", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libwsimg.so; raises ImportError (never falls back) when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2601_19714_amd.build.build()")
    # torch first: its HIP runtime is then the one the library binds to (device memory and
    # streams come from torch; two runtimes in one process do not share devices)
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.wsimg_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Params), i64, vp]
    L.wsimg_plan_create_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Params), i64, i32, vp]
    L.wsimg_plan_destroy.argtypes = [vp]
    L.wsimg_plan_set_stream.argtypes = [vp, vp]
    L.wsimg_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    L.wsimg_plan_query.argtypes = [ctypes.POINTER(Params), i64, i32, ctypes.POINTER(PlanInfo)]
    for f in (L.wsimg_image, L.wsimg_grid):
        f.argtypes = [vp, i64, vp, vp, vp, dbl, vp, ctypes.POINTER(Stats)]
    L.wsimg_image_batch.argtypes = [vp, i32, ctypes.POINTER(i64), vp, vp, vp, ctypes.POINTER(dbl), vp,
                                    ctypes.POINTER(Stats)]
    L.wsimg_predict.argtypes = [vp, i64, vp, vp, dbl, vp, vp, ctypes.POINTER(Stats)]
    L.wsimg_image_noalloc.argtypes = [ctypes.POINTER(Params), i64, vp, vp, vp, dbl, vp, vp, ctypes.POINTER(Stats)]
    L.wsimg_set_timing.argtypes = [vp, i32]
    L.wsimg_read_timing.argtypes = [vp, ctypes.POINTER(Timing)]
    for f in (L.wsimg_plan_create, L.wsimg_plan_create_batch, L.wsimg_plan_destroy, L.wsimg_plan_set_stream,
              L.wsimg_plan_get_info, L.wsimg_plan_query, L.wsimg_image, L.wsimg_image_batch, L.wsimg_predict, L.wsimg_grid,
              L.wsimg_set_timing, L.wsimg_image_noalloc,
              L.wsimg_read_timing):
        f.restype = ctypes.c_int
    L.wsimg_stage_name.argtypes = [i32]
    L.wsimg_stage_name.restype = ctypes.c_char_p
    L.wsimg_status_string.argtypes = [ctypes.c_int]
    L.wsimg_status_string.restype = ctypes.c_char_p
    L.wsimg_last_error.argtypes = []
    L.wsimg_last_error.restype = ctypes.c_char_p
    L.wsimg_version.argtypes = []
    L.wsimg_version.restype = i32
    _lib = L
    return L
