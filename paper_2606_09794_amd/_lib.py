"""ctypes binding of libnasg.so (argument marshalling only).

The structures mirror ``include/nasg.h`` field for field. Loading fails loudly
when the library has not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnasg.so")

NASG_OK = 0
NASG_F32, NASG_BF16 = 0, 1
NORM_EXACT, NORM_APPROX = 0, 1
GRAD_OVERWRITE, GRAD_ACCUMULATE = 0, 1
PARAM_QUAT, PARAM_ANGLES = 0, 1
FAMILIES = {"nasgabor": 0, "nasg": 1, "sg": 2, "sb": 3, "sc": 4, "asg": 5}
KERNEL_NASG_FWD, KERNEL_NASG_BWD, KERNEL_SH_FWD, KERNEL_SH_BWD = 0, 1, 2, 3
STREAM_READ, STREAM_WRITE, STREAM_COPY = 0, 1, 2
NOALLOC_SCRATCH_BYTES = 64 << 20
KNN_MAX_K, KNN_MAX_CAMERAS = 32, 1 << 16


class NasgParams(C.Structure):
    _fields_ = [("quat", C.c_void_p), ("shape", C.c_void_p), ("rgbw", C.c_void_p),
                ("c0", C.c_void_p), ("n", C.c_int64), ("k", C.c_int32), ("dtype", C.c_int32),
                ("param", C.c_int32), ("family", C.c_int32)]


class NasgViews(C.Structure):
    _fields_ = [("means", C.c_void_p), ("cams", C.c_void_p), ("dirs", C.c_void_p),
                ("v", C.c_int32)]


class NasgGrads(C.Structure):
    _fields_ = [("quat", C.c_void_p), ("shape", C.c_void_p), ("rgbw", C.c_void_p),
                ("c0", C.c_void_p), ("geom", C.c_void_p)]


class NasgScene(C.Structure):
    _fields_ = [("p", NasgParams), ("views", NasgViews), ("grad_rgb", C.c_void_p),
                ("g", NasgGrads), ("rgb", C.c_void_p)]


class NasgBatchTuning(C.Structure):
    _fields_ = [("tile_iters", C.c_int32), ("blocks_per_cu", C.c_int32)]


class NasgBatch(C.Structure):
    _fields_ = [("workspace", C.c_void_p), ("bytes", C.c_size_t), ("n_items", C.c_int32),
                ("n_scenes", C.c_int32), ("grid", C.c_int32), ("norm", C.c_int32),
                ("token", C.c_uint64), ("raw", C.c_int32), ("pad", C.c_int32)]


class NasgTuning(C.Structure):
    _fields_ = [("lanes", C.c_int32), ("views_per_lane", C.c_int32), ("block", C.c_int32),
                ("bcast", C.c_int32)]


class NasgCamera(C.Structure):
    _fields_ = [("rot", C.c_double * 9), ("t", C.c_double * 3), ("fx", C.c_double),
                ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32)]


class NasgGaussians(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("rots", C.c_void_p),
                ("opac", C.c_void_p), ("colors", C.c_void_p), ("n", C.c_int64)]


EXPORTS = {
    "nasg_eval_fwd": (C.c_int, [C.POINTER(NasgParams), C.POINTER(NasgViews), C.c_void_p,
                                C.c_int32, C.c_void_p]),
    "nasg_eval_bwd": (C.c_int, [C.POINTER(NasgParams), C.POINTER(NasgViews), C.c_void_p,
                                C.POINTER(NasgGrads), C.c_void_p, C.c_int32, C.c_int32,
                                C.c_void_p]),
    "sh3_eval_fwd": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(NasgViews), C.c_void_p,
                               C.c_void_p]),
    "sh3_eval_bwd": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(NasgViews), C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "nasg_batched_workspace_bytes": (C.c_size_t, [C.POINTER(NasgScene), C.c_int32,
                                                  C.POINTER(NasgBatchTuning)]),
    "nasg_batched_plan": (C.c_int, [C.POINTER(NasgScene), C.c_int32, C.c_int32,
                                    C.POINTER(NasgBatchTuning), C.c_void_p, C.c_size_t,
                                    C.POINTER(NasgBatch), C.c_void_p]),
    "nasg_batched_run": (C.c_int, [C.POINTER(NasgBatch), C.c_void_p]),
    "nasg_raster_workspace_bytes": (C.c_size_t, [C.c_int64, C.POINTER(NasgCamera), C.c_int32]),
    "nasg_raster_fwd": (C.c_int, [C.POINTER(NasgGaussians), C.POINTER(NasgCamera), C.c_int32,
                                  C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "nasg_raster_bwd": (C.c_int, [C.POINTER(NasgGaussians), C.POINTER(NasgCamera), C.c_int32,
                                  C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "nasg_raster_fwd_noalloc": (C.c_int, [C.POINTER(NasgGaussians), C.POINTER(NasgCamera),
                                          C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "nasg_hbm_stream": (C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                                  C.c_int32, C.c_int32, C.c_void_p]),
    "nasg_camera_knn": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                  C.c_void_p]),
    "nasg_status_string": (C.c_char_p, [C.c_int]),
    "nasg_set_tuning": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                  C.POINTER(NasgTuning)]),
    "nasg_get_tuning": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                  C.POINTER(NasgTuning)]),
}

_lib = None


class NasgError(RuntimeError):
    pass


def lib() -> C.CDLL:
    """Load libnasg.so once; raise if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise NasgError(f"{LIB_PATH} is not built; run `python -m paper_2606_09794_amd.build`")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def check(status: int, what: str) -> None:
    if status != NASG_OK:
        msg = lib().nasg_status_string(status).decode()
        raise NasgError(f"{what} failed with status {status}: {msg}")
