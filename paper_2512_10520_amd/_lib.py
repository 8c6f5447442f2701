"""ctypes view of the C ABI in include/mt.h (libmt.so built in-tree).

No fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmt.so")

MT_OK = 0
ERRORS = {-1: "MT_ERR_INVALID_ARG", -2: "MT_ERR_SHAPE", -3: "MT_ERR_EMPTY_HIST",
          -4: "MT_ERR_NOT_LOADED", -5: "MT_ERR_OOM", -6: "MT_ERR_HIP", -7: "MT_ERR_LIMIT"}
MT_MODE_PLAIN, MT_MODE_PERSISTENT, MT_MODE_VARIANT_WAVES = 0, 1, 2
MT_SAMPLER_CDF, MT_SAMPLER_ALIAS = 0, 1
MT_INTERP_TRILINEAR, MT_INTERP_NEAREST = 0, 1
MT_AXIS_LOG_LOSS, MT_AXIS_LOG_SCAT = 1, 2
MT_OPT_GUIDE_BITS, MT_OPT_ADJOINT_BLOCK, MT_OPT_ADJOINT_LDS_HISTORY = 1, 2, 3
MT_NOALLOC_SCRATCH_BYTES = 1 << 20
ST_RUNNING, ST_PMIN, ST_ZMAX, ST_XMAX, ST_YMAX, ST_MAXSTEPS, ST_INVALID = range(7)
CKPT_EVERY = 16

# Names of every entry point the header declares (checked by the CPU tests).
EXPORTS = ("mt_load_histograms", "mt_load_histograms_ex", "mt_optimal_edges",
           "mt_load_geometry", "mt_load_blocks", "mt_load_field", "mt_propagate",
           "mt_propagate_noalloc", "mt_propagate_backward", "mt_autotune", "mt_set_option",
           "mt_last_error", "mt_release", "mt_device_info")


class MtParams(C.Structure):
    _fields_ = [
        ("step_m", C.c_double), ("max_steps", C.c_int32), ("p_min", C.c_double),
        ("seed", C.c_uint64), ("n_variants", C.c_int32), ("scales", C.c_void_p),
        ("mode", C.c_int32), ("block", C.c_int32), ("compact_every", C.c_int32),
        ("use_graph", C.c_int32), ("ckpt_every", C.c_int32), ("ckpt", C.c_void_p),
        ("tape", C.c_void_p), ("trace", C.c_void_p), ("n_trace", C.c_int64),
        ("trace_steps", C.c_int32), ("tally", C.c_void_p),
        ("z_det", C.c_double), ("r_ap", C.c_double), ("r_scale", C.c_double),
        ("sampler", C.c_int32), ("interp", C.c_int32), ("stage_field", C.c_int32),
    ]


class MtMuons(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("x", "y", "z", "px", "py", "pz", "q")]


class MtResult(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("status", "n_steps", "volume")]


_lock = threading.Lock()
_lib = None


def load():
    """Load libmt.so; raise if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is missing: build the HIP library first "
                    "(python -m paper_2512_10520_amd.csrc.build)")
            L = C.CDLL(LIB_PATH)
            vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
            L.mt_load_histograms.argtypes = [i32, i32, vp, i32, dbl, dbl, i32, dbl, dbl, vp]
            L.mt_load_histograms_ex.argtypes = [i32, i32, vp, i32, dbl, dbl, i32, dbl, dbl, vp,
                                                i32]
            L.mt_optimal_edges.argtypes = [vp, vp, i32, dbl, vp, i32, C.POINTER(i32)]
            L.mt_load_geometry.argtypes = [i32, vp, vp, vp, vp, i32, vp]
            L.mt_load_blocks.argtypes = [i32, vp, vp, vp, vp, i32, vp]
            L.mt_load_field.argtypes = [i32, i32, i32, vp, vp, vp]
            L.mt_propagate.argtypes = [C.POINTER(MtParams), i64, C.POINTER(MtMuons),
                                       C.POINTER(MtMuons), C.POINTER(MtResult), vp]
            L.mt_propagate_noalloc.argtypes = [C.POINTER(MtParams), i64, C.POINTER(MtMuons),
                                               C.POINTER(MtMuons), C.POINTER(MtResult), vp]
            L.mt_propagate_backward.argtypes = [C.POINTER(MtParams), i64, C.POINTER(MtMuons),
                                                C.POINTER(MtResult), vp, vp, vp, vp]
            L.mt_autotune.argtypes = [C.POINTER(MtParams), i64, C.POINTER(MtMuons),
                                      C.POINTER(MtMuons), C.POINTER(MtResult), vp,
                                      C.POINTER(i32), C.POINTER(i32), C.POINTER(C.c_float)]
            L.mt_set_option.argtypes = [i32, i64]
            L.mt_last_error.restype = C.c_char_p
            L.mt_last_error.argtypes = []
            L.mt_release.restype = None
            L.mt_release.argtypes = []
            L.mt_device_info.argtypes = [vp]
            for name in EXPORTS:
                if name not in ("mt_last_error", "mt_release"):
                    getattr(L, name).restype = C.c_int
            _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != MT_OK:
        msg = load().mt_last_error().decode(errors="replace")
        raise RuntimeError(f"{ERRORS.get(rc, rc)}: {msg}")
