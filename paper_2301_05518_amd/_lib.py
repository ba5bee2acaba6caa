"""ctypes declarations of libtwolink.so (the C ABI in include/twolink.h)."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtwolink.so")

TL_OK = 0
ERRORS = {
    -1: "TL_ERR_ARG", -2: "TL_ERR_SHAPE", -3: "TL_ERR_PRECISION", -4: "TL_ERR_DEVICE",
    -5: "TL_ERR_HIP", -6: "TL_ERR_NOMEM", -7: "TL_ERR_UNSUPPORTED",
}
TL_W12 = 16       # OR into a precision: twelve-real (two-row) link storage
TL_ONELINK = 32   # OR into a precision: a one-link field and the one-link operators
_BASE = {"f64": 0, "f32": 1, "f16s": 2, "bf16": 3}
# "<prec>[-w12][-onelink]"
PREC = {b + w + o: v | (TL_W12 if w else 0) | (TL_ONELINK if o else 0)
        for b, v in _BASE.items() for w in ("", "-w12") for o in ("", "-onelink")}
TL_PLAIN, TL_GRAPH, TL_AUTOTUNE, TL_ONE_STEP = 1, 2, 4, 8
TL_NORM2, TL_DOT, TL_SITE_NORM = 0, 1, 2

# every symbol the header declares
EXPORTS = [
    "tl_version", "tl_create", "tl_destroy", "tl_set_stream", "tl_sync", "tl_last_error",
    "tl_check_geom", "tl_twolinks_bytes", "tl_build_twolinks", "tl_pack_links", "tl_laplacian", "tl_smear",
    "tl_plan_create", "tl_plan_load", "tl_plan_run", "tl_plan_store", "tl_plan_reduce",
    "tl_plan_time", "tl_plan_get_info", "tl_plan_destroy", "tl_reduce", "tl_reduce_noalloc", "tl_stream_time", "tl_get_stats",
]


class Geom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4)]


class Job(ctypes.Structure):
    _fields_ = [
        ("g", Geom),
        ("W", ctypes.c_void_p),
        ("w_slices", ctypes.POINTER(ctypes.c_int32)),
        ("n_w_slices", ctypes.c_int32),
        ("n_rhs", ctypes.c_int32),
        ("t_of_rhs", ctypes.POINTER(ctypes.c_int32)),
        ("psi", ctypes.c_void_p),
    ]


class CtxStats(ctypes.Structure):
    _fields_ = [("graphs_captured", ctypes.c_int64), ("tune_sweeps", ctypes.c_int64),
                ("tune_hits", ctypes.c_int64), ("smear_plan_hits", ctypes.c_int64)]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("n_groups", ctypes.c_int32), ("group_width", ctypes.c_int32), ("n_tiles", ctypes.c_int32),
        ("variant", ctypes.c_int32), ("block", ctypes.c_int32), ("tz", ctypes.c_int32),
        ("grid", ctypes.c_int32), ("nt", ctypes.c_int32), ("flip", ctypes.c_int32),
        ("launches_per_step", ctypes.c_int32), ("steps_per_launch", ctypes.c_int32), ("tile_width", ctypes.c_int32),
        ("rhs_sites", ctypes.c_int64), ("bytes_per_step", ctypes.c_double),
        ("flops_per_step", ctypes.c_double), ("resident_bytes", ctypes.c_int64),
    ]


_lib = None


def load() -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2301_05518_amd.build` "
            "(there is no CPU fallback for the smearing path)")
    # torch first: the library then binds to the HIP runtime torch has loaded, so the
    # process holds one runtime whose device and stream handles both sides share
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    pg, pj = ctypes.POINTER(Geom), ctypes.POINTER(Job)
    pi32 = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "tl_version": (i32, []),
        "tl_create": (i32, [ctypes.POINTER(vp), i32, vp]),
        "tl_destroy": (i32, [vp]),
        "tl_set_stream": (i32, [vp, vp]),
        "tl_sync": (i32, [vp]),
        "tl_last_error": (ctypes.c_char_p, [vp]),
        "tl_check_geom": (i32, [pg]),
        "tl_twolinks_bytes": (ctypes.c_size_t, [pg, i32, i32]),
        "tl_build_twolinks": (i32, [vp, pg, vp, pi32, i32, i32, vp]),
        "tl_pack_links": (i32, [vp, pg, vp, pi32, i32, i32, vp]),
        "tl_laplacian": (i32, [vp, pg, vp, pi32, i32, i32, i32, vp, vp]),
        "tl_smear": (i32, [vp, pj, i32, i32, dbl, i32, ctypes.c_uint]),
        "tl_plan_create": (i32, [vp, pj, i32, i32, dbl, i32, ctypes.c_uint, ctypes.POINTER(vp)]),
        "tl_plan_load": (i32, [vp]),
        "tl_plan_run": (i32, [vp]),
        "tl_plan_store": (i32, [vp]),
        "tl_plan_reduce": (i32, [vp, i32, vp, vp]),
        "tl_plan_time": (i32, [vp, i32, ctypes.POINTER(dbl)]),
        "tl_plan_get_info": (i32, [vp, ctypes.POINTER(PlanInfo)]),
        "tl_plan_destroy": (i32, [vp]),
        "tl_reduce": (i32, [vp, i32, i64, i32, vp, vp, vp]),
        "tl_reduce_noalloc": (i32, [vp, i32, i64, i32, vp, vp, vp]),
        "tl_stream_time": (i32, [vp, vp, i64, i32, i32, i32, i32, ctypes.POINTER(dbl)]),
        "tl_get_stats": (i32, [vp, ctypes.POINTER(CtxStats)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class TwolinkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
