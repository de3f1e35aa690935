"""ctypes view of libgrav's C ABI (declared in include/grav.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  If the library is missing, loading raises instead of falling back.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrav.so")

GRAV_OK, GRAV_EINVAL, GRAV_ENOMEM, GRAV_EDEVICE, GRAV_EUNSUPPORTED, GRAV_EBUSY = range(6)
GRAV_FP64, GRAV_MIXED = 0, 1

# Every extern "C" function include/grav.h declares.
EXPORTS = (
    "grav_desc_init", "grav_plan", "grav_plan_destroy", "grav_plan_bytes", "grav_plan_info",
    "grav_plan_work", "grav_plan_check",
    "grav_eval", "grav_adjoint", "grav_direct", "grav_direct_noalloc", "grav_analytic", "grav_set_profiling", "grav_stage_times", "grav_operator",
    "grav_harmonics", "grav_status_string", "grav_version",
)


class GravDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("origin", ctypes.c_double * 3),
        ("h", ctypes.c_double),
        ("quad_order", ctypes.c_int32),
        ("n_points", ctypes.c_int64),
        ("points", ctypes.POINTER(ctypes.c_double)),
        ("voxel_centres", ctypes.c_int32),
        ("components", ctypes.c_int32),
        ("p", ctypes.c_int32),
        ("leaf_size", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("batch", ctypes.c_int32),
        ("G", ctypes.c_double),
        ("device", ctypes.c_int32),
        ("n_sources", ctypes.c_int64),
        ("sources", ctypes.POINTER(ctypes.c_double)),
        ("source_volumes", ctypes.POINTER(ctypes.c_double)),
    ]


class GravError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib_or_none().grav_status_string(code).decode() if _lib_or_none() else str(code)
        super().__init__("%s failed: %s (code %d)" % (where, msg, code))


_lock = threading.Lock()
_lib = None


def _lib_or_none():
    return _lib


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libgrav.so (build it first with ``python -m paper_1107_5951_amd.build``)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise ImportError("libgrav.so not found at %s; run paper_1107_5951_amd/build.py" % path)
        lib = ctypes.CDLL(path)
        vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        sig = {
            "grav_desc_init": ([ctypes.POINTER(GravDesc)], None),
            "grav_plan": ([ctypes.POINTER(GravDesc), ctypes.POINTER(vp)], ctypes.c_int),
            "grav_plan_destroy": ([vp], None),
            "grav_plan_bytes": ([vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)],
                                ctypes.c_int),
            "grav_plan_info": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                ctypes.POINTER(i64)], ctypes.c_int),
            "grav_plan_work": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)],
                               ctypes.c_int),
            "grav_plan_check": ([vp, ctypes.c_char_p, i32], ctypes.c_int),
            "grav_eval": ([vp, vp, vp, vp], ctypes.c_int),
            "grav_adjoint": ([vp, vp, vp, vp], ctypes.c_int),
            "grav_direct": ([vp, vp, vp, vp], ctypes.c_int),
            "grav_direct_noalloc": ([vp, vp, vp, vp], ctypes.c_int),
            "grav_analytic": ([vp, vp, vp, vp], ctypes.c_int),
            "grav_set_profiling": ([vp, i32], ctypes.c_int),
            "grav_stage_times": ([vp, ctypes.POINTER(ctypes.c_char_p), dp, i32, ctypes.POINTER(i32)],
                                 ctypes.c_int),
            "grav_operator": ([i32, i32, i32, i32, i32, i32, dp], ctypes.c_int),
            "grav_harmonics": ([i32, i32, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp],
                               ctypes.c_int),
            "grav_status_string": ([ctypes.c_int], ctypes.c_char_p),
            "grav_version": ([], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
        return lib


def check(code: int, where: str) -> None:
    if code != GRAV_OK:
        raise GravError(code, where)
