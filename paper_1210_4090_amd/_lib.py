"""ctypes declarations of the C ABI in include/lo.h (argument marshalling only).

Loads the in-tree liblo.so built by paper_1210_4090_amd/build.py.  There is
no fallback: if the library is missing every call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblo.so")

LO_OK = 0
LO_ERR_INVALID = 1
LO_ERR_UNSUPPORTED = 2
LO_ERR_OOM = 3
LO_ERR_HIP = 4
LO_ERR_WINDOW = 5
LO_BRUTE = 0
LO_FAST = 1
LO_FLAG_NO_GRAPH = 1
LO_FLAG_AUTOTUNE = 2

_f64p = ctypes.POINTER(ctypes.c_double)


class LoDesc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("period", ctypes.c_double * 3),
        ("tau", ctypes.c_double),
        ("P", ctypes.c_double * 3),
        ("kstar_tab", ctypes.c_void_p * 3),
        ("kstar_half", ctypes.c_int64 * 3),
        ("window", ctypes.c_int32 * 3),
        ("method", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("t0", ctypes.c_double),
    ]


class LoPotential(ctypes.Structure):
    _fields_ = [
        ("table", ctypes.c_void_p),
        ("nmodes", ctypes.c_int32),
        ("basis", ctypes.c_void_p),
        ("coef", ctypes.c_void_p),
        ("tcoef", ctypes.c_void_p),
        ("ntcoef", ctypes.c_int64),
    ]


class LoError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__("%s failed: %s (status %d)" % (fn, msg, status))
        self.status = status


_lib = None

# name -> (restype, argtypes)
SIGNATURES = {
    "lo_plan": (ctypes.c_int, [ctypes.POINTER(LoDesc), ctypes.POINTER(LoPotential), ctypes.POINTER(ctypes.c_void_p)]),
    "lo_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "lo_set_coef": (ctypes.c_int, [ctypes.c_void_p, _f64p]),
    "lo_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "lo_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                              ctypes.c_void_p, ctypes.c_void_p]),
    "lo_effective_H": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(LoDesc), ctypes.POINTER(LoPotential),
                                      ctypes.c_double, _f64p, ctypes.c_void_p]),
    "lo_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_void_p, ctypes.c_void_p, _f64p, ctypes.c_void_p]),
    "lo_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "lo_last_diag": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "lo_kinetic_table": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _f64p]),
    "lo_time_kernels": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, _f64p,
                                       ctypes.c_void_p]),
    "lo_run_decomp": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                     ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.c_void_p]),
    "lo_run_semigroup1": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                         ctypes.c_void_p]),
    "lo_run_record": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_void_p]),
    "lo_backward_recorded": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                            ctypes.c_void_p, _f64p, ctypes.c_void_p]),
    "lo_step_noalloc": (ctypes.c_int, [ctypes.POINTER(LoDesc), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p]),
}
LO_NOALLOC_MAX_POINTS = 4194304


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is missing: build it with paper_1210_4090_amd/build.py "
                               "(or __graft_entry__.build())" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(fn: str, status: int) -> None:
    if status != LO_OK:
        msg = lib().lo_status_string(status).decode()
        raise LoError(fn, status, msg)
