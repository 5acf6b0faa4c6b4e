"""Build-and-load helper for the oracle's plain C sums (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bie_sums.c")
_LIB = os.path.join(_HERE, "liboracle_bie.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile bie_sums.c with gcc (-O2, OpenMP over targets)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_bie_sums.restype = None
        L.oracle_bie_sums.argtypes = ([ctypes.c_int, ctypes.c_int] + [ctypes.c_double] * 4 + [ctypes.c_int]
                                      + [dp] * 10 + [ctypes.c_int] + [dp] * 7 + [ip, ctypes.c_int, dp])
        _lib = L
    return _lib


def dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def iptr(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
