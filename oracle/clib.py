"""Build and load the oracle's plain-C helpers (gcc, no GPU code)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bilu.c")
_LIB = os.path.join(_HERE, "_liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.oracle_bilu0.argtypes = [ctypes.c_int, P, P, P, P, P]
        L.oracle_bilu0.restype = ctypes.c_int
        L.oracle_bilu0_solve.argtypes = [ctypes.c_int, P, P, P, P, P, P, P]
        L.oracle_bilu0_solve.restype = None
        L.oracle_iluk_symbolic.argtypes = [ctypes.c_int, P, P, ctypes.c_int, ctypes.c_long, P, P, P]
        L.oracle_iluk_symbolic.restype = ctypes.c_long
        L.oracle_inv33.argtypes = [P, P]
        L.oracle_inv33.restype = ctypes.c_int
        _lib = L
    return _lib


def ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)
