"""Build and load the generator's C forward model (gcc + OpenMP, no GPU code)."""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fvgen.c")
_LIB = os.path.join(_HERE, "_libfvgen.so")
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.fv_forward.argtypes = [P, P, ctypes.c_double, ctypes.c_int, ctypes.c_int, P, P, P, P, P, ctypes.c_int,
                                 P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, P, P]
        L.fv_forward.restype = ctypes.c_int
        _lib = L
    return _lib
