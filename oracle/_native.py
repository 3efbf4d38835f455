"""ctypes loader for oracle/native.c (test infrastructure only)."""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "native.c")
LIB = os.path.join(_HERE, "liboracle_native.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile native.c with gcc (no fast-math) into oracle/liboracle_native.so."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                        "-fno-fast-math", "-ffp-contract=off", SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        L.oracle_grid_accumulate.argtypes = [i64, i64, i64, p, p, p, p, p, p, p, p]
        L.oracle_grid_accumulate.restype = None
        L.oracle_dft.argtypes = [i64, p, p, p, p, p, i64, p, p, p, p]
        L.oracle_dft.restype = None
        L.oracle_degrid.argtypes = [i64, i64, i64, p, p, p, p, p, p]
        L.oracle_degrid.restype = None
        L.oracle_kb_eval.argtypes = [i64, p, i64, ctypes.c_double, p]
        L.oracle_kb_eval.restype = None
        _lib = L
    return _lib


def ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)
