"""Loader for the oracle's C helper (sequential FP64 loops). Test infrastructure."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "c", "orc_seq.c")
LIB = os.path.join(_HERE, "c", "liborc_seq.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle's C helper with gcc (no contraction of multiply-add)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        L.orc_codes.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_void_p]
        L.orc_codes.restype = None
        L.orc_sqdist.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]
        L.orc_sqdist.restype = None
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = None
        _lib = L
    return _lib


def codes(V: np.ndarray, A: np.ndarray, beta: np.ndarray, w: float) -> np.ndarray:
    V = np.ascontiguousarray(V, dtype=np.float32)
    A = np.ascontiguousarray(A, dtype=np.float32)
    beta = np.ascontiguousarray(beta, dtype=np.float32)
    n, D = V.shape
    m = A.shape[0]
    assert A.shape[1] == D and beta.shape == (m,)
    out = np.empty((n, m), dtype=np.int32)
    lib().orc_codes(V.ctypes.data, n, D, A.ctypes.data, beta.ctypes.data, m, float(w),
                    out.ctypes.data)
    return out


def set_threads(n: int) -> None:
    """Threads of the helper's OpenMP loops (the code projection)."""
    lib().orc_set_threads(int(n))


def sqdist(q: np.ndarray, Y: np.ndarray, rows: np.ndarray) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float32)
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty(rows.shape[0], dtype=np.float64)
    lib().orc_sqdist(q.ctypes.data, Y.ctypes.data, rows.ctypes.data, rows.shape[0],
                     Y.shape[1], out.ctypes.data)
    return out
