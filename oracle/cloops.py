"""ctypes access to ``oracle/loops.c`` (test infrastructure only).

``build()`` compiles the C file with gcc into ``oracle/_loops.so``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "loops.c")
LIB = os.path.join(HERE, "_loops.so")

_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.oracle_greedy_mis.argtypes = [i64, p, p, p]
        L.oracle_greedy_mis.restype = i64
        L.oracle_greedy_colour.argtypes = [i64, p, p, p]
        L.oracle_greedy_colour.restype = i64
        L.oracle_block_gs.argtypes = [i64, p, p, p, p, p, p, p]
        L.oracle_block_gs.restype = None
        L.oracle_scalar_gs.argtypes = [i64, p, p, p, p, p, p]
        L.oracle_scalar_gs.restype = None
        L.oracle_block_gs_update.argtypes = [i64, p, p, p, p, p, p, p]
        L.oracle_block_gs_update.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def greedy_mis(indptr: np.ndarray, indices: np.ndarray) -> np.ndarray:
    """Coarse mask of the greedy maximal independent set in index order."""
    n = indptr.shape[0] - 1
    ip = np.ascontiguousarray(indptr, dtype=np.int64)
    ix = np.ascontiguousarray(indices, dtype=np.int64)
    st = np.zeros(n, dtype=np.int8)
    lib().oracle_greedy_mis(n, _p(ip), _p(ix), _p(st))
    return st == 1


def greedy_colour(indptr: np.ndarray, indices: np.ndarray) -> np.ndarray:
    n = indptr.shape[0] - 1
    ip = np.ascontiguousarray(indptr, dtype=np.int64)
    ix = np.ascontiguousarray(indices, dtype=np.int64)
    col = np.zeros(n, dtype=np.int32)
    lib().oracle_greedy_colour(n, _p(ip), _p(ix), _p(col))
    return col


def block_gs(order, indptr, indices, vals, dinv, b, x) -> None:
    """In-place block Gauss-Seidel sweep over ``order`` (x modified)."""
    o = np.ascontiguousarray(order, dtype=np.int64)
    ip = np.ascontiguousarray(indptr, dtype=np.int64)
    ix = np.ascontiguousarray(indices, dtype=np.int64)
    v = np.ascontiguousarray(vals, dtype=np.float64)
    d = np.ascontiguousarray(dinv, dtype=np.float64)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    assert x.flags.c_contiguous and x.dtype == np.float64
    lib().oracle_block_gs(o.shape[0], _p(o), _p(ip), _p(ix), _p(v), _p(d), _p(bb), _p(x))


def block_gs_update(order, indptr, indices, vals, dinv, b, x) -> None:
    """In-place block Gauss-Seidel sweep in correction form (x modified)."""
    o = np.ascontiguousarray(order, dtype=np.int64)
    ip = np.ascontiguousarray(indptr, dtype=np.int64)
    ix = np.ascontiguousarray(indices, dtype=np.int64)
    v = np.ascontiguousarray(vals, dtype=np.float64)
    d = np.ascontiguousarray(dinv, dtype=np.float64)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    assert x.flags.c_contiguous and x.dtype == np.float64
    lib().oracle_block_gs_update(o.shape[0], _p(o), _p(ip), _p(ix), _p(v), _p(d), _p(bb), _p(x))


def scalar_gs(order, indptr, indices, vals, b, x) -> None:
    o = np.ascontiguousarray(order, dtype=np.int64)
    ip = np.ascontiguousarray(indptr, dtype=np.int64)
    ix = np.ascontiguousarray(indices, dtype=np.int64)
    v = np.ascontiguousarray(vals, dtype=np.float64)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    assert x.flags.c_contiguous and x.dtype == np.float64
    lib().oracle_scalar_gs(o.shape[0], _p(o), _p(ip), _p(ix), _p(v), _p(bb), _p(x))
