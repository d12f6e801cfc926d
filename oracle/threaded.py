"""The oracle on every host core (test infrastructure only).

Inside ``on_threads(h, n)`` the oracle's order-independent loops run on n
host threads through OpenMP (``omp_loops.c``), for timing the oracle on all
host cores beside its single-thread timing:

- ``BlockCSR.matvec`` (the Krylov operator, residuals, the saddle blocks):
  rows in parallel;
- the transfers ``P^T r`` and ``P e`` of every level of an SPD hierarchy
  ``h``: rows of P^T and P in parallel (P^T stored once; a saddle
  hierarchy, which also slices P for its pressure block, keeps scipy's);
- ``gauss_seidel`` on a level whose node order is grouped by colour (Section
  3.3's block Gauss-Seidel by colours): the nodes of one colour in parallel,
  which gives the sequential sweep's result bit for bit; a level in plain
  index order keeps the oracle's sequential sweep;
- ``jacobi``: its residual through the threaded product and the D^{-1} step
  per node in parallel.

Dot products and vector updates stay numpy's (its BLAS decides their
threads). Every other step, the cycle's recursion and the Krylov method are
the oracle's own code, unchanged.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from contextlib import contextmanager

import numpy as np
import scipy.sparse as sp

from . import amg, sparse

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "omp_loops.c")
LIB = os.path.join(HERE, "_omp_loops.so")

_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-fopenmp", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        p, i64, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
        L.omp_set_threads.argtypes = [ctypes.c_int]
        L.omp_threads.restype = ctypes.c_int
        L.omp_bsr_matvec.argtypes = [i64, i64, i64, p, p, p, p, p]
        L.omp_csr_matvec.argtypes = [i64, p, p, p, p, p]
        L.omp_block_gs_colours.argtypes = [i64, p, p, p, p, p, p, p, p]
        L.omp_block_jacobi.argtypes = [i64, p, p, p, f64, p]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def bsr_matvec(M: sparse.BlockCSR, x: np.ndarray) -> np.ndarray:
    """y = M x as BlockCSR.matvec computes it, rows on the host threads."""
    br, bc = M.bshape
    xs = _f64(x).reshape(M.ncols, bc)
    y = np.empty((M.nrows, br))
    ip = np.ascontiguousarray(M.indptr, dtype=np.int64)
    ix = np.ascontiguousarray(M.indices, dtype=np.int64)
    vals = _f64(M.vals)
    lib().omp_bsr_matvec(M.nrows, br, bc, _p(ip), _p(ix), _p(vals), _p(xs), _p(y))
    return y


class _CSR:
    """A scalar CSR matrix (P or P^T) whose products run on the host threads,
    for a column vector or a block of columns."""

    def __init__(self, m: sp.csr_matrix, T: "_CSR | None" = None):
        m = sp.csr_matrix(m)
        self.shape = m.shape
        self.indptr = np.ascontiguousarray(m.indptr, dtype=np.int64)
        self.indices = np.ascontiguousarray(m.indices, dtype=np.int64)
        self.data = _f64(m.data)
        self._m = m
        self._T = T

    @property
    def T(self) -> "_CSR":
        if self._T is None:
            self._T = _CSR(self._m.T.tocsr(), T=self)
        return self._T

    def __matmul__(self, x):
        x = _f64(x)
        cols = x.reshape(x.shape[0], -1)
        out = np.empty((self.shape[0], cols.shape[1]))
        for c in range(cols.shape[1]):
            xc = np.ascontiguousarray(cols[:, c])
            yc = np.empty(self.shape[0])
            lib().omp_csr_matvec(self.shape[0], _p(self.indptr), _p(self.indices), _p(self.data), _p(xc), _p(yc))
            out[:, c] = yc
        return out.reshape((self.shape[0],) + x.shape[1:])


def _colour_starts(lev) -> tuple | None:
    """Colour boundaries of the level's forward and backward orders, or None
    when its order is not grouped by colour."""
    col = np.asarray(lev.colors)
    if lev.order_fwd is None or not np.all(np.diff(col[lev.order_fwd]) >= 0):
        return None
    counts = np.bincount(col, minlength=int(col.max()) + 1 if col.size else 0).astype(np.int64)
    fwd = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    bwd = np.concatenate([[0], np.cumsum(counts[::-1])]).astype(np.int64)
    return fwd, bwd


def gauss_seidel_colours(lev, b: np.ndarray, x: np.ndarray, forward: bool, starts) -> np.ndarray:
    x = _f64(x).copy()
    order = np.ascontiguousarray(lev.order_fwd if forward else lev.order_bwd, dtype=np.int64)
    cs = starts[0] if forward else starts[1]
    ip = np.ascontiguousarray(lev.A.indptr, dtype=np.int64)
    ix = np.ascontiguousarray(lev.A.indices, dtype=np.int64)
    vals, dinv, bb = _f64(lev.A.vals), _f64(lev.dinv), _f64(b)
    lib().omp_block_gs_colours(cs.shape[0] - 1, _p(cs), _p(order), _p(ip), _p(ix), _p(vals), _p(dinv), _p(bb),
                               _p(x))
    return x


def jacobi(lev, b: np.ndarray, x: np.ndarray, omega: float) -> np.ndarray:
    r = _f64(b).reshape(-1, 3) - bsr_matvec(lev.A, x)
    xs = _f64(x).reshape(-1, 3)
    out = np.empty_like(xs)
    lib().omp_block_jacobi(lev.n, _p(_f64(lev.dinv)), _p(_f64(r)), _p(xs), float(omega), _p(out))
    return out


def threads() -> int:
    return int(lib().omp_threads())


@contextmanager
def on_threads(h, n: int):
    """Run the oracle's order-independent loops on n host threads while
    inside; restores the oracle's own functions and h's transfers after."""
    L = lib()
    L.omp_set_threads(int(n))
    starts = {id(lev): _colour_starts(lev) for lev in h.levels}
    saved_P = [lev.P for lev in h.levels]
    seq_gs, seq_ja, seq_mv = amg.gauss_seidel, amg.jacobi, sparse.BlockCSR.matvec

    def gs(lev, b, x, forward):
        s = starts.get(id(lev))
        if s is None:
            return seq_gs(lev, b, x, forward)
        return gauss_seidel_colours(lev, b, x, forward, s)

    try:
        for lev in h.levels:
            if lev.P is not None and not h.saddle:
                lev.P = _CSR(lev.P)
        amg.gauss_seidel = gs
        amg.jacobi = jacobi
        sparse.BlockCSR.matvec = bsr_matvec
        yield
    finally:
        amg.gauss_seidel, amg.jacobi = seq_gs, seq_ja
        sparse.BlockCSR.matvec = seq_mv
        for lev, P in zip(h.levels, saved_P):
            lev.P = P
