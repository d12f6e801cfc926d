"""Reduced-precision reading of the V-cycle (test infrastructure only).

Not in the paper: the addition that runs the preconditioner with the finest
operator rounded to FP32 and the coarse operators stored in BF16 with one
scale per scalar row (reading R18), inside an FP64 outer Krylov loop. This
module computes, in FP64 arithmetic, the cycle that such a preconditioner
defines, so that a reduced-precision implementation can be compared with it
to the rounding of its FP32 vectors and accumulations instead of to the
much larger effect of the BF16 operator values:

* level 0: every stored value rounded to FP32 (round to nearest even);
* levels 1 .. L-1 (MIXED) or all non-coarsest levels (FP32): per scalar row
  r of node i the scale s = fp32(|a_(i,r),(i,r)|) (the row's largest
  magnitude when the diagonal is zero, 1 for a zero row); every value of the
  row is stored as bf16(a / s) and used as bf16(a / s) * s, where bf16() is
  round to nearest even at 8 significant bits;
* the smoothers' inverted diagonal blocks are those of the unrounded
  operator; a Gauss-Seidel sweep updates x_i += D_i^{-1} (b_i - sum_j A_ij x_j)
  with the rounded row (own block included), Jacobi x += omega D^{-1} (b - A x);
* transfers and the coarsest solve as in the FP64 cycle (Algorithm 1);
* optionally the cycle from level d down, entered from zero, is an explicit
  map T_d: the FP64 cycle's matrix from level d, each entry rounded to BF16
  (MIXED) or FP32 (FP32).

Parity unpinned as a reading of the paper (it has no reduced precision);
the rounding functions are pinned to their definitions, and the cycle to
the FP64 cycle when no rounding is applied.
"""
from __future__ import annotations

import numpy as np

from . import amg, cloops
from .sparse import BlockCSR


def bf16_round(v: np.ndarray) -> np.ndarray:
    """Round FP64 values to nearest even at 8 significant bits (BF16's
    precision; exponents stay those of FP64, fine for the scaled values of
    the operators)."""
    u = np.ascontiguousarray(v, dtype=np.float64).view(np.uint64)
    drop = np.uint64(45)                      # 52 - 7 mantissa bits dropped
    half = np.uint64((1 << 44) - 1)
    lsb = (u >> drop) & np.uint64(1)
    r = (u + half + lsb) & ~np.uint64((1 << 45) - 1)
    out = r.view(np.float64)
    return np.where(np.isnan(v), v, out)


def fp32_round(v: np.ndarray) -> np.ndarray:
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


def row_scales(A: BlockCSR) -> np.ndarray:
    """(n, br): the scale of every scalar row (reading R18)."""
    n = A.nrows
    br = A.bshape[0]
    rows = A.row_of()
    diag = np.abs(np.einsum("nii->ni", A.diag_blocks()))
    s = diag.copy()
    for r in range(br):
        zero = s[:, r] == 0.0
        if zero.any():
            rowmax = np.zeros(n)
            np.maximum.at(rowmax, rows, np.abs(A.vals[:, r, :]).max(axis=1))
            s[zero, r] = np.where(rowmax[zero] == 0.0, 1.0, rowmax[zero])
    return fp32_round(s)


def round_operator(A: BlockCSR, kind: str) -> BlockCSR:
    """The operator as a reduced-precision cycle uses it: kind 'fp32' or 'bf16'."""
    if kind == "fp32":
        vals = fp32_round(A.vals)
    else:
        s = row_scales(A)[A.row_of()]            # (nnz, br)
        vals = bf16_round(A.vals / s[:, :, None]) * s[:, :, None]
    return BlockCSR(A.indptr, A.indices, vals, A.ncols)


def reduced_operators(h: amg.Hierarchy, precision: str = "MIXED") -> list:
    """One rounded operator per non-coarsest level (None on the coarsest);
    precision 'FP64' keeps every operator unrounded."""
    ops = []
    for l, lev in enumerate(h.levels):
        if l == h.L:
            ops.append(None)
        elif precision == "FP64":
            ops.append(lev.A)
        elif l == 0 or precision == "FP32":
            ops.append(round_operator(lev.A, "fp32"))
        else:
            ops.append(round_operator(lev.A, "bf16"))
    return ops


def coarse_end_map(h: amg.Hierarchy, sm: amg.Smoother, d: int, precision: str = "MIXED") -> np.ndarray:
    """T_d: the FP64 cycle from level d (zero initial guess) as a matrix,
    each entry rounded to the coarse levels' value type."""
    n = 3 * h.levels[d].n
    cols = []
    for e in np.eye(n):
        b = e.reshape(-1, 3)
        if d == h.L:
            cols.append(amg.coarse_solve(h, e))
        else:
            cols.append(amg.cycle(h, d, sm, b, np.zeros_like(b)).ravel())
    T = np.stack(cols, axis=1)
    if precision == "FP64":
        return T
    return bf16_round(T) if precision == "MIXED" else fp32_round(T)


def _smooth(lev, A, sm, l, b, x, pre):
    steps = sm.pre if pre else sm.post
    for _ in range(steps):
        if sm.kind == "JA":
            r = b - A.matvec(x)
            x = x + sm.level_omega(l) * np.einsum("nij,nj->ni", lev.dinv, r)
        elif sm.kind == "GS":
            forward = pre or sm.post_forward
            order = lev.order_fwd if forward else lev.order_bwd
            x = np.ascontiguousarray(x, dtype=np.float64).copy()
            cloops.block_gs_update(order, A.indptr, A.indices, A.vals, lev.dinv, np.ascontiguousarray(b), x)
        else:
            raise ValueError(sm.kind)
    return x


def reduced_cycle(h, ops, sm, l, b, x, nu=1, tail=None):
    """Algorithm 1 on the rounded operators ``ops`` (``tail`` = (d, T_d) or None)."""
    lev = h.levels[l]
    A = ops[l]
    x = _smooth(lev, A, sm, l, b, x, pre=True)
    r = b - A.matvec(x)
    bc = (lev.P.T @ r).reshape(-1, 3)
    if l + 1 == h.L:
        xc = amg.coarse_solve(h, bc.ravel()).reshape(-1, 3)
    elif tail is not None and tail[0] == l + 1:
        xc = (tail[1] @ bc.ravel()).reshape(-1, 3)
        for _ in range(nu - 1):
            xc = reduced_cycle(h, ops, sm, l + 1, bc, xc, nu, tail)
    else:
        xc = np.zeros_like(bc)
        for _ in range(nu):
            xc = reduced_cycle(h, ops, sm, l + 1, bc, xc, nu, tail)
    x = x + lev.P @ xc
    return _smooth(lev, A, sm, l, b, x, pre=False)


def reduced_preconditioner(h, sm, precision="MIXED", tail_level=None, cycles=1, nu=1):
    """z = M^{-1} r of the reduced-precision cycle (SPD hierarchies)."""
    ops = reduced_operators(h, precision)
    tail = None
    if tail_level is not None and 0 < tail_level <= h.L:
        tail = (tail_level, coarse_end_map(h, sm, tail_level, precision))

    def apply(r):
        r = np.asarray(r, dtype=np.float64).reshape(-1, 3)
        if h.L == 0:
            return amg.coarse_solve(h, r.ravel()).reshape(-1, 3)
        x = np.zeros_like(r)
        for _ in range(cycles):
            x = reduced_cycle(h, ops, sm, 0, r, x, nu, tail)
        return x
    return apply
