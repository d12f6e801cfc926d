"""Krylov drivers around the AMG preconditioner (test infrastructure only).

The paper uses the AMG V-cycle as a preconditioner of CG for the SPD systems
(Section 4.2-4.3) and of GMRES for the saddle point systems (Section 4.4-4.5),
stopping when the relative l2 residual ||f - A u_k|| / ||f - A u_0|| falls
below the tolerance. Readings: x_0 = 0 unless given; the stopping test uses the
recursively updated residual, and the true residual is recomputed at exit;
GMRES is right-preconditioned flexible GMRES with restart 100 and modified
Gram-Schmidt; the saddle stopping norm is the Euclidean norm of [r_u; r_p].

* ``pcg``   preconditioned conjugate gradients (fixed SPD preconditioner);
* ``fcg``   flexible CG, one-term truncation (Notay): beta_k makes p_k
            A-orthogonal to p_{k-1}, alpha_k = <p_k, r_k> / <p_k, A p_k>;
* ``fgmres`` flexible GMRES(m).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class KrylovResult:
    x: np.ndarray
    iters: int
    relres: float                   # true relative residual at exit
    history: list = field(default_factory=list)   # recursive relres per iteration
    converged: bool = False


def pcg(matvec, prec, b, tol=1e-8, maxit=500, x0=None) -> KrylovResult:
    b = np.asarray(b, dtype=np.float64).ravel()
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64).ravel().copy()
    r = b - matvec(x)
    r0 = np.linalg.norm(r)
    hist = [1.0]
    if r0 == 0.0:
        return KrylovResult(x, 0, 0.0, hist, True)
    z = prec(r)
    p = z.copy()
    rz = r @ z
    it = 0
    conv = False
    while it < maxit:
        q = matvec(p)
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        rel = np.linalg.norm(r) / r0
        hist.append(rel)
        if rel <= tol:
            conv = True
            break
        z = prec(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    true = np.linalg.norm(b - matvec(x)) / r0
    return KrylovResult(x, it, true, hist, conv)


def fcg(matvec, prec, b, tol=1e-8, maxit=500, x0=None) -> KrylovResult:
    b = np.asarray(b, dtype=np.float64).ravel()
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64).ravel().copy()
    r = b - matvec(x)
    r0 = np.linalg.norm(r)
    hist = [1.0]
    if r0 == 0.0:
        return KrylovResult(x, 0, 0.0, hist, True)
    p_prev = q_prev = None
    pq_prev = 0.0
    it = 0
    conv = False
    while it < maxit:
        z = prec(r)
        if p_prev is None:
            p = z
        else:
            p = z - ((z @ q_prev) / pq_prev) * p_prev
        q = matvec(p)
        pq = p @ q
        alpha = (p @ r) / pq
        x += alpha * p
        r -= alpha * q
        it += 1
        rel = np.linalg.norm(r) / r0
        hist.append(rel)
        p_prev, q_prev, pq_prev = p, q, pq
        if rel <= tol:
            conv = True
            break
    true = np.linalg.norm(b - matvec(x)) / r0
    return KrylovResult(x, it, true, hist, conv)


def fgmres(matvec, prec, b, tol=1e-8, maxit=500, restart=100, x0=None) -> KrylovResult:
    b = np.asarray(b, dtype=np.float64).ravel()
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64).ravel().copy()
    r = b - matvec(x)
    r0 = np.linalg.norm(r)
    hist = [1.0]
    if r0 == 0.0:
        return KrylovResult(x, 0, 0.0, hist, True)
    it = 0
    conv = False
    beta = r0
    while it < maxit and not conv:
        m = restart
        V = np.zeros((m + 1, b.shape[0]))
        Z = np.zeros((m, b.shape[0]))
        Hm = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        gvec = np.zeros(m + 1)
        gvec[0] = beta
        V[0] = r / beta
        j_used = 0
        for j in range(m):
            Z[j] = prec(V[j])
            w = matvec(Z[j])
            for i in range(j + 1):
                Hm[i, j] = w @ V[i]
                w = w - Hm[i, j] * V[i]
            Hm[j + 1, j] = np.linalg.norm(w)
            if Hm[j + 1, j] != 0.0:
                V[j + 1] = w / Hm[j + 1, j]
            for i in range(j):
                t = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
                Hm[i + 1, j] = -sn[i] * Hm[i, j] + cs[i] * Hm[i + 1, j]
                Hm[i, j] = t
            den = np.hypot(Hm[j, j], Hm[j + 1, j])
            cs[j], sn[j] = Hm[j, j] / den, Hm[j + 1, j] / den
            Hm[j, j] = den
            Hm[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = cs[j] * gvec[j]
            it += 1
            j_used = j + 1
            rel = abs(gvec[j + 1]) / r0
            hist.append(rel)
            if rel <= tol or it >= maxit:
                conv = rel <= tol
                break
        y = np.linalg.solve(np.triu(Hm[:j_used, :j_used]), gvec[:j_used])
        x = x + Z[:j_used].T @ y
        r = b - matvec(x)
        beta = np.linalg.norm(r)
    true = np.linalg.norm(b - matvec(x)) / r0
    return KrylovResult(x, it, true, hist, conv)
