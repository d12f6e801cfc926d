"""The paper's algebraic multigrid method, written out plainly in FP64.

Test infrastructure only (see ``oracle/__init__``).

Section 3.2 (coarsening), SPD case: the coarse levels are built from two
separate graphs, the connectivity of K_ll (linear nodes) and of K_qq
(quadratic nodes); the coupling K_ql is ignored. Each graph gets its own
coarse/fine split and interpolation; the prolongation is the block-diagonal
P = diag(I, J) acting on R^3 node vectors, restriction is P^T, and coarse
operators are Galerkin products A_{l+1} = P^T A_l P.
Saddle case: velocity as above, pressure with the linear-node graph and its
own interpolation H, P = diag(I, J, H), K_{l+1} = P^T K_l P.

Readings where the paper is silent (it defers the C/F selection and weights
to a cited work that it does not reproduce):
* graphs are the structural patterns (every node pair sharing an element,
  explicit zeros kept), without self loops;
* C/F split: greedy maximal independent set visiting nodes in index order;
* interpolation: a coarse node copies its value, a fine node takes the plain
  average over its coarse graph neighbours (weights 1/|C_i|);
* coarse numbering: coarse linear nodes then coarse quadratic nodes, each in
  fine index order; the pressure graph is the linear-node graph, so H is the
  linear block of P;
* coarsening stops when a level has at most ``coarse_max`` unknowns (300),
  after ``max_levels`` levels, or when a level would keep > 90% of its nodes;
  the coarsest system is solved by dense LU with partial pivoting.

Section 3.1 (Algorithm 1, the basic AMG iteration) is ``cycle``; Section 3.3's
smoothers are ``jacobi``, ``gauss_seidel`` (block, lexicographic or by
colours), ``sgs_step`` (segregated Gauss-Seidel / Uzawa), ``bs_step``
(Braess-Sarazin) and ``vanka_step`` (multiplicative Vanka). Parity unpinned: the exact iteration counts of the paper's
tables (they depend on unstated details). The Braess-Sarazin inner Schur
cycle and the sGS pressure scaling follow the readings in their docstrings;
both are pinned to their dense definitions.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import cloops
from .sparse import BlockCSR

# --------------------------------------------------------------------------
# graphs, splitting, interpolation
# --------------------------------------------------------------------------


def node_graph(M: BlockCSR, lo: int, hi: int) -> tuple[np.ndarray, np.ndarray]:
    """CSR graph of the node range [lo, hi) of the structural pattern, no self loops."""
    S = M.pattern()[lo:hi, lo:hi].tocoo()
    keep = S.row != S.col
    G = sp.csr_matrix((np.ones(int(keep.sum())), (S.row[keep], S.col[keep])), shape=(hi - lo, hi - lo))
    G.sort_indices()
    return G.indptr.astype(np.int64), G.indices.astype(np.int64)


def averaging_prolongation(indptr: np.ndarray, indices: np.ndarray, cmask: np.ndarray) -> sp.csr_matrix:
    """P (n x nc): coarse node i -> e_{c(i)}; fine node i -> average of its coarse neighbours."""
    n = cmask.shape[0]
    cidx = np.cumsum(cmask) - 1
    rows, cols, vals = [], [], []
    ci = np.nonzero(cmask)[0]
    rows.append(ci)
    cols.append(cidx[ci])
    vals.append(np.ones(ci.shape[0]))
    r_of = np.repeat(np.arange(n), np.diff(indptr))
    sel = (~cmask[r_of]) & cmask[indices] & (indices != r_of)
    fr, fc = r_of[sel], indices[sel]
    cnt = np.bincount(fr, minlength=n)
    assert np.all(cnt[~cmask] > 0), "a fine node without a coarse neighbour"
    rows.append(fr)
    cols.append(cidx[fc])
    vals.append(1.0 / cnt[fr])
    P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, int(cmask.sum())))
    P.sort_indices()
    return P


def split_level(A: BlockCSR, nlin: int, nquad: int, separate: bool = True):
    """Coarse masks and prolongation for one level.

    Returns (P, nlin_c, nquad_c). With ``separate`` the linear and quadratic
    graphs are split independently (the paper's strategy); otherwise the
    whole node graph is split as one (the classical "non-separating" one).
    """
    n = nlin + nquad
    if not separate:
        ip, ix = node_graph(A, 0, n)
        P = averaging_prolongation(ip, ix, cloops.greedy_mis(ip, ix))
        return P, P.shape[1], 0
    ipl, ixl = node_graph(A, 0, nlin)
    ipq, ixq = node_graph(A, nlin, n)
    Pl = averaging_prolongation(ipl, ixl, cloops.greedy_mis(ipl, ixl))
    Pq = averaging_prolongation(ipq, ixq, cloops.greedy_mis(ipq, ixq))
    P = sp.block_diag([Pl, Pq], format="csr")
    P.sort_indices()
    return P, Pl.shape[1], Pq.shape[1]


def galerkin(M: BlockCSR, L: sp.csr_matrix, R: sp.csr_matrix) -> BlockCSR:
    """L^T M R on node blocks: values from the scalar product (L(x)I)^T M (R(x)I),
    pattern = structural product |L|^T pattern(M) |R| (explicit zeros kept)."""
    br, bc = M.bshape
    Lp = sp.csr_matrix((np.ones(L.nnz), L.indices, L.indptr), shape=L.shape)
    Rp = sp.csr_matrix((np.ones(R.nnz), R.indices, R.indptr), shape=R.shape)
    S = (Lp.T @ M.pattern() @ Rp).tocsr()
    S.sort_indices()
    Ls = sp.kron(L, sp.eye(br), format="csr")
    Rs = sp.kron(R, sp.eye(bc), format="csr")
    V = (Ls.T @ M.scipy() @ Rs).tocoo()
    out = BlockCSR(S.indptr.astype(np.int64), S.indices.astype(np.int64),
                   np.zeros((S.nnz, br, bc)), S.shape[1])
    skeys = np.repeat(np.arange(S.shape[0]), np.diff(S.indptr)).astype(np.int64) * S.shape[1] + S.indices
    vkeys = (V.row // br).astype(np.int64) * S.shape[1] + (V.col // bc)
    pos = np.searchsorted(skeys, vkeys)
    assert np.all(skeys[pos] == vkeys)
    out.vals[pos, V.row % br, V.col % bc] = V.data
    return out


# --------------------------------------------------------------------------
# hierarchy
# --------------------------------------------------------------------------
@dataclass
class Level:
    A: BlockCSR
    nlin: int
    nquad: int
    P: sp.csr_matrix | None = None      # prolongation from level l+1 to l
    B: BlockCSR | None = None
    C: BlockCSR | None = None
    dinv: np.ndarray | None = None      # inverted 3x3 diagonal blocks
    colors: np.ndarray | None = None
    order_fwd: np.ndarray | None = None
    order_bwd: np.ndarray | None = None
    schur: "Hierarchy | None" = None     # Braess-Sarazin: scalar AMG on C + B (2D)^-1 B^T
    sgs_diag: np.ndarray | None = None   # sGS pressure scaling diag(B M_A^-1 B^T + C)
    vanka: "VankaPatches | None" = None  # multiplicative Vanka patches and their order

    @property
    def n(self) -> int:
        return self.A.nrows

    @property
    def npres(self) -> int:
        return 0 if self.B is None else self.B.nrows

    @property
    def H(self) -> sp.csr_matrix | None:
        """Pressure prolongation: the linear-node block of P."""
        if self.P is None:
            return None
        return self.P[: self.nlin].tocsc()[:, : self.P_nlin_c].tocsr()

    P_nlin_c: int = 0


@dataclass
class Hierarchy:
    levels: list
    coarse_lu: tuple
    saddle: bool = False
    scalar: bool = False
    pinned: int = -1          # coarsest pressure DOF pinned (singular Stokes), -1 if none

    @property
    def L(self) -> int:
        return len(self.levels) - 1

    def sizes(self):
        return [lev.n for lev in self.levels]


def setup(A: BlockCSR, nlin: int, nquad: int, *, B: BlockCSR | None = None,
          C: BlockCSR | None = None, singular: bool = False, separate: bool = True,
          coarse_max: int = 300, max_levels: int = 10, coloured: bool = True) -> Hierarchy:
    """Build the level hierarchy (Section 3.2) and the coarsest LU."""
    levels = [Level(A, nlin, nquad, B=B, C=C)]
    saddle = B is not None
    while True:
        lev = levels[-1]
        dofs = 3 * lev.n + lev.npres
        if dofs <= coarse_max or len(levels) == max_levels:
            break
        P, ncl, ncq = split_level(lev.A, lev.nlin, lev.nquad, separate)
        if P.shape[1] > 0.9 * lev.n:
            break
        lev.P = P
        lev.P_nlin_c = ncl
        Ac = galerkin(lev.A, P, P)
        nxt = Level(Ac, ncl, ncq)
        if saddle:
            H = lev.H
            nxt.B = galerkin(lev.B, H, P)
            nxt.C = galerkin(lev.C, H, H) if lev.C is not None else None
        levels.append(nxt)
    for lev in levels:
        lev.dinv = np.linalg.inv(lev.A.diag_blocks())
        ip, ix = lev.A.indptr, lev.A.indices
        lev.colors = cloops.greedy_colour(ip, ix)
        lev.order_fwd = np.lexsort((np.arange(lev.n), lev.colors)) if coloured else np.arange(lev.n)
        lev.order_bwd = lev.order_fwd[::-1].copy() if coloured else np.arange(lev.n)[::-1].copy()
    h = Hierarchy(levels, None, saddle=saddle)
    Kc = coarse_matrix(levels[-1])
    if saddle and singular:
        h.pinned = Kc.shape[0] - 1
        Kc[h.pinned, :] = 0.0
        Kc[:, h.pinned] = 0.0
        Kc[h.pinned, h.pinned] = 1.0
    h.coarse_lu = sla.lu_factor(Kc)
    return h


def coarse_matrix(lev: Level) -> np.ndarray:
    A = lev.A.dense()
    if lev.B is None:
        return A
    B = lev.B.dense()
    C = lev.C.dense() if lev.C is not None else np.zeros((B.shape[0], B.shape[0]))
    return np.block([[A, B.T], [B, -C]])


def coarse_solve(h: Hierarchy, b: np.ndarray) -> np.ndarray:
    rhs = b.copy()
    if h.pinned >= 0:
        rhs[h.pinned] = 0.0
    return sla.lu_solve(h.coarse_lu, rhs)


# --------------------------------------------------------------------------
# smoothers (Section 3.3)
# --------------------------------------------------------------------------
def jacobi(lev: Level, b: np.ndarray, x: np.ndarray, omega: float) -> np.ndarray:
    """Damped block Jacobi: x + omega D_b^{-1} (b - A x)."""
    r = b - lev.A.matvec(x)
    return x + omega * np.einsum("nij,nj->ni", lev.dinv, r)


def gauss_seidel(lev: Level, b: np.ndarray, x: np.ndarray, forward: bool) -> np.ndarray:
    """One block Gauss-Seidel sweep in the level's node order (colours or index)."""
    x = np.ascontiguousarray(x, dtype=np.float64).copy()
    order = lev.order_fwd if forward else lev.order_bwd
    cloops.block_gs(order, lev.A.indptr, lev.A.indices, lev.A.vals, lev.dinv,
                    np.ascontiguousarray(b), x)
    return x


@dataclass
class Smoother:
    """Smoother choice in the paper's naming: 'JA-1-1-0.5', 'GS-1-1', 'sGS-1-1',
    'BS-1-1' (Braess-Sarazin). pre/post counts, JA damping, sGS parameters."""
    kind: str = "GS"
    pre: int = 1
    post: int = 1
    omega: float = 0.5            # JA damping (Section 4.2: 0.5)
    sgs_omega: float = 0.125      # sGS pressure parameter (Section 4.4)
    sgs_damping: float = 0.5      # sGS M_A = damped block Jacobi with damping 0.5
    omegas: tuple | None = None   # per-level JA damping (overrides omega)
    # post-smoothing GS sweeps forward like the pre-smoothing ones. Reading of
    # Section 4: under CG the cycle must be symmetric (forward pre, backward
    # post), while the stand-alone solver tables follow same-direction sweeps
    # (with backward post-sweeps they would need about 2.5x the iterations)
    post_forward: bool = False
    # sGS (2,2) block: -omega^{-1} diag(B M_A^{-1} B^T + C) (reading R14) when
    # True, the literal -omega^{-1} I of Section 3.3 when False
    sgs_scaled: bool = True

    @staticmethod
    def parse(name: str) -> "Smoother":
        parts = name.split("-")
        kind = {"JA": "JA", "GS": "GS", "sGS": "SGS", "BS": "BS", "Braess": "BS", "Vanka": "VANKA"}[parts[0]]
        if parts[0] == "Braess":
            parts = ["BS"] + parts[2:]
        s = Smoother(kind, int(parts[1]), int(parts[2]))
        if kind in ("JA", "VANKA") and len(parts) > 3:
            s.omega = float(parts[3])
        elif kind == "VANKA":
            s.omega = VANKA_OMEGA
        return s

    def level_omega(self, l: int) -> float:
        if self.omegas is not None:
            return float(self.omegas[min(l, len(self.omegas) - 1)])
        return self.omega


def smooth_spd(h: Hierarchy, l: int, sm: Smoother, b, x, pre: bool):
    lev = h.levels[l]
    steps = sm.pre if pre else sm.post
    for _ in range(steps):
        if sm.kind == "JA":
            x = jacobi(lev, b, x, sm.level_omega(l))
        elif sm.kind == "GS":
            x = gauss_seidel(lev, b, x, forward=pre or sm.post_forward)
        else:
            raise ValueError(sm.kind)
    return x


def saddle_residual(lev: Level, f, g, u, p):
    """[f - A u - B^T p ; g - B u + C p]."""
    ru = f - lev.A.matvec(u) - lev.B.transpose().matvec(p.reshape(-1, 1))
    rp = g - lev.B.matvec(u)[:, 0]
    if lev.C is not None:
        rp = rp + lev.C.matvec(p.reshape(-1, 1))[:, 0]
    return ru, rp


def sgs_pressure_diag(lev: Level, damping: float) -> np.ndarray:
    """diag(B M_A^{-1} B^T + C) with M_A^{-1} = damping * D_b^{-1}."""
    rows = lev.B.row_of()
    bv = lev.B.vals[:, 0, :]                               # (nnz, 3)
    q = np.einsum("ki,kij,kj->k", bv, lev.dinv[lev.B.indices], bv)
    d = damping * np.bincount(rows, weights=q, minlength=lev.npres)
    if lev.C is not None:
        d = d + lev.C.diag_blocks()[:, 0, 0]
    return d


def sgs_step(lev: Level, sm: Smoother, f, g, u, p):
    """Segregated Gauss-Seidel (Uzawa) step, Section 3.3:
    K_hat = [[M_A, 0], [B, -omega^{-1} S_d]], M_A = damped block Jacobi (0.5).

    Reading: the paper writes the (2,2) block as -omega^{-1} I with
    omega = 0.125; taken literally the pressure update does not scale with the
    mesh (B ~ h^2, so B M_A^{-1} B^T ~ h^3) and FGMRES needs several times
    the paper's iterations. The block is read as -omega^{-1} S_d with
    S_d = diag(B M_A^{-1} B^T + C), omega = 0.125; ``sm.sgs_scaled = False``
    gives the literal form.
    Solving K_hat [du; dp] = [r_u; r_p]: du = M_A^{-1} r_u,
    dp = omega S_d^{-1} (B du - r_p).
    """
    ru, rp = saddle_residual(lev, f, g, u, p)
    du = sm.sgs_damping * np.einsum("nij,nj->ni", lev.dinv, ru)
    dp = sm.sgs_omega * (lev.B.matvec(du)[:, 0] - rp)
    if sm.sgs_scaled:
        if lev.sgs_diag is None:
            lev.sgs_diag = sgs_pressure_diag(lev, sm.sgs_damping)
        dp = dp / lev.sgs_diag
    return u + du, p + dp


def bs_step(lev: Level, sm: Smoother, f, g, u, p):
    """Braess-Sarazin step: K_hat = [[A_hat, B^T], [B, B A_hat^{-1} B^T - S_hat]].

    A_hat = 2 D with D the (scalar) diagonal of A. Solving K_hat [du; dp] = r:
    S_hat dp = B A_hat^{-1} r_u - r_p, du = A_hat^{-1} (r_u - B^T dp), where
    S_hat^{-1} is one V(1,1) Gauss-Seidel cycle of the scalar AMG hierarchy of
    S = C + B A_hat^{-1} B^T (zero initial guess). Pinned against the dense
    block formula, and the inner cycle against its dense two-grid definition
    (triangular solves for the coloured sweeps, exact coarsest solve).
    """
    ru, rp = saddle_residual(lev, f, g, u, p)
    ahat_inv = 1.0 / (2.0 * np.einsum("nii->ni", lev.A.diag_blocks()))
    du0 = ahat_inv * ru
    rs = lev.B.matvec(du0)[:, 0] - rp
    dp = scalar_vcycle(lev.schur, 0, rs, np.zeros_like(rs))
    du = ahat_inv * (ru - lev.B.transpose().matvec(dp.reshape(-1, 1)))
    return u + du, p + dp


# --------------------------------------------------------------------------
# multiplicative Vanka (Section 3.3)
# --------------------------------------------------------------------------
VANKA_OMEGA = 0.8   # damping of the local corrections (the paper gives no value; reading R15)


@dataclass
class VankaPatches:
    nodes: list            # velocity nodes of patch i (sorted)
    dofs: list             # saddle-vector indices: 3 * node + c for every node, then the pressure
    order: np.ndarray      # processing order: by colour, then index
    colors: np.ndarray
    K: sp.csr_matrix       # the level's saddle matrix [[A, B^T], [B, -C]]


def saddle_matrix(lev: Level) -> sp.csr_matrix:
    Bs = lev.B.scipy()
    C = lev.C.scipy() if lev.C is not None else sp.csr_matrix((lev.npres, lev.npres))
    return sp.bmat([[lev.A.scipy(), Bs.T], [Bs, -C]], format="csr")


def vanka_patches(lev: Level) -> VankaPatches:
    """Patch i holds pressure DOF i and every velocity DOF of the nodes coupled
    to it through B (the structural pattern of B_ll and B_lq). Two patches may
    be processed at the same time when they share no velocity node, A couples
    none of their nodes and C does not couple their pressures: then the
    multiplicative sweep in (colour, index) order equals the sequential sweep
    in that order. Colours: greedy first-fit in index order on that conflict
    graph (reading R19)."""
    npres, n = lev.npres, lev.n
    nodes = [lev.B.indices[lev.B.indptr[i]:lev.B.indptr[i + 1]].copy() for i in range(npres)]
    N = sp.csr_matrix((np.ones(lev.B.nnz), lev.B.indices, lev.B.indptr), shape=(npres, n))
    conf = (N @ lev.A.pattern() @ N.T).tocsr()
    if lev.C is not None:
        conf = (conf + lev.C.pattern()).tocsr()
    conf.sort_indices()
    colors = cloops.greedy_colour(conf.indptr, conf.indices)
    order = np.lexsort((np.arange(npres), colors))
    nv = 3 * n
    dofs = [np.concatenate([(3 * nd[:, None] + np.arange(3)[None, :]).ravel(), [nv + i]]) for i, nd in enumerate(nodes)]
    return VankaPatches(nodes, dofs, order, colors, saddle_matrix(lev))


def vanka_step(lev: Level, sm: Smoother, f, g, u, p):
    """One multiplicative Vanka sweep: for every patch in order, the local
    system (the saddle matrix restricted to the patch) is solved for the
    current residual on the patch, and omega times the correction is added."""
    if lev.vanka is None:
        lev.vanka = vanka_patches(lev)
    V = lev.vanka
    x = np.concatenate([np.asarray(u, dtype=np.float64).ravel(), np.asarray(p, dtype=np.float64)])
    b = np.concatenate([np.asarray(f, dtype=np.float64).ravel(), np.asarray(g, dtype=np.float64)])
    K = V.K
    for i in V.order:
        idx = V.dofs[i]
        r = b[idx] - K[idx] @ x
        Ki = K[idx][:, idx].toarray()
        x[idx] += sm.omega * np.linalg.solve(Ki, r)
    nv = 3 * lev.n
    return x[:nv].reshape(-1, 3), x[nv:]


# --------------------------------------------------------------------------
# scalar AMG on the Braess-Sarazin Schur complements
# --------------------------------------------------------------------------
def schur_operator(lev: Level) -> BlockCSR:
    """S = C + B (2D)^{-1} B^T on the pressure nodes (1x1 blocks, structural pattern)."""
    d = 2.0 * np.einsum("nii->ni", lev.A.diag_blocks()).ravel()
    Bs = lev.B.scipy()
    S = Bs @ sp.diags(1.0 / d) @ Bs.T
    Bp = lev.B.pattern()
    pat = (Bp @ Bp.T).tocsr()
    if lev.C is not None:
        S = S + lev.C.scipy()
        pat = (pat + lev.C.pattern()).tocsr()
    pat.sort_indices()
    Sc = S.tocoo()
    out = BlockCSR(pat.indptr.astype(np.int64), pat.indices.astype(np.int64),
                   np.zeros((pat.nnz, 1, 1)), pat.shape[1])
    skeys = np.repeat(np.arange(pat.shape[0]), np.diff(pat.indptr)).astype(np.int64) * pat.shape[1] + pat.indices
    vkeys = Sc.row.astype(np.int64) * pat.shape[1] + Sc.col
    pos = np.searchsorted(skeys, vkeys)
    out.vals[pos, 0, 0] = Sc.data
    return out


@dataclass
class ScalarLevel:
    S: BlockCSR
    H: sp.csr_matrix | None
    order_fwd: np.ndarray
    order_bwd: np.ndarray


def schur_hierarchy(h: Hierarchy, l: int):
    """Scalar hierarchy S_l, H^T S_l H, ... down to the saddle coarsest level."""
    S = schur_operator(h.levels[l])
    out = []
    for k in range(l, h.L + 1):
        lev = h.levels[k]
        H = lev.H if k < h.L else None
        col = cloops.greedy_colour(S.indptr, S.indices)
        fwd = np.lexsort((np.arange(S.nrows), col))
        out.append(ScalarLevel(S, H, fwd, fwd[::-1].copy()))
        if H is None:
            break
        S = galerkin(S, H, H)
    Sd = out[-1].S.dense()
    if h.pinned >= 0:
        # the constant pressure is in the kernel of the cavity's Schur complement
        Sd[-1, :] = 0.0
        Sd[:, -1] = 0.0
        Sd[-1, -1] = 1.0
    return out, sla.lu_factor(Sd), h.pinned >= 0


def scalar_vcycle(sh, k: int, b: np.ndarray, x: np.ndarray) -> np.ndarray:
    levels, lu, pinned = sh
    lev = levels[k]
    S = lev.S
    if k == len(levels) - 1:
        rhs = b.copy()
        if pinned:
            rhs[-1] = 0.0
        return sla.lu_solve(lu, rhs)
    x = x.copy()
    cloops.scalar_gs(lev.order_fwd, S.indptr, S.indices, S.vals.ravel(), b, x)
    r = b - S.matvec(x.reshape(-1, 1))[:, 0]
    xc = scalar_vcycle(sh, k + 1, lev.H.T @ r, np.zeros(lev.H.shape[1]))
    x = x + lev.H @ xc
    cloops.scalar_gs(lev.order_bwd, S.indptr, S.indices, S.vals.ravel(), b, x)
    return x


def prepare_bs(h: Hierarchy) -> None:
    for l in range(h.L):
        h.levels[l].schur = schur_hierarchy(h, l)


# --------------------------------------------------------------------------
# Algorithm 1
# --------------------------------------------------------------------------
def cycle(h: Hierarchy, l: int, sm: Smoother, b: np.ndarray, x: np.ndarray, nu: int = 1) -> np.ndarray:
    """Algorithm 1 for an SPD hierarchy: AMG(K_l, x_l, b_l) with nu recursive
    calls (pinned for nu = 1 and 2 by the dense recursive error operator)."""
    lev = h.levels[l]
    x = smooth_spd(h, l, sm, b, x, pre=True)
    r = b - lev.A.matvec(x)
    bc = (lev.P.T @ r).reshape(-1, 3)
    if l + 1 == h.L:
        xc = coarse_solve(h, bc.ravel()).reshape(-1, 3)
    else:
        xc = np.zeros_like(bc)
        for _ in range(nu):
            xc = cycle(h, l + 1, sm, bc, xc, nu)
    x = x + lev.P @ xc
    return smooth_spd(h, l, sm, b, x, pre=False)


def saddle_cycle(h: Hierarchy, l: int, sm: Smoother, f, g, u, p, nu: int = 1):
    """Algorithm 1 for the saddle hierarchy with the sGS, BS or Vanka smoother
    (pinned by the dense error operator S (I - P K_c^{-1} P^T K) S)."""
    lev = h.levels[l]
    step = {"SGS": sgs_step, "BS": bs_step, "VANKA": vanka_step}[sm.kind]
    for _ in range(sm.pre):
        u, p = step(lev, sm, f, g, u, p)
    ru, rp = saddle_residual(lev, f, g, u, p)
    H = lev.H
    fc = (lev.P.T @ ru).reshape(-1, 3)
    gc = H.T @ rp
    if l + 1 == h.L:
        nv = fc.shape[0]
        sol = coarse_solve(h, np.concatenate([fc.ravel(), gc]))
        uc, pc = sol[: 3 * nv].reshape(-1, 3), sol[3 * nv:]
    else:
        uc, pc = np.zeros_like(fc), np.zeros_like(gc)
        for _ in range(nu):
            uc, pc = saddle_cycle(h, l + 1, sm, fc, gc, uc, pc, nu)
    u = u + lev.P @ uc
    p = p + H @ pc
    for _ in range(sm.post):
        u, p = step(lev, sm, f, g, u, p)
    return u, p


def preconditioner(h: Hierarchy, sm: Smoother, cycles: int = 1, nu: int = 1):
    """z = M^{-1} r: ``cycles`` successive applications of Algorithm 1 from zero
    (reading R17; two cycles square the error operator of one)."""
    if not h.saddle:
        def apply(r):
            r = np.asarray(r).reshape(-1, 3)
            if h.L == 0:
                return coarse_solve(h, r.ravel()).reshape(-1, 3)
            x = np.zeros_like(r)
            for _ in range(cycles):
                x = cycle(h, 0, sm, r, x, nu)
            return x
        return apply
    nv = h.levels[0].n

    def apply_saddle(r):
        f, g = r[: 3 * nv].reshape(-1, 3), r[3 * nv:]
        u, p = np.zeros_like(f), np.zeros_like(g)
        for _ in range(cycles):
            u, p = saddle_cycle(h, 0, sm, f, g, u, p, nu)
        return np.concatenate([u.ravel(), p])
    return apply_saddle


def operator_complexity(h: Hierarchy) -> float:
    nnz = [lev.A.nnz for lev in h.levels]
    return sum(nnz) / nnz[0]


def structural_sizes(pattern: BlockCSR, nlin: int, nquad: int, *, separate: bool = True,
                     coarse_max: int = 300, max_levels: int = 10):
    """Level sizes from the structural pattern alone (values play no part in
    the coarsening): list of (nlin, nquad) per level (nquad = 0 when not separate)."""
    M = BlockCSR(pattern.indptr, pattern.indices, np.ones((pattern.nnz, 1, 1)), pattern.ncols)
    sizes = [(nlin, nquad)]
    while True:
        n = nlin + nquad
        if 3 * n <= coarse_max or len(sizes) == max_levels:
            break
        P, ncl, ncq = split_level(M, nlin, nquad, separate)
        if P.shape[1] > 0.9 * n:
            break
        Pp = sp.csr_matrix((np.ones(P.nnz), P.indices, P.indptr), shape=P.shape)
        S = (Pp.T @ M.pattern() @ Pp).tocsr()
        S.sort_indices()
        M = BlockCSR(S.indptr.astype(np.int64), S.indices.astype(np.int64), np.ones((S.nnz, 1, 1)), S.shape[1])
        nlin, nquad = ncl, ncq
        sizes.append((nlin, nquad))
    return sizes
