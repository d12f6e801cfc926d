"""Input systems for the library: the paper's model problems on cube meshes.

Section 2 of the paper defines the systems the method solves (vector
Laplacian, pure-displacement elasticity, mixed elasticity and Stokes with a
hierarchical quadratic basis, Taylor-Hood for the mixed forms). This module
builds them for the synthetic workloads and hands the library host arrays in
the C ABI's layout. It is the harness side of the problem generation: the
element integrals use a 4-point Gauss rule of degree 2 (exact here, since
every integrand is a quadratic polynomial on each tetrahedron), written
independently of the test oracle, which integrates in closed form.

Conventions shared with the oracle because the method depends on them (the
coarsening is order dependent): vertex (i, j, k) of the n^3 lattice has id
i + (n+1)(j + (n+1)k); nodes are the vertices, then the edges sorted by their
(smaller, larger) vertex ids; each cube is split into the 6 Kuhn tetrahedra
(with ``mirrored`` the split is reflected in the upper half of each axis).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass

import numpy as np

import synth

# edges of a tetrahedron carrying phi_5 .. phi_10 (Section 2.3)
_TET_EDGES = np.array([(0, 1), (1, 2), (2, 3), (0, 2), (0, 3), (1, 3)])

# degree-2 Gauss rule on a tetrahedron: 4 points, barycentric (a, b, b, b)
_QA = (5.0 + 3.0 * math.sqrt(5.0)) / 20.0
_QB = (5.0 - math.sqrt(5.0)) / 20.0
_QLAM = np.full((4, 4), _QB) + np.eye(4) * (_QA - _QB)
_QW = np.full(4, 0.25)


@dataclass
class CubeMesh:
    n: int
    xyz: np.ndarray        # (nv, 3)
    tet: np.ndarray        # (nt, 4)
    edge: np.ndarray       # (ne, 2)
    tnode: np.ndarray      # (nt, 10)

    @property
    def nv(self):
        return self.xyz.shape[0]

    @property
    def ne(self):
        return self.edge.shape[0]


def cube_mesh(n: int, mirrored: bool = False) -> CubeMesh:
    s = n + 1
    idx = np.arange(s ** 3)
    xyz = np.stack([idx % s, (idx // s) % s, idx // (s * s)], axis=1) / n
    cubes = np.array(list(itertools.product(range(n), repeat=3)))[:, ::-1]   # (i, j, k), i fastest
    cubes = cubes[np.lexsort((cubes[:, 0], cubes[:, 1], cubes[:, 2]))]
    flip = (2 * cubes >= n) if mirrored else np.zeros_like(cubes, dtype=bool)
    origin = cubes + flip
    sign = np.where(flip, -1, 1)
    tets = np.empty((cubes.shape[0], 6, 4), dtype=np.int64)
    for t, order in enumerate(itertools.permutations(range(3))):
        corner = origin.copy()
        tets[:, t, 0] = corner @ np.array([1, s, s * s])
        for step, axis in enumerate(order, start=1):
            corner[:, axis] += sign[:, axis]
            tets[:, t, step] = corner @ np.array([1, s, s * s])
    tet = tets.reshape(-1, 4)
    ends = np.sort(np.concatenate([tet[:, e] for e in _TET_EDGES]), axis=1)
    code = np.unique(ends[:, 0] * s ** 3 + ends[:, 1])
    edge = np.stack([code // s ** 3, code % s ** 3], axis=1)
    lo = np.minimum(tet[:, _TET_EDGES[:, 0]], tet[:, _TET_EDGES[:, 1]])
    hi = np.maximum(tet[:, _TET_EDGES[:, 0]], tet[:, _TET_EDGES[:, 1]])
    enode = s ** 3 + np.searchsorted(code, lo * s ** 3 + hi)
    return CubeMesh(n, xyz, tet, edge, np.concatenate([tet, enode], axis=1))


# ---------------------------------------------------------------- integrals
def _geometry(mesh: CubeMesh, tets: np.ndarray):
    P = mesh.xyz[tets]
    J = P[:, 1:] - P[:, :1]                       # rows: edge vectors
    det = np.linalg.det(J)
    # barycentric gradients: J grad(lambda_i) = e_i for i = 1..3
    Gi = np.linalg.solve(J, np.broadcast_to(np.eye(3), J.shape)).transpose(0, 2, 1)
    G = np.concatenate([-Gi.sum(axis=1, keepdims=True), Gi], axis=1)
    return G, np.abs(det) / 6.0


def _basis_grads(G: np.ndarray) -> np.ndarray:
    """Gradients of phi_1..phi_10 at the quadrature points: (nt, Q, 10, 3)."""
    lin = np.broadcast_to(G[:, None], (G.shape[0], 4, 4, 3))
    p, q = _TET_EDGES[:, 0], _TET_EDGES[:, 1]
    quad = 4.0 * (_QLAM[None, :, p, None] * G[:, None, q, :] + _QLAM[None, :, q, None] * G[:, None, p, :])
    return np.concatenate([lin, quad], axis=2)


def _element_scalar_laplace(G, vol):
    """sum_q w grad phi_k . grad phi_m per element, (nt, 10, 10)."""
    dphi = _basis_grads(G)                                    # (nt, Q, 10, 3)
    nt, nq = dphi.shape[0], dphi.shape[1]
    w = vol[:, None] * _QW[None, :]
    X = dphi.transpose(0, 2, 1, 3).reshape(nt, 10, nq * 3)
    Xw = (dphi * w[:, :, None, None]).transpose(0, 2, 1, 3).reshape(nt, 10, nq * 3)
    return np.matmul(Xw, np.swapaxes(X, 1, 2))


def _element_blocks(G, vol, kind, lam, mu):
    dphi = _basis_grads(G)                                    # (nt, Q, 10, 3)
    nt = dphi.shape[0]
    w = vol[:, None] * _QW[None, :]                           # (nt, Q)
    # H[t,k,m,c,d] = sum_q w d_c phi_k d_d phi_m
    D = dphi.reshape(nt, 4, 30)
    H = np.matmul(np.swapaxes(D * w[:, :, None], 1, 2), D).reshape(nt, 10, 3, 10, 3)
    H = H.transpose(0, 1, 3, 2, 4)
    lap = np.trace(H, axis1=3, axis2=4)
    I3 = np.eye(3)
    if kind == "laplace":
        return lap[..., None, None] * I3
    sym = mu * (lap[..., None, None] * I3 + np.swapaxes(H, 3, 4))
    if kind == "elastic":
        return sym + lam * H
    return sym                                                # 2 mu eps:eps


def _pattern(rows, cols, nrows, ncols):
    key = rows.astype(np.int64) * ncols + cols
    uniq, where = np.unique(key, return_inverse=True)
    r = uniq // ncols
    rowptr = np.searchsorted(r, np.arange(nrows + 1)).astype(np.int32)
    return rowptr, (uniq % ncols).astype(np.int32), where.ravel()


def _accumulate(where, vals, nnz):
    flat = vals.reshape(vals.shape[0], -1)
    out = np.empty((nnz, flat.shape[1]))
    for p in range(flat.shape[1]):
        out[:, p] = np.bincount(where, weights=flat[:, p], minlength=nnz)
    return out


def _batches(nt, size=24576):
    return [(a, min(nt, a + size)) for a in range(0, nt, size)]


def velocity_operator(mesh: CubeMesh, kind: str, lam=0.0, mu=1.0, scalar=False):
    N = mesh.nv + mesh.ne
    T = mesh.tnode
    rows = np.repeat(T, 10, axis=1).ravel()
    cols = np.tile(T, (1, 10)).ravel()
    rowptr, col, where = _pattern(rows, cols, N, N)
    width = 1 if scalar else 9
    val = np.zeros((col.shape[0], width))
    for a, b in _batches(T.shape[0]):
        G, vol = _geometry(mesh, mesh.tet[a:b])
        if scalar and kind == "laplace":
            K = _element_scalar_laplace(G, vol)
        else:
            K = _element_blocks(G, vol, kind, lam, mu)
            K = K[..., 0, 0] if scalar else K
        val += _accumulate(where[a * 100:b * 100], K.reshape(-1, width), col.shape[0])
    return rowptr, col, val


def divergence_operator(mesh: CubeMesh):
    """B[p, k] = -int lambda_p d_c psi_k (1x3 blocks), pressure rows = vertices."""
    T = mesh.tnode
    rows = np.repeat(mesh.tet, 10, axis=1).ravel()
    cols = np.tile(T, (1, 4)).ravel()
    rowptr, col, where = _pattern(rows, cols, mesh.nv, mesh.nv + mesh.ne)
    val = np.zeros((col.shape[0], 3))
    for a, b in _batches(T.shape[0]):
        G, vol = _geometry(mesh, mesh.tet[a:b])
        dphi = _basis_grads(G)
        w = vol[:, None] * _QW[None, :]
        Be = -np.einsum("tq,qp,tqkc->tpkc", w, _QLAM, dphi, optimize=True)
        val += _accumulate(where[a * 40:b * 40], Be.reshape(-1, 3), col.shape[0])
    return rowptr, col, val


def pressure_mass(mesh: CubeMesh, scale: float):
    rows = np.repeat(mesh.tet, 4, axis=1).ravel()
    cols = np.tile(mesh.tet, (1, 4)).ravel()
    rowptr, col, where = _pattern(rows, cols, mesh.nv, mesh.nv)
    val = np.zeros((col.shape[0], 1))
    for a, b in _batches(mesh.tet.shape[0]):
        _, vol = _geometry(mesh, mesh.tet[a:b])
        w = vol[:, None] * _QW[None, :]
        Me = scale * np.einsum("tq,qa,qb->tab", w, _QLAM, _QLAM)
        val += _accumulate(where[a * 16:b * 16], Me.reshape(-1, 1), col.shape[0])
    return rowptr, col, val


# ---------------------------------------------------------------- boundary data
def _dirichlet(mesh: CubeMesh, vmask: np.ndarray, g):
    """Lifting vector (vertex: g, edge: midpoint surplus) and Dirichlet node mask."""
    N = mesh.nv + mesh.ne
    lift = np.zeros((N, 3))
    mask = np.zeros(N, dtype=bool)
    mask[: mesh.nv] = vmask
    lift[: mesh.nv][vmask] = g(mesh.xyz[vmask])
    a, b = mesh.edge[:, 0], mesh.edge[:, 1]
    on = vmask[a] & vmask[b]
    mask[mesh.nv:] = on
    ea, eb = mesh.xyz[a[on]], mesh.xyz[b[on]]
    lift[mesh.nv:][on] = g(0.5 * (ea + eb)) - 0.5 * (g(ea) + g(eb))
    return lift, mask


def _block_matvec(rowptr, col, val, x, bs_out, bs_in):
    rows = np.repeat(np.arange(rowptr.shape[0] - 1), np.diff(rowptr))
    xb = x.reshape(-1, bs_in)[col]
    if val.shape[1] == 1 and bs_out == 3:
        contrib = val * xb
    else:
        contrib = np.einsum("kij,kj->ki", val.reshape(-1, bs_out, bs_in), xb)
    out = np.zeros((rowptr.shape[0] - 1, bs_out))
    for c in range(bs_out):
        out[:, c] = np.bincount(rows, weights=contrib[:, c], minlength=rowptr.shape[0] - 1)
    return out


def _eliminate(rowptr, col, val, rhs, lift, mask, scalar):
    b = rhs - _block_matvec(rowptr, col, val, lift, 3, 3)
    rows = np.repeat(np.arange(rowptr.shape[0] - 1), np.diff(rowptr))
    off = (mask[rows] | mask[col]) & (rows != col)
    val[off] = 0.0
    b[mask] = 0.0
    return b


def _face_x1_load(mesh: CubeMesh, traction: np.ndarray) -> np.ndarray:
    n, s = mesh.n, mesh.n + 1
    F = np.zeros((mesh.nv + mesh.ne, 3))
    j, k = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    v = lambda jj, kk: (n + s * jj + s * s * kk).ravel()
    tris = [np.stack([v(j, k), v(j + 1, k), v(j + 1, k + 1)], 1),
            np.stack([v(j, k), v(j, k + 1), v(j + 1, k + 1)], 1)]
    area = 0.5 / (n * n)
    for t, tri in enumerate(tris):
        share = traction[:, :, t, :].reshape(-1, 3) * (area / 3.0)
        for c in range(3):
            np.add.at(F, tri[:, c], share)
        code = np.concatenate([mesh.edge[:, 0:1] * s ** 3 + mesh.edge[:, 1:2]]).ravel()
        for a, b in ((0, 1), (1, 2), (0, 2)):
            lo, hi = np.minimum(tri[:, a], tri[:, b]), np.maximum(tri[:, a], tri[:, b])
            np.add.at(F, mesh.nv + np.searchsorted(code, lo * s ** 3 + hi), share)
    return F


# ---------------------------------------------------------------- systems
@dataclass
class LinearSystem:
    """Host arrays in the layout of amg_system plus the right-hand side."""
    name: str
    n: int
    n_lin: int
    n_quad: int
    n_pres: int
    bs: int
    A_rowptr: np.ndarray
    A_col: np.ndarray
    A_val: np.ndarray            # flat: 9 (bs 3) or 1 (bs 1) doubles per entry
    rhs: np.ndarray              # flat: 3N (+ n_pres)
    lift: np.ndarray             # (N, 3)
    B_rowptr: np.ndarray | None = None
    B_col: np.ndarray | None = None
    B_val: np.ndarray | None = None
    C_rowptr: np.ndarray | None = None
    C_col: np.ndarray | None = None
    C_val: np.ndarray | None = None
    pressure_kernel: bool = False

    @property
    def nodes(self) -> int:
        return self.n_lin + self.n_quad

    @property
    def dofs(self) -> int:
        return 3 * self.nodes + self.n_pres


def _spd(name, mesh, kind, lam, mu, vmask, g, load, scalar):
    rowptr, col, val = velocity_operator(mesh, kind, lam, mu, scalar=scalar)
    lift, mask = _dirichlet(mesh, vmask, g)
    N = mesh.nv + mesh.ne
    rhs = np.zeros((N, 3)) if load is None else load
    if scalar:
        full = np.zeros((val.shape[0], 9))
        full[:, [0, 4, 8]] = val
        b = _eliminate(rowptr, col, full, rhs, lift, mask, False)
        val = full[:, :1].copy()
    else:
        b = _eliminate(rowptr, col, val, rhs, lift, mask, False)
    return LinearSystem(name, mesh.n, mesh.nv, mesh.ne, 0, 1 if scalar else 3, rowptr, col,
                        np.ascontiguousarray(val.ravel()), np.ascontiguousarray(b.ravel()), lift)


def laplace(n: int, workload: int = synth.LAPLACE_SMALL, i: int = 0, scalar: bool = True) -> LinearSystem:
    """Vector Laplacian, trigonometric Dirichlet data on x = 0, Neumann 0 elsewhere.
    scalar=True stores A_s with A = A_s (x) I_3 (bs = 1)."""
    mesh = cube_mesh(n)
    data = synth.trig_dirichlet(workload, i)
    vmask = mesh.xyz[:, 0] == 0.0
    return _spd(f"vector-laplacian-{n}", mesh, "laplace", 0.0, 1.0, vmask,
                lambda X: data(X[:, 1], X[:, 2]), None, scalar)


def laplace_rhs(sysm: LinearSystem, workload: int, i: int) -> np.ndarray:
    """Right-hand side of the same Laplacian for another Dirichlet data set."""
    mesh = cube_mesh(sysm.n)
    data = synth.trig_dirichlet(workload, i)
    lift, mask = _dirichlet(mesh, mesh.xyz[:, 0] == 0.0, lambda X: data(X[:, 1], X[:, 2]))
    rowptr, col, val = velocity_operator(mesh, "laplace", scalar=True)
    full = np.zeros((val.shape[0], 9))
    full[:, [0, 4, 8]] = val
    return np.ascontiguousarray(_eliminate(rowptr, col, full, np.zeros_like(lift), lift, mask, False).ravel())


def laplace_rhs_many(sysm: LinearSystem, workload: int, ids) -> list:
    """laplace_rhs for several Dirichlet data sets, the operator assembled
    once: with A = A_s (x) I_3 and zero load, the eliminated right-hand side
    is -A_s g on the free rows (g the lifting, nonzero on Dirichlet nodes
    only) and 0 on the Dirichlet rows."""
    import scipy.sparse as sps
    mesh = cube_mesh(sysm.n)
    rowptr, col, val = velocity_operator(mesh, "laplace", scalar=True)
    N = mesh.nv + mesh.ne
    A = sps.csr_matrix((np.asarray(val).ravel(), col, rowptr), shape=(N, N))
    out = []
    for i in ids:
        data = synth.trig_dirichlet(workload, i)
        lift, mask = _dirichlet(mesh, mesh.xyz[:, 0] == 0.0, lambda X, d=data: d(X[:, 1], X[:, 2]))
        rhs = -(A @ lift)
        rhs[mask] = 0.0
        out.append(np.ascontiguousarray(rhs.ravel()))
    return out


def elasticity(n: int, i: int = 0, E: float = 1.0, nu: float = 0.3,
               workload: int = synth.ELASTICITY) -> LinearSystem:
    """Pure-displacement elasticity, clamped x = 0, random traction on x = 1."""
    mesh = cube_mesh(n)
    lam, mu = synth.lame(E, nu)
    load = _face_x1_load(mesh, synth.face_traction(workload, i, n))
    vmask = mesh.xyz[:, 0] == 0.0
    return _spd(f"elasticity-{n}", mesh, "elastic", lam, mu, vmask,
                lambda X: np.zeros((X.shape[0], 3)), load, False)


def _saddle(name, mesh, mu, lam_inv, vmask, g, load, closed) -> LinearSystem:
    """[[A, B^T], [B, -C]] with A from 2 mu eps:eps, B = -int q div v,
    C = (1/lambda) int p q (absent for Stokes); Dirichlet velocity data
    eliminated symmetrically (B's Dirichlet columns cleared, g = -B lift)."""
    rowptr, col, val = velocity_operator(mesh, "stokesA", 0.0, mu)
    brow, bcol, bval = divergence_operator(mesh)
    lift, mask = _dirichlet(mesh, vmask, g)
    gp = -_block_matvec(brow, bcol, bval, lift, 1, 3)[:, 0]
    N = mesh.nv + mesh.ne
    f = _eliminate(rowptr, col, val, np.zeros((N, 3)) if load is None else load, lift, mask, False)
    bval[mask[bcol]] = 0.0
    sysm = LinearSystem(name, mesh.n, mesh.nv, mesh.ne, mesh.nv, 3, rowptr, col, np.ascontiguousarray(val.ravel()),
                        np.ascontiguousarray(np.concatenate([f.ravel(), gp])), lift,
                        B_rowptr=brow, B_col=bcol, B_val=np.ascontiguousarray(bval.ravel()),
                        pressure_kernel=bool(closed and lam_inv == 0.0))
    if lam_inv != 0.0:
        crow, ccol, cval = pressure_mass(mesh, lam_inv)
        sysm.C_rowptr, sysm.C_col, sysm.C_val = crow, ccol, np.ascontiguousarray(cval.ravel())
    return sysm


def mixed_elasticity(n: int, i: int = 0, E: float = 1.0, nu: float = 0.49999,
                     workload: int = synth.MIXED_ELAST) -> LinearSystem:
    """Mixed displacement-pressure elasticity (Section 2.1), clamped x = 0,
    random traction on x = 1; p = -lambda div u."""
    mesh = cube_mesh(n)
    lam, mu = synth.lame(E, nu)
    load = _face_x1_load(mesh, synth.face_traction(workload, i, n))
    return _saddle(f"mixed-elasticity-{n}", mesh, mu, 1.0 / lam, mesh.xyz[:, 0] == 0.0,
                   lambda X: np.zeros((X.shape[0], 3)), load, False)


def stokes_cavity(n: int, speed: float, mu: float = 0.5) -> LinearSystem:
    """Lid-driven Stokes cavity: u = (speed, 0, 0) on the open lid z = 1
    (the lid's rim is no-slip), u = 0 on the other faces. Kuhn split reflected
    in the upper half of each axis: on the plain split, tetrahedra with all
    vertices on the boundary carry spurious Taylor-Hood pressure modes."""
    mesh = cube_mesh(n, mirrored=True)
    X = mesh.xyz
    on_b = np.any((X == 0.0) | (X == 1.0), axis=1)

    def g(P):
        out = np.zeros((P.shape[0], 3))
        lid = (np.abs(P[:, 2] - 1.0) < 1e-12) & (P[:, 0] > 1e-12) & (P[:, 0] < 1 - 1e-12) \
            & (P[:, 1] > 1e-12) & (P[:, 1] < 1 - 1e-12)
        out[lid, 0] = speed
        return out
    return _saddle(f"stokes-cavity-{n}", mesh, mu, 0.0, on_b, g, None, True)


def paper_cube(n: int, kind: str = "laplace", lam: float = 1.73e6, mu: float = 1.15e6) -> LinearSystem:
    """Section 4.1's data: u = 0 on z = 0, u = (0, 0, 1) on z = 1, zero
    Neumann data elsewhere; kind "laplace", "elastic" or "mixed" (the mixed
    displacement-pressure form of Section 4.4, C = (1/lambda) mass)."""
    mesh = cube_mesh(n)
    z = mesh.xyz[:, 2]
    vmask = (z == 0.0) | (z == 1.0)

    def g(X):
        out = np.zeros((X.shape[0], 3))
        out[X[:, 2] == 1.0, 2] = 1.0
        return out
    if kind == "mixed":
        return _saddle(f"paper-mixed-{n}", mesh, mu, 1.0 / lam, vmask, g, None, False)
    return _spd(f"paper-{kind}-{n}", mesh, "laplace" if kind == "laplace" else "elastic", lam, mu,
                vmask, g, None, kind == "laplace")
