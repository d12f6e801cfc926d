"""Hierarchical quadratic (and Taylor-Hood) finite element systems, FP64.

Test infrastructure only (see ``oracle/__init__``).

Follows Section 2 of the paper:
* model problems: vector Laplacian, pure-displacement elasticity, mixed
  displacement-pressure elasticity, Stokes (Section 2.1);
* homogenised weak forms a(u,v), b(v,q) = -int q div v, c(p,q) = (1/lambda)
  int p q (0 for Stokes), F = int_GammaN g_N . v - a(g_D, v) (Section 2.2);
* hierarchical basis phi_1..4 = lambda_i, phi_5..10 = 4 lambda_a lambda_b over
  the tet's edges (Section 2.3); pressure: linear hat functions on all vertices;
* block systems A u = f (SPD) and [[A, B^T], [B, -C]] [u; p] = [f; g] with the
  DOF order [u_l; u_q] and [u_l; u_q; p_l] (Section 2.4).

All element integrals are exact: every integrand is a polynomial in the
barycentric coordinates and
    int_T lambda_1^a1 ... lambda_4^a4 dx = 6|T| a1! a2! a3! a4! / (a1+..+a4+3)!.
Gradients of the basis are linear in the barycentric coordinates, so the
stiffness integrals only need int lambda_a lambda_b = |T| (1 + delta_ab) / 20.

Dirichlet data (reading of Section 2.2's homogenisation): Dirichlet nodes are
kept in the system; the lifting vector g holds the interpolated data
(vertex: g(x); edge node: g(midpoint) - (g(a) + g(b)) / 2, the hierarchical
surplus); the right-hand side becomes F - K g; rows and columns of Dirichlet
nodes are cleared except their diagonal block, and their right-hand side is 0.
Cleared entries stay in the pattern as explicit zeros.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .mesh import LOCAL_EDGES, Mesh, face_triangles_x1, kuhn_mesh
from .sparse import BlockCSR, from_pairs, scatter_add


# --------------------------------------------------------------------------
# element geometry and basis gradients
# --------------------------------------------------------------------------
def tet_geometry(mesh: Mesh, tets: np.ndarray | None = None):
    """Barycentric gradients (nt, 4, 3) and volumes (nt,)."""
    T = mesh.tets if tets is None else tets
    X = mesh.coords[T]                                  # (nt, 4, 3)
    M = np.transpose(X[:, 1:] - X[:, :1], (0, 2, 1))    # columns x_i - x_0
    Minv = np.linalg.inv(M)                              # rows = grad lambda_1..3
    grads = np.concatenate([-Minv.sum(axis=1, keepdims=True), Minv], axis=1)
    vol = np.abs(np.linalg.det(M)) / 6.0
    return grads, vol


def basis_gradient_coeffs(grads: np.ndarray) -> np.ndarray:
    """alpha[t, k, d, a]: d/dx_d phi_k = sum_a alpha[t,k,d,a] lambda_a.

    Linear phi_k = lambda_k has a constant gradient g_k = g_k * sum_a lambda_a.
    Quadratic phi = 4 lambda_p lambda_q has gradient 4 (lambda_p g_q + lambda_q g_p).
    """
    nt = grads.shape[0]
    alpha = np.zeros((nt, 10, 3, 4))
    for k in range(4):
        alpha[:, k, :, :] = grads[:, k, :, None]
    for e, (p, q) in enumerate(LOCAL_EDGES):
        alpha[:, 4 + e, :, p] += 4.0 * grads[:, q, :]
        alpha[:, 4 + e, :, q] += 4.0 * grads[:, p, :]
    return alpha


def mass_p1(vol: np.ndarray) -> np.ndarray:
    """int_T lambda_a lambda_b = |T| (1 + delta_ab) / 20, shape (nt, 4, 4)."""
    return vol[:, None, None] * (np.ones((4, 4)) + np.eye(4))[None] / 20.0


def derivative_integrals(alpha: np.ndarray, vol: np.ndarray) -> np.ndarray:
    """D[t, k, c, m, d] = int_T d_c phi_k d_d phi_m."""
    nt = alpha.shape[0]
    M2 = mass_p1(vol)
    a = alpha.reshape(nt, 30, 4)
    D = np.matmul(np.matmul(a, M2), np.transpose(a, (0, 2, 1)))
    return D.reshape(nt, 10, 3, 10, 3)


# --------------------------------------------------------------------------
# element matrices of the bilinear forms (3x3 node blocks)
# --------------------------------------------------------------------------
def element_blocks(D: np.ndarray, kind: str, lam: float = 0.0, mu: float = 1.0) -> np.ndarray:
    """Element blocks K[t, k, m, c, d] for nodes k, m and components c, d.

    * 'laplace':  int grad u : grad v          -> delta_cd G_km
    * 'elastic':  int 2 mu eps:eps + lam div div -> mu (delta_cd G + D^{dc}) + lam D^{cd}
    * 'stokesA':  2 mu int eps:eps              -> mu (delta_cd G + D^{dc})
    with G_km = sum_c D[k,c,m,c] and D^{cd}_km = D[k,c,m,d].
    """
    G = np.einsum("tkcmc->tkm", D)
    eye = np.eye(3)
    Dcd = np.transpose(D, (0, 1, 3, 2, 4))          # [t, k, m, c, d] = D^{cd}
    Ddc = np.transpose(D, (0, 1, 3, 4, 2))          # [t, k, m, c, d] = D^{dc}
    if kind == "laplace":
        return G[..., None, None] * eye
    if kind == "elastic":
        return mu * (G[..., None, None] * eye + Ddc) + lam * Dcd
    if kind == "stokesA":
        return mu * (G[..., None, None] * eye + Ddc)
    raise ValueError(kind)


# --------------------------------------------------------------------------
# systems
# --------------------------------------------------------------------------
@dataclass
class SPDSystem:
    mesh: Mesh
    A: BlockCSR            # (N x N) 3x3 blocks, structural pattern
    b: np.ndarray          # (N, 3) homogenised right-hand side
    lift: np.ndarray       # (N, 3) Dirichlet lifting (zero off Gamma_D)
    dirichlet: np.ndarray  # (N,) bool

    @property
    def nlin(self) -> int:
        return self.mesh.nv

    @property
    def nquad(self) -> int:
        return self.mesh.ne


@dataclass
class SaddleSystem:
    mesh: Mesh
    A: BlockCSR            # velocity block, 3x3 blocks
    B: BlockCSR            # pressure rows x velocity nodes, 1x3 blocks
    C: BlockCSR | None     # pressure x pressure, 1x1 blocks (None for Stokes)
    f: np.ndarray          # (N, 3)
    g: np.ndarray          # (Np,)
    lift: np.ndarray
    dirichlet: np.ndarray
    singular: bool = False  # constant pressure in the kernel (all-Dirichlet Stokes)

    @property
    def nlin(self) -> int:
        return self.mesh.nv

    @property
    def nquad(self) -> int:
        return self.mesh.ne

    @property
    def npres(self) -> int:
        return self.mesh.nv


def _chunks(nt: int, size: int = 32768):
    for s in range(0, nt, size):
        yield s, min(nt, s + size)


def assemble_velocity_block(mesh: Mesh, kind: str, lam: float = 0.0, mu: float = 1.0) -> BlockCSR:
    T = mesh.tet_nodes
    nt = T.shape[0]
    rows = np.repeat(T, 10, axis=1).ravel()
    cols = np.tile(T, (1, 10)).ravel()
    N = mesh.nnodes
    A, pos = from_pairs(rows, cols, N, N, 3, 3)
    for s, e in _chunks(nt):
        grads, vol = tet_geometry(mesh, mesh.tets[s:e])
        D = derivative_integrals(basis_gradient_coeffs(grads), vol)
        K = element_blocks(D, kind, lam, mu)                 # (nt, 10, 10, 3, 3)
        scatter_add(A, pos[s * 100:e * 100], K.reshape(-1, 3, 3))
    return A


def assemble_divergence(mesh: Mesh) -> BlockCSR:
    """B[p, k] (1x3 block): -int lambda_p d_c psi_k, pressure p over the vertices."""
    T = mesh.tet_nodes
    nt = T.shape[0]
    rows = np.repeat(mesh.tets, 10, axis=1).ravel()
    cols = np.tile(T, (1, 4)).ravel()
    B, pos = from_pairs(rows, cols, mesh.nv, mesh.nnodes, 1, 3)
    for s, e in _chunks(nt):
        grads, vol = tet_geometry(mesh, mesh.tets[s:e])
        alpha = basis_gradient_coeffs(grads)                 # (nt, 10, 3, 4)
        M2 = mass_p1(vol)                                    # (nt, 4, 4)
        Be = -np.einsum("tpa,tkca->tpkc", M2, alpha)         # (nt, 4, 10, 3)
        scatter_add(B, pos[s * 40:e * 40], Be.reshape(-1, 1, 3))
    return B


def assemble_pressure_mass(mesh: Mesh, scale: float) -> BlockCSR:
    """C[p, q] = scale * int lambda_p lambda_q (scale = 1/lambda)."""
    nt = mesh.tets.shape[0]
    rows = np.repeat(mesh.tets, 4, axis=1).ravel()
    cols = np.tile(mesh.tets, (1, 4)).ravel()
    C, pos = from_pairs(rows, cols, mesh.nv, mesh.nv, 1, 1)
    for s, e in _chunks(nt):
        _, vol = tet_geometry(mesh, mesh.tets[s:e])
        scatter_add(C, pos[s * 16:e * 16], scale * mass_p1(vol).reshape(-1, 1, 1))
    return C


def traction_load_x1(mesh: Mesh, traction: np.ndarray) -> np.ndarray:
    """Load vector of a piecewise-constant traction on the face x = 1.

    traction has shape (n, n, 2, 3) (see ``face_triangles_x1``). On a triangle F,
    int_F lambda_i = |F|/3 and int_F 4 lambda_a lambda_b = |F|/3, so each of
    the triangle's 3 vertices and 3 edge nodes receives |F| g / 3.
    """
    F = np.zeros((mesh.nnodes, 3))
    tri = face_triangles_x1(mesh).reshape(-1, 3)
    t = traction.reshape(-1, 3)
    P = mesh.coords[tri]
    area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    share = (area / 3.0)[:, None] * t
    for a in range(3):
        np.add.at(F, tri[:, a], share)
    for a, b in ((0, 1), (1, 2), (0, 2)):
        np.add.at(F, mesh.edge_id(tri[:, a], tri[:, b]), share)
    return F


def interpolate_dirichlet(mesh: Mesh, mask_v: np.ndarray, func) -> tuple[np.ndarray, np.ndarray]:
    """Lifting vector and Dirichlet node mask for data func(points)->(k,3).

    mask_v marks the Dirichlet vertices; an edge node is Dirichlet when both of
    its vertices are. Vertex value g(x); edge value g(mid) - (g(a)+g(b))/2.
    """
    N = mesh.nnodes
    lift = np.zeros((N, 3))
    dmask = np.zeros(N, dtype=bool)
    vs = np.nonzero(mask_v)[0]
    dmask[vs] = True
    lift[vs] = func(mesh.coords[vs])
    ea, eb = mesh.edges[:, 0], mesh.edges[:, 1]
    es = np.nonzero(mask_v[ea] & mask_v[eb])[0]
    dmask[mesh.nv + es] = True
    mid = 0.5 * (mesh.coords[ea[es]] + mesh.coords[eb[es]])
    lift[mesh.nv + es] = func(mid) - 0.5 * (func(mesh.coords[ea[es]]) + func(mesh.coords[eb[es]]))
    return lift, dmask


def apply_dirichlet(A: BlockCSR, rhs: np.ndarray, lift: np.ndarray, dmask: np.ndarray) -> np.ndarray:
    """Homogenise: rhs - A lift, clear Dirichlet rows/cols (keep diagonal block)."""
    b = rhs - A.matvec(lift)
    rows = A.row_of()
    clear = (dmask[rows] | dmask[A.indices]) & (rows != A.indices)
    A.vals[clear] = 0.0
    b[dmask] = 0.0
    return b


def _vertex_mask(mesh: Mesh, axis: int, value: float) -> np.ndarray:
    return np.abs(mesh.coords[:, axis] - value) < 1e-12


# --------------------------------------------------------------------------
# problem builders
# --------------------------------------------------------------------------
def vector_laplacian(n: int, dirichlet_func, dirichlet_mask_v=None) -> SPDSystem:
    """-Delta u = 0, u = g_D on x=0 (default), zero Neumann elsewhere."""
    mesh = kuhn_mesh(n)
    A = assemble_velocity_block(mesh, "laplace")
    mask_v = _vertex_mask(mesh, 0, 0.0) if dirichlet_mask_v is None else dirichlet_mask_v(mesh)
    lift, dmask = interpolate_dirichlet(mesh, mask_v, dirichlet_func)
    b = apply_dirichlet(A, np.zeros((mesh.nnodes, 3)), lift, dmask)
    return SPDSystem(mesh, A, b, lift, dmask)


def laplace_trig(n: int, data) -> SPDSystem:
    """Vector Laplacian with trigonometric Dirichlet data g(y, z) on x=0."""
    return vector_laplacian(n, lambda X: data(X[:, 1], X[:, 2]))


def elasticity_traction(n: int, lam: float, mu: float, traction: np.ndarray) -> SPDSystem:
    """Pure-displacement elasticity, clamped x=0, traction on x=1."""
    mesh = kuhn_mesh(n)
    A = assemble_velocity_block(mesh, "elastic", lam, mu)
    mask_v = _vertex_mask(mesh, 0, 0.0)
    lift, dmask = interpolate_dirichlet(mesh, mask_v, lambda X: np.zeros((X.shape[0], 3)))
    b = apply_dirichlet(A, traction_load_x1(mesh, traction), lift, dmask)
    return SPDSystem(mesh, A, b, lift, dmask)


def paper_cube_bc(mesh: Mesh):
    """Section 4.1's data: u = 0 on z=0, u = (0,0,1) on z=1, Neumann 0 elsewhere."""
    bottom = _vertex_mask(mesh, 2, 0.0)
    top = _vertex_mask(mesh, 2, 1.0)

    def func(X):
        out = np.zeros((X.shape[0], 3))
        out[np.abs(X[:, 2] - 1.0) < 1e-12, 2] = 1.0
        return out
    return bottom | top, func


def paper_spd(n: int, kind: str, lam: float = 1.73e6, mu: float = 1.15e6) -> SPDSystem:
    mesh = kuhn_mesh(n)
    A = assemble_velocity_block(mesh, kind, lam, mu)
    mask_v, func = paper_cube_bc(mesh)
    lift, dmask = interpolate_dirichlet(mesh, mask_v, func)
    b = apply_dirichlet(A, np.zeros((mesh.nnodes, 3)), lift, dmask)
    return SPDSystem(mesh, A, b, lift, dmask)


def paper_mixed(n: int, lam: float = 1.73e6, mu: float = 1.15e6) -> "SaddleSystem":
    """Section 4.4: the mixed form of the elasticity problem on Section 4.1's data."""
    mesh = kuhn_mesh(n)
    mask_v, func = paper_cube_bc(mesh)
    return saddle_system(mesh, mu, 1.0 / lam, mask_v, func)


def saddle_system(mesh: Mesh, mu: float, lam_inv: float, mask_v: np.ndarray, func,
                  load: np.ndarray | None = None, closed: bool = False) -> SaddleSystem:
    """[[A, B^T], [B, -C]] for mixed elasticity (lam_inv = 1/lambda) or Stokes (0)."""
    A = assemble_velocity_block(mesh, "stokesA", 0.0, mu)
    B = assemble_divergence(mesh)
    C = assemble_pressure_mass(mesh, lam_inv) if lam_inv != 0.0 else None
    lift, dmask = interpolate_dirichlet(mesh, mask_v, func)
    F = np.zeros((mesh.nnodes, 3)) if load is None else load
    # f = F - A g - B^T 0 ; g_p = G - B g with G = 0 (Section 2.2)
    g = -B.matvec(lift)[:, 0]
    f = apply_dirichlet(A, F, lift, dmask)
    B.vals[dmask[B.indices]] = 0.0
    # closed: velocity Dirichlet data on the whole boundary; with C = 0 the
    # constant pressure is then in the kernel
    return SaddleSystem(mesh, A, B, C, f, g, lift, dmask, bool(closed and C is None))


def mixed_elasticity_traction(n: int, lam: float, mu: float, traction: np.ndarray) -> SaddleSystem:
    mesh = kuhn_mesh(n)
    mask_v = _vertex_mask(mesh, 0, 0.0)
    return saddle_system(mesh, mu, 1.0 / lam, mask_v, lambda X: np.zeros((X.shape[0], 3)),
                         traction_load_x1(mesh, traction))


def stokes_lid(n: int, speed: float, mu: float = 0.5) -> SaddleSystem:
    """Lid-driven cavity: u = (speed, 0, 0) on the open lid z=1 (rim no-slip), 0 elsewhere.

    Uses the mirrored Kuhn split (see ``kuhn_mesh``): with velocity Dirichlet
    data on the whole boundary the only pressure kernel is then the constant.
    """
    mesh = kuhn_mesh(n, mirrored=True)
    X = mesh.coords
    on_bdry = np.any((np.abs(X) < 1e-12) | (np.abs(X - 1.0) < 1e-12), axis=1)

    def func(P):
        out = np.zeros((P.shape[0], 3))
        lid = ((np.abs(P[:, 2] - 1.0) < 1e-12) & (P[:, 0] > 1e-12) & (P[:, 0] < 1 - 1e-12)
               & (P[:, 1] > 1e-12) & (P[:, 1] < 1 - 1e-12))
        out[lid, 0] = speed
        return out
    return saddle_system(mesh, mu, 0.0, on_bdry, func, closed=True)


def full_solution(sysm, x: np.ndarray) -> np.ndarray:
    """Undo the homogenisation: u = x + lifting."""
    return np.asarray(x).reshape(-1, 3) + sysm.lift


def lagrange_exact(mesh: Mesh, func) -> np.ndarray:
    """Hierarchical P2 coefficients interpolating func (exact for quadratics)."""
    lift, _ = interpolate_dirichlet(mesh, np.ones(mesh.nv, dtype=bool), func)
    return lift


def lame_from(E: float, nu: float) -> tuple[float, float]:
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


def integrate_monomial(vol: float, powers) -> float:
    """6|T| a1! a2! a3! a4! / (sum a + 3)!  (exact barycentric integral)."""
    num = 6.0 * vol * np.prod([math.factorial(int(a)) for a in powers])
    return num / math.factorial(int(sum(powers)) + 3)


def structural_pattern(mesh: Mesh) -> BlockCSR:
    """Node pattern of the P2 system (all node pairs sharing a tet), no values."""
    T = mesh.tet_nodes
    rows = np.repeat(T, 10, axis=1).ravel()
    cols = np.tile(T, (1, 10)).ravel()
    M, _ = from_pairs(rows, cols, mesh.nnodes, mesh.nnodes, 1, 1)
    return M
