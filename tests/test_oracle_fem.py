"""Pins of the oracle's mesh and finite element assembly against facts fixed
by the paper and by mathematics (exact counts, closed forms, patch tests)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fem, mesh as M
from oracle.sparse import BlockCSR


def _all_boundary(mesh):
    X = mesh.coords
    return np.any((np.abs(X) < 1e-12) | (np.abs(X - 1) < 1e-12), axis=1)


# ---------------------------------------------------------------- counts
@pytest.mark.parametrize("mirrored", [False, True])
def test_table1_counts(golden, mirrored):
    """Section 4.1 mesh table: cubes, nodes, midside nodes, DOF counts."""
    for n, cubes, nodes, mid, dof_e, dof_s in golden("table1_mesh_counts.txt"):
        n = int(n)
        if n > 16 and mirrored:
            continue
        m = M.kuhn_mesh(n, mirrored)
        assert m.tets.shape[0] == 6 * int(cubes)
        assert m.nv == int(nodes)
        assert m.ne == int(mid)
        assert 3 * m.nnodes == int(dof_e)
        assert 3 * m.nnodes + m.nv == int(dof_s)


@pytest.mark.parametrize("n,mirrored", [(1, False), (3, False), (4, True), (5, True)])
def test_mesh_topology(n, mirrored):
    m = M.kuhn_mesh(n, mirrored)
    bf = M.boundary_faces(m)
    nfaces = (4 * m.tets.shape[0] + bf.shape[0]) // 2
    # Euler characteristic of a ball: V - E + F - T = 1
    assert m.nv - m.ne + nfaces - m.tets.shape[0] == 1
    assert bf.shape[0] == 12 * n * n
    _, vol = fem.tet_geometry(m)
    assert np.all(vol > 0)
    assert abs(vol.sum() - 1.0) < 1e-12
    if mirrored:
        assert not _all_boundary(m)[m.tets].all(axis=1).any()


def test_face_triangles_are_boundary_faces():
    m = M.kuhn_mesh(3)
    tri = np.sort(M.face_triangles_x1(m).reshape(-1, 3), axis=1)
    bf = M.boundary_faces(m)
    key = lambda t: set(map(tuple, t))
    assert key(tri) <= key(bf)
    assert len(key(tri)) == 2 * 9


# ---------------------------------------------------------------- integrals
def test_exact_integration_vs_quadrature():
    """int lambda_a lambda_b = |T|(1+delta)/20 against a degree-2-exact rule
    (4-point Keast rule) and against the monomial formula."""
    m = M.kuhn_mesh(1)
    _, vol = fem.tet_geometry(m)
    a, b = 0.5854101966249685, 0.1381966011250105
    pts = np.array([[a, b, b, b], [b, a, b, b], [b, b, a, b], [b, b, b, a]])
    quad = np.einsum("qa,qb->ab", pts, pts) / 4.0
    assert np.allclose(fem.mass_p1(vol)[0] / vol[0], quad, atol=1e-15)
    assert abs(fem.integrate_monomial(1.0, (1, 1, 0, 0)) - 1 / 20) < 1e-15
    assert abs(fem.integrate_monomial(1.0, (2, 0, 0, 0)) - 1 / 10) < 1e-15


def test_quadratic_basis_gradient_coeffs():
    """grad(4 l_p l_q) = 4 (l_p grad l_q + l_q grad l_p), checked by finite
    differences of the basis functions at a random point of one tet."""
    m = M.kuhn_mesh(1)
    grads, _ = fem.tet_geometry(m, m.tets[:1])
    alpha = fem.basis_gradient_coeffs(grads)[0]
    X = m.coords[m.tets[0]]
    rng = np.random.default_rng(3)
    lam = rng.dirichlet(np.ones(4))
    x = lam @ X

    def bary(y):
        Mx = np.vstack([X.T, np.ones(4)])
        return np.linalg.solve(Mx, np.append(y, 1.0))

    def phi(y):
        l = bary(y)
        out = list(l)
        for p, q in M.LOCAL_EDGES:
            out.append(4 * l[p] * l[q])
        return np.array(out)

    h = 1e-6
    fd = np.stack([(phi(x + h * e) - phi(x - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
    an = np.einsum("kda,a->kd", alpha, lam)
    assert np.allclose(fd, an, atol=1e-7)


# ---------------------------------------------------------------- structure
def test_laplace_constants_and_p1_stencil():
    n = 4
    m = M.kuhn_mesh(n)
    A = fem.assemble_velocity_block(m, "laplace")
    Ad = A.dense()
    assert np.abs(Ad - Ad.T).max() < 1e-15
    one = np.zeros((m.nnodes, 3))
    one[: m.nv] = 1.0                       # the constant function: vertex values 1
    assert np.abs(A.matvec(one)).max() < 1e-14
    # K_ll of the hierarchical basis is the P1 stiffness; on the Kuhn mesh its
    # interior rows are the 7-point stencil h * (6, -1 x 6).
    h = 1.0 / n
    v = M.vid(n, 2, 2, 2)
    Kll = Ad[0::3, 0::3][: m.nv, : m.nv]
    row = Kll[v]
    nz = np.nonzero(np.abs(row) > 1e-14)[0]
    expect = {v: 6 * h}
    for d in (1, n + 1, (n + 1) ** 2):
        expect[v + d] = -h
        expect[v - d] = -h
    assert set(nz) == set(expect)
    for k, val in expect.items():
        assert abs(row[k] - val) < 1e-14


def test_elasticity_rigid_body_kernel():
    m = M.kuhn_mesh(2)
    lam, mu = fem.lame_from(1.0, 0.3)
    A = fem.assemble_velocity_block(m, "elastic", lam, mu)
    modes = []
    for t in np.eye(3):
        v = np.zeros((m.nnodes, 3))
        v[: m.nv] = t
        modes.append(v)
    for w in np.eye(3):
        v = np.zeros((m.nnodes, 3))
        v[: m.nv] = np.cross(w, m.coords)    # linear field: no edge surplus
        modes.append(v)
    scale = np.abs(A.vals).max()
    for v in modes:
        assert np.abs(A.matvec(v)).max() < 1e-14 * scale
    Ad = A.dense()
    assert np.abs(Ad - Ad.T).max() < 1e-15 * scale
    ev = np.linalg.eigvalsh(Ad)
    assert np.sum(np.abs(ev) < 1e-12 * scale) == 6


def test_divergence_of_interior_and_mass():
    m = M.kuhn_mesh(3)
    B = fem.assemble_divergence(m)
    C = fem.assemble_pressure_mass(m, 1.0)
    assert abs(C.dense().sum() - 1.0) < 1e-14          # int 1 = |Omega|
    interior = ~_all_boundary(m)
    # sum_p B[p, k] = -int d_c psi_k = 0 for nodes off the boundary
    Bd = B.dense()
    colsum = Bd.sum(axis=0).reshape(-1, 3)
    node_int = np.zeros(m.nnodes, dtype=bool)
    node_int[: m.nv] = interior
    ea, eb = m.edges[:, 0], m.edges[:, 1]
    Xm = 0.5 * (m.coords[ea] + m.coords[eb])
    node_int[m.nv:] = ~np.any((np.abs(Xm) < 1e-12) | (np.abs(Xm - 1) < 1e-12), axis=1)
    assert np.abs(colsum[node_int]).max() < 1e-15
    # B applied to the linear field u = x e_x: div u = 1 -> B u = -int phi_p
    u = np.zeros((m.nnodes, 3))
    u[: m.nv, 0] = m.coords[:, 0]
    assert np.allclose(B.matvec(u)[:, 0], -C.dense().sum(axis=1), atol=1e-15)


# ---------------------------------------------------------------- patch tests
def _solve_spd(A, b):
    return np.linalg.solve(A.dense(), b.ravel()).reshape(-1, 3)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_patch_laplace_harmonic_quadratic(n):
    m = M.kuhn_mesh(n)
    u = lambda X: np.stack([X[:, 0] ** 2 - X[:, 1] ** 2, X[:, 0] * X[:, 1], X[:, 2] + 0.3 * X[:, 0]], 1)
    s = fem.vector_laplacian(n, u, _all_boundary)
    x = _solve_spd(s.A, s.b)
    assert np.abs(fem.full_solution(s, x) - fem.lagrange_exact(m, u)).max() < 1e-13


@pytest.mark.parametrize("n", [1, 2])
def test_patch_elasticity_quadratic(n):
    m = M.kuhn_mesh(n)
    lam, mu = fem.lame_from(1.0, 0.3)
    u = lambda X: np.stack([X[:, 0] ** 2 - X[:, 1] ** 2, -2 * X[:, 0] * X[:, 1], 0 * X[:, 2]], 1)
    A = fem.assemble_velocity_block(m, "elastic", lam, mu)
    lift, dm = fem.interpolate_dirichlet(m, _all_boundary(m), u)
    b = fem.apply_dirichlet(A, np.zeros((m.nnodes, 3)), lift, dm)
    x = _solve_spd(A, b)
    assert np.abs(x + lift - fem.lagrange_exact(m, u)).max() < 1e-13


def test_patch_uniaxial_traction():
    """Uniaxial stress u = a (x, -nu' y, -nu' z): traction (E a, 0, 0) on x = 1,
    free lateral faces; reproduced exactly with the x = 1 traction load."""
    n = 2
    m = M.kuhn_mesh(n)
    lam, mu = fem.lame_from(1.0, 0.3)
    a = 0.01
    nup = lam / (2 * (lam + mu))
    E = mu * (3 * lam + 2 * mu) / (lam + mu)
    u = lambda X: np.stack([a * X[:, 0], -nup * a * X[:, 1], -nup * a * X[:, 2]], 1)
    A = fem.assemble_velocity_block(m, "elastic", lam, mu)
    lift, dm = fem.interpolate_dirichlet(m, np.abs(m.coords[:, 0]) < 1e-12, u)
    tr = np.zeros((n, n, 2, 3))
    tr[..., 0] = E * a
    b = fem.apply_dirichlet(A, fem.traction_load_x1(m, tr), lift, dm)
    x = _solve_spd(A, b)
    assert np.abs(x + lift - fem.lagrange_exact(m, u)).max() < 1e-15


def test_paper_bc_laplace_is_linear():
    """Section 4.1 data (u = 0 on z = 0, (0,0,1) on z = 1, Neumann 0 elsewhere):
    the vector Laplacian's solution is u = (0, 0, z), which P2 reproduces."""
    s = fem.paper_spd(3, "laplace")
    x = _solve_spd(s.A, s.b)
    ex = fem.lagrange_exact(s.mesh, lambda X: np.stack([0 * X[:, 0], 0 * X[:, 0], X[:, 2]], 1))
    assert np.abs(fem.full_solution(s, x) - ex).max() < 1e-13


def _saddle_dense(s):
    A, B = s.A.dense(), s.B.dense()
    C = s.C.dense() if s.C is not None else np.zeros((B.shape[0], B.shape[0]))
    return np.block([[A, B.T], [B, -C]]), np.concatenate([s.f.ravel(), s.g])


@pytest.mark.parametrize("n", [1, 2])
def test_patch_mixed_elasticity(n):
    """u = (x, 0, 0), div u = 1, p = -lambda div u = -lambda (Section 2.1)."""
    m = M.kuhn_mesh(n)
    lam, mu = 3.0, 0.7
    u = lambda X: np.stack([X[:, 0], 0 * X[:, 1], 0 * X[:, 2]], 1)
    s = fem.saddle_system(m, mu, 1 / lam, _all_boundary(m), u)
    K, rhs = _saddle_dense(s)
    sol = np.linalg.solve(K, rhs)
    N = 3 * m.nnodes
    assert np.abs(sol[:N].reshape(-1, 3) + s.lift - fem.lagrange_exact(m, u)).max() < 1e-13
    assert np.abs(sol[N:] + lam).max() < 1e-12


@pytest.mark.parametrize("n", [2, 4])
def test_stokes_consistency(n):
    """u = (y^2, 0, 0), p = 2 mu x solves Stokes with zero body force; the
    interpolant satisfies the discrete equations exactly."""
    m = M.kuhn_mesh(n)
    mu = 0.5
    u = lambda X: np.stack([X[:, 1] ** 2, 0 * X[:, 1], 0 * X[:, 2]], 1)
    s = fem.saddle_system(m, mu, 0.0, _all_boundary(m), u)
    xe = fem.lagrange_exact(m, u) - s.lift
    pe = 2 * mu * m.coords[:, 0]
    r1 = s.A.matvec(xe) + s.B.transpose().matvec(pe.reshape(-1, 1)) - s.f
    r2 = s.B.matvec(xe)[:, 0] - s.g
    assert np.abs(r1).max() < 1e-14 and np.abs(r2).max() < 1e-15


@pytest.mark.parametrize("n", [2, 3])
def test_stokes_cavity_kernel_is_constants(n):
    """Lid-driven cavity on the mirrored split: the saddle matrix has exactly
    one null vector (constant pressure) and the right-hand side is consistent."""
    s = fem.stokes_lid(n, 1.3)
    K, rhs = _saddle_dense(s)
    ns = sla.null_space(K)
    assert ns.shape[1] == 1
    N = 3 * s.mesh.nnodes
    assert np.abs(ns[:N]).max() < 1e-10
    assert np.abs(ns[N:] - ns[N:].mean()).max() < 1e-10
    assert abs(ns[:, 0] @ rhs) < 1e-13
    assert s.singular


def test_plain_kuhn_cavity_has_spurious_pressure_modes():
    """Why the cavity uses the mirrored split: on the plain split the
    all-Dirichlet Taylor-Hood system has more than the constant in its kernel."""
    m = M.kuhn_mesh(2)
    s = fem.saddle_system(m, 0.5, 0.0, _all_boundary(m), lambda X: np.zeros((X.shape[0], 3)))
    K, _ = _saddle_dense(s)
    assert sla.null_space(K).shape[1] > 1


def test_dirichlet_elimination_symmetric():
    s = fem.laplace_trig(3, __import__("synth").trig_dirichlet(0, 1))
    Ad = s.A.dense()
    assert np.abs(Ad - Ad.T).max() < 1e-15
    assert np.all(s.b[s.dirichlet] == 0)
    # explicit zeros stay in the pattern
    assert s.A.nnz == fem.structural_pattern(s.mesh).nnz
