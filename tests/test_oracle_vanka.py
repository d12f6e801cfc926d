"""Pins of the oracle's multiplicative Vanka smoother (Section 3.3): the patch
of an interior vertex, the multiplicative Schwarz error operator, colour
independence and the fixed point."""
import numpy as np

from oracle import amg, mesh as M, workloads


def _level(n, nu=0.3):
    o = workloads.mixed_elasticity(n, nu=nu)
    return o, amg.Level(o.A, o.nlin, o.nquad, B=o.B, C=o.C)


def test_interior_patch_is_the_vertex_star():
    """An interior vertex of the Kuhn mesh has 14 neighbours and a link with
    24 triangles, hence 14 + 24 - 2 = 36 rim edges (Euler) and 14 spokes:
    15 vertices + 50 edges = 65 P2 nodes, 3 * 65 + 1 = 196 unknowns."""
    o, lev = _level(4)
    V = amg.vanka_patches(lev)
    v = M.vid(4, 2, 2, 2)
    assert len(V.nodes[v]) == 65
    assert len(V.dofs[v]) == 196
    # the vertices of the patch are the vertex and its 14 neighbours
    assert (V.nodes[v] < o.nlin).sum() == 15


def test_sweep_is_the_product_of_local_projections():
    """x_new = x* - E (x* - x), E = prod_i (I - omega R_i^T K_i^{-1} R_i K)
    over the patches in processing order (dense, tiny mesh)."""
    o, lev = _level(2)
    sm = amg.Smoother.parse("Vanka-1-1-0.7")
    V = amg.vanka_patches(lev)
    K = V.K.toarray()
    nd = K.shape[0]
    rng = np.random.default_rng(3)
    b, x = rng.standard_normal(nd), rng.standard_normal(nd)
    xs = np.linalg.solve(K, b)
    E = np.eye(nd)
    for i in V.order:
        idx = V.dofs[i]
        R = np.zeros((idx.size, nd))
        R[np.arange(idx.size), idx] = 1.0
        T = np.eye(nd) - 0.7 * R.T @ np.linalg.solve(K[np.ix_(idx, idx)], R @ K)
        E = T @ E
    nv = 3 * o.A.nrows
    u, p = amg.vanka_step(lev, sm, b[:nv].reshape(-1, 3), b[nv:], x[:nv].reshape(-1, 3), x[nv:])
    got = np.concatenate([u.ravel(), p])
    assert np.abs(got - (xs - E @ (xs - x))).max() < 1e-10 * np.abs(xs).max()


def test_same_colour_patches_are_independent():
    o, lev = _level(3)
    V = amg.vanka_patches(lev)
    K = V.K.tocsr()
    for c in np.unique(V.colors):
        members = np.where(V.colors == c)[0]
        seen = np.zeros(K.shape[0], dtype=bool)
        for i in members:
            assert not seen[V.dofs[i]].any()          # disjoint
            seen[V.dofs[i]] = True
        for i in members:
            touched = np.unique(K[V.dofs[i]].indices)  # DOFs whose value enters patch i's residual
            others = np.concatenate([V.dofs[j] for j in members if j != i]) if members.size > 1 else []
            assert not np.isin(others, touched).any()


def test_exact_solution_is_a_fixed_point():
    o, lev = _level(2)
    V = amg.vanka_patches(lev)
    K = V.K.toarray()
    b = np.random.default_rng(4).standard_normal(K.shape[0])
    xs = np.linalg.solve(K, b)
    nv = 3 * o.A.nrows
    u, p = amg.vanka_step(lev, amg.Smoother.parse("Vanka-1-1"), b[:nv].reshape(-1, 3), b[nv:],
                          xs[:nv].reshape(-1, 3), xs[nv:])
    assert np.abs(np.concatenate([u.ravel(), p]) - xs).max() < 1e-12 * np.abs(xs).max()
