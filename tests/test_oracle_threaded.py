"""The oracle's all-core loops (used only to time the oracle on every host
core) against the oracle's own functions: the block and scalar products, the
Gauss-Seidel sweep by colours (the same result bit for bit, since no two nodes
of a colour are coupled), block Jacobi, and whole preconditioned solves that
follow the single-thread ones iterate by iterate."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import amg, krylov, sparse, threaded, workloads


@pytest.fixture(scope="module")
def elast():
    o = workloads.elasticity(4)
    return o, amg.setup(o.A, o.nlin, o.nquad)


@pytest.mark.parametrize("shape", [(3, 3), (1, 3), (3, 1), (1, 1)])
def test_block_product(shape):
    rng = np.random.default_rng(1)
    br, bc = shape
    n, m = 57, 41
    pat = sp.random(n, m, density=0.15, random_state=2, format="csr")
    pat.sort_indices()
    M = sparse.BlockCSR(pat.indptr.astype(np.int64), pat.indices.astype(np.int64),
                        rng.standard_normal((pat.nnz, br, bc)), m)
    x = rng.standard_normal((m, bc))
    ref = M.matvec(x)
    got = threaded.bsr_matvec(M, x)
    assert got.shape == ref.shape
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)
    # the dense product decides, independent of either loop
    np.testing.assert_allclose(got.ravel(), M.dense() @ x.ravel(), rtol=1e-12, atol=1e-12)


def test_scalar_transfer_products(elast):
    o, h = elast
    P = h.levels[0].P
    W = threaded._CSR(P)
    rng = np.random.default_rng(3)
    r = rng.standard_normal((P.shape[0], 3))
    e = rng.standard_normal((P.shape[1], 3))
    np.testing.assert_allclose(W.T @ r, P.T @ r, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(W @ e, P @ e, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(W @ e[:, 0], P @ e[:, 0], rtol=1e-13, atol=1e-13)
    assert W.T.T is W


@pytest.mark.parametrize("forward", [True, False])
def test_gs_by_colours_is_the_sequential_sweep(elast, forward):
    o, h = elast
    rng = np.random.default_rng(4)
    threaded.lib().omp_set_threads(4)
    for lev in h.levels[:-1]:
        starts = threaded._colour_starts(lev)
        assert starts is not None
        b = rng.standard_normal((lev.n, 3))
        x = rng.standard_normal((lev.n, 3))
        ref = amg.gauss_seidel(lev, b, x, forward)
        got = threaded.gauss_seidel_colours(lev, b, x, forward, starts)
        assert np.array_equal(got, ref)


def test_jacobi(elast):
    o, h = elast
    lev = h.levels[1]
    rng = np.random.default_rng(5)
    b = rng.standard_normal((lev.n, 3))
    x = rng.standard_normal((lev.n, 3))
    np.testing.assert_allclose(threaded.jacobi(lev, b, x, 0.5), amg.jacobi(lev, b, x, 0.5), rtol=1e-13, atol=1e-13)


def test_index_order_keeps_the_sequential_sweep():
    o = workloads.elasticity(3)
    h = amg.setup(o.A, o.nlin, o.nquad, coloured=False)
    assert all(threaded._colour_starts(lev) is None for lev in h.levels)


@pytest.mark.parametrize("sm", ["GS-1-1", "JA-1-1-0.5"])
def test_threaded_solve_follows_the_oracle(elast, sm):
    o, h = elast
    prec = amg.preconditioner(h, amg.Smoother.parse(sm))
    mv = lambda v: o.A.matvec(v).ravel()
    pc = lambda r: prec(r).ravel()
    b = o.b.ravel()
    ref = krylov.pcg(mv, pc, b, tol=1e-10, maxit=100)
    seq = (amg.gauss_seidel, amg.jacobi, sparse.BlockCSR.matvec, [lev.P for lev in h.levels])
    with threaded.on_threads(h, 4):
        assert threaded.threads() == 4
        got = krylov.pcg(mv, pc, b, tol=1e-10, maxit=100)
    assert (amg.gauss_seidel, amg.jacobi, sparse.BlockCSR.matvec) == seq[:3]
    assert all(a is b_ for a, b_ in zip([lev.P for lev in h.levels], seq[3]))
    assert ref.iters == got.iters
    np.testing.assert_allclose(got.history, ref.history, rtol=1e-8, atol=1e-14)
    np.testing.assert_allclose(got.x, ref.x, rtol=1e-10, atol=1e-12)
