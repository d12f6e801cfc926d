"""Parity of the saddle point path (mixed elasticity, Stokes cavity) with the
FP64 oracle: saddle Galerkin hierarchy, K apply, sGS step, V-cycle, FGMRES."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1503_01287_amd as amg  # noqa: E402
from oracle import amg as oamg, krylov, workloads  # noqa: E402

DEV = torch.device("cuda:0")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


CASES = {
    "mixed3-nu0.3": (lambda: amg.problems.mixed_elasticity(3, nu=0.3),
                     lambda: workloads.mixed_elasticity(3, nu=0.3)),
    "mixed5-nu0.49999": (lambda: amg.problems.mixed_elasticity(5), lambda: workloads.mixed_elasticity(5)),
    "cavity4": (lambda: amg.problems.stokes_cavity(4, 1.3), lambda: workloads.stokes(4, 1.3)),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    hs, os_ = CASES[request.param]
    return request.param, hs(), os_()


def _oh(o):
    return oamg.setup(o.A, o.nlin, o.nquad, B=o.B, C=o.C, singular=o.singular)


def _mv(o):
    A, B = o.A, o.B
    Bt = B.transpose()
    nv = 3 * A.nrows

    def mv(z):
        u, p = z[:nv].reshape(-1, 3), z[nv:]
        top = A.matvec(u).ravel() + Bt.matvec(p.reshape(-1, 1)).ravel()
        bot = B.matvec(u)[:, 0]
        if o.C is not None:
            bot = bot - o.C.matvec(p.reshape(-1, 1))[:, 0]
        return np.concatenate([top, bot])
    return mv


def test_saddle_hierarchy(case):
    name, hs, o = case
    s = amg.AMGSolver(hs, smoother="sGS-1-1", krylov="FGMRES")
    h = _oh(o)
    assert s.num_levels == len(h.levels)
    for l, lev in enumerate(h.levels):
        info = s.level_info(l)
        assert (info.n_lin, info.n_quad, info.n_pres) == (lev.nlin, lev.nquad, lev.npres), (name, l)
        rp, col, val = s.level_matrix(l, "B")
        assert np.array_equal(rp, lev.B.indptr) and np.array_equal(col, lev.B.indices)
        assert rel(val.reshape(-1, 1, 3), lev.B.vals) < 1e-13, (name, l)
        if lev.C is not None:
            rp, col, val = s.level_matrix(l, "C")
            assert np.array_equal(col, lev.C.indices)
            assert rel(val.ravel(), lev.C.vals.ravel()) < 1e-13


def test_saddle_apply_and_sgs_step(case):
    name, hs, o = case
    s = amg.AMGSolver(hs, smoother="sGS-1-1", krylov="FGMRES")
    rng = np.random.default_rng(21)
    z = rng.standard_normal(hs.dofs)
    y = torch.zeros(hs.dofs, dtype=torch.float64, device=DEV)
    s.apply(0, dev(z), y)
    assert rel(host(y), _mv(o)(z)) < 1e-13
    h = _oh(o)
    lev = h.levels[0]
    sm = oamg.Smoother.parse("sGS-1-1")
    nv = 3 * lev.n
    b = rng.standard_normal(hs.dofs)
    xd = dev(z)
    s.smooth(0, dev(b), xd)
    u, p = oamg.sgs_step(lev, sm, b[:nv].reshape(-1, 3), b[nv:], z[:nv].reshape(-1, 3), z[nv:])
    assert rel(host(xd), np.concatenate([u.ravel(), p])) < 1e-12


@pytest.mark.parametrize("cycles", [1, 2])
def test_saddle_vcycle(case, cycles):
    name, hs, o = case
    s = amg.AMGSolver(hs, smoother="sGS-1-1", krylov="FGMRES", cycles=cycles)
    h = _oh(o)
    prec = oamg.preconditioner(h, oamg.Smoother.parse("sGS-1-1"), cycles=cycles)
    r = np.random.default_rng(22).standard_normal(hs.dofs)
    z = torch.zeros(hs.dofs, dtype=torch.float64, device=DEV)
    s.precondition(dev(r), z)
    assert rel(host(z), prec(r)) < 1e-11, name


def test_saddle_fgmres_solve(case):
    name, hs, o = case
    tol = 1e-9
    s = amg.AMGSolver(hs, smoother="sGS-1-1", krylov="FGMRES")
    b = dev(hs.rhs)
    x = torch.zeros_like(b)
    res = s.solve(b, x, tol=tol, maxit=400)
    assert res.converged and res.relres <= tol * 1.01, (name, res)
    h = _oh(o)
    prec = oamg.preconditioner(h, oamg.Smoother.parse("sGS-1-1"))
    rhs = np.concatenate([o.f.ravel(), o.g])
    ref = krylov.fgmres(_mv(o), prec, rhs, tol=tol, maxit=400)
    assert abs(res.iters - ref.iters) <= 1, (name, res.iters, ref.iters)
    xs = host(x)
    nv = 3 * o.A.nrows
    if o.singular:
        xs[nv:] -= xs[nv:].mean()
        refx = ref.x.copy()
        refx[nv:] -= refx[nv:].mean()
    else:
        refx = ref.x
    assert np.linalg.norm(xs - refx) / np.linalg.norm(refx) < 1e-7


def test_fgmres_on_spd_system():
    """FGMRES with the SPD V-cycle: same iterates as the oracle's FGMRES."""
    hs, o = amg.problems.elasticity(4), workloads.elasticity(4)
    s = amg.AMGSolver(hs, smoother="GS-1-1", krylov="FGMRES")
    b = dev(hs.rhs)
    x = torch.zeros_like(b)
    res = s.solve(b, x, tol=1e-10, maxit=200)
    assert res.converged
    h = oamg.setup(o.A, o.nlin, o.nquad)
    prec = oamg.preconditioner(h, oamg.Smoother.parse("GS-1-1"))
    ref = krylov.fgmres(lambda v: o.A.matvec(v).ravel(), lambda r: prec(r).ravel(), o.b.ravel(), tol=1e-10)
    assert abs(res.iters - ref.iters) <= 1
    assert np.linalg.norm(host(x) - ref.x) / np.linalg.norm(ref.x) < 1e-8


def test_saddle_stationary_iteration():
    hs, o = amg.problems.mixed_elasticity(3, nu=0.3), workloads.mixed_elasticity(3, nu=0.3)
    s = amg.AMGSolver(hs, smoother="sGS-2-2", krylov="NONE")
    b = dev(hs.rhs)
    x = torch.zeros_like(b)
    res = s.solve(b, x, tol=1e-6, maxit=2000)
    assert res.converged, res


@pytest.mark.parametrize("smoother", ["sGS-1-1", "BS-1-1"])
def test_zero_blocks_dropped_after_setup(smoother):
    """After the pattern-based setup the solve kernels stream A and B without
    their numerically zero blocks (here the cavity's Dirichlet couplings): on
    every level the kept counts equal the nonzero blocks (plus A's diagonal)
    of the exported structural operators, those still equal the oracle's,
    and the operator and one cycle still equal the oracle's."""
    hs, o = amg.problems.stokes_cavity(5, 1.1), workloads.stokes(5, 1.1)
    s = amg.AMGSolver(hs, smoother=smoother, krylov="FGMRES")
    h = _oh(o)
    dropped = 0
    for l, lev in enumerate(h.levels):
        info = s.level_info(l)
        rp, col, val = s.level_matrix(l, "A")
        assert np.array_equal(rp, lev.A.indptr) and np.array_equal(col, lev.A.indices)
        rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
        keep = (np.abs(val).max(axis=1) > 0) | (col == rows)
        assert info.kept_A == keep.sum() and info.nnz_A == len(col), l
        _, _, bval = s.level_matrix(l, "B")
        assert info.kept_B == (np.abs(bval).max(axis=1) > 0).sum() and info.nnz_B == len(bval), l
        dropped += info.nnz_A - info.kept_A
    assert dropped > 0
    rng = np.random.default_rng(22)
    z = rng.standard_normal(hs.dofs)
    y = torch.zeros(hs.dofs, dtype=torch.float64, device=DEV)
    s.apply(0, dev(z), y)
    assert rel(host(y), _mv(o)(z)) < 1e-13
    if smoother.startswith("BS"):
        oamg.prepare_bs(h)
    prec = oamg.preconditioner(h, oamg.Smoother.parse(smoother))
    zc = torch.zeros(hs.dofs, dtype=torch.float64, device=DEV)
    s.precondition(dev(z), zc)
    assert rel(host(zc), prec(z)) < 1e-10
    s.close()
