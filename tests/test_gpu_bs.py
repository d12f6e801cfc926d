"""Parity of the Braess-Sarazin smoother (Section 3.3) with the FP64 oracle:
Schur complements S_l = C + B (2D)^{-1} B^T, one smoothing step (scalar
V-cycle inside), the saddle V-cycle and FGMRES with it."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1503_01287_amd as amg  # noqa: E402
from oracle import amg as oamg, krylov, workloads  # noqa: E402

DEV = torch.device("cuda:0")

CASES = {
    "mixed3-nu0.3": (lambda: amg.problems.mixed_elasticity(3, nu=0.3),
                     lambda: workloads.mixed_elasticity(3, nu=0.3)),
    "mixed5-nu0.49999": (lambda: amg.problems.mixed_elasticity(5), lambda: workloads.mixed_elasticity(5)),
    "cavity4": (lambda: amg.problems.stokes_cavity(4, 1.3), lambda: workloads.stokes(4, 1.3)),
    "cavity6": (lambda: amg.problems.stokes_cavity(6, 0.7), lambda: workloads.stokes(6, 0.7)),
}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    hs, os_ = CASES[request.param]
    o = os_()
    h = oamg.setup(o.A, o.nlin, o.nquad, B=o.B, C=o.C, singular=o.singular)
    oamg.prepare_bs(h)
    s = amg.AMGSolver(hs(), smoother="BS-1-1", krylov="FGMRES")
    yield request.param, s, o, h
    s.close()


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


def test_schur_complements(case):
    name, s, o, h = case
    assert s.num_levels == len(h.levels)
    for l in range(h.L):
        info = s.level_info(l)
        levels = h.levels[l].schur[0]
        assert info.schur_levels == len(levels), (name, l)
        S = levels[0].S
        rp, col, val = s.level_matrix(l, "S")
        assert np.array_equal(rp, S.indptr) and np.array_equal(col, S.indices), (name, l)
        assert rel(val.ravel(), S.vals.ravel()) < 1e-13, (name, l)
    assert s.level_info(h.L).schur_levels == 0


def test_bs_step(case):
    name, s, o, h = case
    lev = h.levels[0]
    nv = 3 * lev.n
    n = nv + lev.npres
    rng = np.random.default_rng(31)
    z, b = rng.standard_normal(n), rng.standard_normal(n)
    xd = dev(z)
    s.smooth(0, dev(b), xd)
    sm = oamg.Smoother.parse("BS-1-1")
    u, p = oamg.bs_step(lev, sm, b[:nv].reshape(-1, 3), b[nv:], z[:nv].reshape(-1, 3), z[nv:])
    assert rel(host(xd), np.concatenate([u.ravel(), p])) < 1e-11, name


@pytest.mark.parametrize("cycles", [1, 2])
def test_bs_vcycle(case, cycles):
    name, _, o, h = case
    hs = CASES[name][0]()
    s2 = amg.AMGSolver(hs, smoother="BS-1-1", krylov="FGMRES", cycles=cycles)
    prec = oamg.preconditioner(h, oamg.Smoother.parse("BS-1-1"), cycles=cycles)
    r = np.random.default_rng(32).standard_normal(hs.dofs)
    z = torch.zeros(hs.dofs, dtype=torch.float64, device=DEV)
    s2.precondition(dev(r), z)
    assert rel(host(z), prec(r)) < 1e-10, name
    s2.close()


def test_bs_fgmres_solve(case):
    name, _, o, h = case
    hs = CASES[name][0]()
    tol = 1e-9
    s = amg.AMGSolver(hs, smoother="BS-1-1", krylov="FGMRES")
    b = dev(hs.rhs)
    x = torch.zeros_like(b)
    res = s.solve(b, x, tol=tol, maxit=400)
    assert res.converged and res.relres <= tol * 1.01, (name, res)
    prec = oamg.preconditioner(h, oamg.Smoother.parse("BS-1-1"))
    rhs = np.concatenate([o.f.ravel(), o.g])
    ref = krylov.fgmres(_mv(o), prec, rhs, tol=tol, maxit=400)
    assert abs(res.iters - ref.iters) <= 1, (name, res.iters, ref.iters)
    xs = host(x)
    nv = 3 * o.A.nrows
    refx = ref.x.copy()
    if o.singular:
        xs[nv:] -= xs[nv:].mean()
        refx[nv:] -= refx[nv:].mean()
    assert np.linalg.norm(xs - refx) / np.linalg.norm(refx) < 1e-7
    s.close()


def test_bs_two_steps_on_level1():
    """Pre- and post-smoothing on a coarse level (Schur hierarchy one level
    shorter) against the oracle's step, twice in a row."""
    hs, o = amg.problems.mixed_elasticity(5), workloads.mixed_elasticity(5)
    h = oamg.setup(o.A, o.nlin, o.nquad, B=o.B, C=o.C, singular=o.singular)
    oamg.prepare_bs(h)
    s = amg.AMGSolver(hs, smoother="BS-1-1", krylov="FGMRES")
    assert h.L >= 2
    lev = h.levels[1]
    nv = 3 * lev.n
    n = nv + lev.npres
    rng = np.random.default_rng(33)
    z, b = rng.standard_normal(n), rng.standard_normal(n)
    xd = dev(z)
    s.smooth(1, dev(b), xd)
    s.smooth(1, dev(b), xd)
    sm = oamg.Smoother.parse("BS-1-1")
    u, p = z[:nv].reshape(-1, 3), z[nv:]
    for _ in range(2):
        u, p = oamg.bs_step(lev, sm, b[:nv].reshape(-1, 3), b[nv:], u, p)
    assert rel(host(xd), np.concatenate([u.ravel(), p])) < 1e-11
    s.close()
