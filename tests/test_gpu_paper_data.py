"""GPU parity with the oracle on the paper's own data (Section 4.1's cube
with u = 0 on z = 0 and u = (0, 0, 1) on z = 1): the stand-alone solver with
forward sweeps on both sides of the coarse correction, non-separating
coarsening under PCG with two W-cycles per iteration (the black-box
comparison), and flexible GMRES on the mixed form of Section 4.4."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1503_01287_amd as amg  # noqa: E402
from oracle import amg as oamg, fem, krylov  # noqa: E402

DEV = torch.device("cuda:0")


def _solve(sysm, tol, **kw):
    s = amg.AMGSolver(sysm, **kw)
    b = torch.from_numpy(sysm.rhs).to(DEV)
    x = torch.zeros_like(b)
    r = s.solve(b, x, tol=tol, maxit=400)
    torch.cuda.synchronize()
    s.close()
    return r, x.cpu().numpy()


def _spd_mv(o):
    return lambda v: o.A.matvec(np.asarray(v).reshape(-1, 3)).ravel()


@pytest.mark.parametrize("n", [4, 6])
def test_standalone_forward_sweeps(n):
    sysm, o = amg.problems.paper_cube(n, "laplace"), fem.paper_spd(n, "laplace")
    r, x = _solve(sysm, 1e-11, smoother="GS-1-1", krylov="NONE")
    h = oamg.setup(o.A, o.nlin, o.nquad)
    sm = oamg.Smoother.parse("GS-1-1")
    sm.post_forward = True
    b = o.b
    xo = np.zeros_like(b)
    r0 = np.linalg.norm(b)
    for it in range(1, 401):
        xo = oamg.cycle(h, 0, sm, b, xo)
        if np.linalg.norm(b - o.A.matvec(xo)) / r0 <= 1e-11:
            break
    assert r.converged and abs(r.iters - it) <= 1, (r.iters, it)
    assert np.linalg.norm(x - xo.ravel()) / np.linalg.norm(xo) < 1e-9


@pytest.mark.parametrize("n", [4, 6])
def test_nonseparating_pcg_two_w_cycles(n):
    sysm, o = amg.problems.paper_cube(n, "laplace"), fem.paper_spd(n, "laplace")
    r, x = _solve(sysm, 1e-11, smoother="GS-1-1", krylov="PCG", nu=2, cycles=2, separate=False)
    h = oamg.setup(o.A, o.nlin, o.nquad, separate=False)
    prec = oamg.preconditioner(h, oamg.Smoother.parse("GS-1-1"), cycles=2, nu=2)
    ref = krylov.pcg(_spd_mv(o), lambda v: prec(v).ravel(), o.b.ravel(), tol=1e-11)
    assert r.converged and abs(r.iters - ref.iters) <= 1, (r.iters, ref.iters)
    assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) < 1e-9


@pytest.mark.parametrize("smoother,cycles", [("BS-1-1", 1), ("BS-1-1", 2), ("sGS-1-1", 1)])
def test_mixed_fgmres(smoother, cycles):
    sysm, o = amg.problems.paper_cube(4, "mixed"), fem.paper_mixed(4)
    r, x = _solve(sysm, 1e-9, smoother=smoother, krylov="FGMRES", cycles=cycles)
    h = oamg.setup(o.A, o.nlin, o.nquad, B=o.B, C=o.C, singular=o.singular)
    if smoother.startswith("BS"):
        oamg.prepare_bs(h)
    Bt = o.B.transpose()
    nv = 3 * o.A.nrows

    def mv(z):
        u, p = z[:nv].reshape(-1, 3), z[nv:]
        return np.concatenate([o.A.matvec(u).ravel() + Bt.matvec(p.reshape(-1, 1)).ravel(),
                               o.B.matvec(u)[:, 0] - o.C.matvec(p.reshape(-1, 1))[:, 0]])
    ref = krylov.fgmres(mv, oamg.preconditioner(h, oamg.Smoother.parse(smoother), cycles=cycles),
                        np.concatenate([o.f.ravel(), o.g]), tol=1e-9)
    assert r.converged and abs(r.iters - ref.iters) <= 1, (r.iters, ref.iters)
    assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) < 1e-7
