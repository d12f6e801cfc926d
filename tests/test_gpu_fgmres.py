"""Flexible GMRES through the C ABI beyond one unrestarted cycle: restarted
FGMRES(m) against the oracle's FGMRES(m) (which orthogonalises by modified
Gram-Schmidt: the same iterates in exact arithmetic), the maxit cut-off
inside and across restart cycles, and a batch of restarted solves against
the systems' single solves."""
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
    "cavity4": (lambda: amg.problems.stokes_cavity(4, 1.3), lambda: workloads.stokes(4, 1.3)),
}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def centred(v, nv, singular):
    v = v.copy()
    if singular:
        v[nv:] -= v[nv:].mean()
    return v


def oracle_mv(o):
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


@pytest.mark.parametrize("m", [3, 7])
@pytest.mark.parametrize("name", list(CASES))
def test_restarted_fgmres_matches_oracle(name, m):
    hs, o = CASES[name][0](), CASES[name][1]()
    tol = 1e-9
    s = amg.AMGSolver(hs, smoother="sGS-1-1", krylov="FGMRES", restart=m)
    b = dev(hs.rhs)
    x = torch.zeros_like(b)
    res = s.solve(b, x, tol=tol, maxit=800)
    s.close()
    assert res.converged and res.relres <= tol * 1.01, (name, m, res)
    h = oamg.setup(o.A, o.nlin, o.nquad, B=o.B, C=o.C, singular=o.singular)
    prec = oamg.preconditioner(h, oamg.Smoother.parse("sGS-1-1"))
    rhs = np.concatenate([o.f.ravel(), o.g])
    ref = krylov.fgmres(oracle_mv(o), prec, rhs, tol=tol, maxit=800, restart=m)
    assert ref.converged
    # a restart shifts where rounding enters; allow one iteration per cycle boundary reached
    assert abs(res.iters - ref.iters) <= 1 + ref.iters // (4 * m), (name, m, res.iters, ref.iters)
    nv = 3 * o.A.nrows
    xs, rx = centred(host(x), nv, o.singular), centred(ref.x, nv, o.singular)
    assert np.linalg.norm(xs - rx) / np.linalg.norm(rx) < 1e-7


@pytest.mark.parametrize("m", [100, 3])
def test_fgmres_maxit_cutoff(m):
    """Stopping at maxit (inside the first cycle, or across restarts): the
    status says so, the iteration count is maxit, and the reported residual
    is the true one of the returned iterate."""
    hs, o = CASES["mixed3-nu0.3"][0](), CASES["mixed3-nu0.3"][1]()
    s = amg.AMGSolver(hs, smoother="sGS-1-1", krylov="FGMRES", restart=m)
    b = dev(hs.rhs)
    x = torch.zeros_like(b)
    res = s.solve(b, x, tol=1e-14, maxit=5)
    s.close()
    assert res.status == 1 and res.iters == 5, res
    rhs = np.concatenate([o.f.ravel(), o.g])
    true = np.linalg.norm(rhs - oracle_mv(o)(host(x))) / np.linalg.norm(rhs)
    assert abs(true - res.relres) <= 1e-10 * max(1.0, true)
    assert true < 1.0


def test_batched_restarted_matches_single_solves():
    """Restarted cycles in lockstep: each system's iterations and solution as
    in its own restarted solve."""
    systems = [amg.problems.stokes_cavity(5, 0.7), amg.problems.mixed_elasticity(3, nu=0.3),
               amg.problems.stokes_cavity(3, 1.2), amg.problems.stokes_cavity(6, 1.6)]
    m, tol = 6, 1e-9
    bsol = amg.BatchedSolver(systems, smoother="BS-1-1", restart=m)
    b = dev(np.concatenate([s.rhs for s in systems]))
    x = torch.zeros_like(b)
    res = bsol.solve(b, x, tol=tol, maxit=600)
    bsol.close()
    xs = host(x)
    off = np.cumsum([0] + [s.dofs for s in systems])
    for i, s in enumerate(systems):
        assert res[i].converged and res[i].relres <= tol * 1.01, (i, res[i])
        single = amg.AMGSolver(s, smoother="BS-1-1", krylov="FGMRES", restart=m)
        xd = torch.zeros(s.dofs, dtype=torch.float64, device=DEV)
        r1 = single.solve(dev(s.rhs), xd, tol=tol, maxit=600)
        single.close()
        assert abs(res[i].iters - r1.iters) <= 1, (i, res[i].iters, r1.iters)
        nv = 3 * s.nodes
        a, c = centred(xs[off[i]:off[i + 1]], nv, s.pressure_kernel), centred(host(xd), nv, s.pressure_kernel)
        assert np.linalg.norm(a - c) / np.linalg.norm(c) < 1e-7, i
