"""Reduced-precision saddle cycle (FP32, and FP32 + BF16 coarse velocity
blocks) inside FP64 flexible GMRES: one cycle against the oracle's FP64
cycle within the bound of its arithmetic, solves against the FP64 solve."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1503_01287_amd as amg  # noqa: E402
from oracle import amg as oamg, workloads  # noqa: E402

DEV = torch.device("cuda:0")

CASES = {
    "mixed3-nu0.3-sGS": (lambda: amg.problems.mixed_elasticity(3, nu=0.3),
                         lambda: workloads.mixed_elasticity(3, nu=0.3), "sGS-1-1"),
    "mixed5-nu0.49999-BS": (lambda: amg.problems.mixed_elasticity(5), lambda: workloads.mixed_elasticity(5),
                            "BS-1-1"),
    "cavity6-BS": (lambda: amg.problems.stokes_cavity(6, 0.8), lambda: workloads.stokes(6, 0.8), "BS-1-1"),
    "cavity4-sGS": (lambda: amg.problems.stokes_cavity(4, 1.3), lambda: workloads.stokes(4, 1.3), "sGS-1-1"),
}
# bound per cycle: FP32 arithmetic (unit roundoff 6e-8) through a few levels
# of smoothing and transfers, BF16 (unit roundoff 4e-3) on the coarse velocity blocks
TOL = {"FP32": 2e-4, "MIXED": 5e-2}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def centre(v, s):
    v = v.copy()
    if s.pressure_kernel:
        nu = 3 * s.nodes
        v[nu:] -= v[nu:].mean()
    return v


@pytest.mark.parametrize("precision", ["FP32", "MIXED"])
@pytest.mark.parametrize("name", list(CASES))
def test_reduced_cycle_vs_oracle(name, precision):
    hs_, os_, sm = CASES[name]
    hs, o = hs_(), os_()
    s = amg.AMGSolver(hs, smoother=sm, krylov="FGMRES", precision=precision)
    h = oamg.setup(o.A, o.nlin, o.nquad, B=o.B, C=o.C, singular=o.singular)
    if sm.startswith("BS"):
        oamg.prepare_bs(h)
    prec = oamg.preconditioner(h, oamg.Smoother.parse(sm))
    r = np.random.default_rng(41).standard_normal(hs.dofs)
    z = torch.zeros(hs.dofs, dtype=torch.float64, device=DEV)
    s.precondition(dev(r), z)
    e = rel(centre(host(z), hs), centre(prec(r), hs))
    assert e < TOL[precision], (name, precision, e)
    s.close()


@pytest.mark.parametrize("precision", ["FP32", "MIXED"])
@pytest.mark.parametrize("name", list(CASES))
def test_reduced_cycle_fgmres_reaches_fp64_solution(name, precision):
    hs = CASES[name][0]()
    sm = CASES[name][2]
    b = dev(hs.rhs)
    ref = amg.AMGSolver(hs, smoother=sm, krylov="FGMRES")
    xr = torch.zeros_like(b)
    rr = ref.solve(b, xr, tol=1e-11, maxit=500)
    s = amg.AMGSolver(hs, smoother=sm, krylov="FGMRES", precision=precision)
    x = torch.zeros_like(b)
    res = s.solve(b, x, tol=1e-9, maxit=500)
    assert res.converged and res.relres <= 1e-9 * 1.01, (name, res)
    x64 = torch.zeros_like(b)
    r64 = ref.solve(b, x64, tol=1e-9, maxit=500)
    assert res.iters <= r64.iters + 3, (name, precision, res.iters, r64.iters)
    assert rel(centre(host(x), hs), centre(host(xr), hs)) < 1e-7
    s.close()
    ref.close()
    del rr


@pytest.mark.parametrize("precision", ["FP32", "MIXED"])
def test_reduced_batch(precision):
    systems = [amg.problems.stokes_cavity(5, 0.7), amg.problems.mixed_elasticity(3, nu=0.3),
               amg.problems.stokes_cavity(3, 1.2), amg.problems.stokes_cavity(7, 1.6)]
    bsol = amg.BatchedSolver(systems, smoother="BS-1-1", precision=precision)
    b = dev(np.concatenate([s.rhs for s in systems]))
    x = torch.zeros_like(b)
    res = bsol.solve(b, x, tol=1e-9)
    xs = host(x)
    o = 0
    for s, r in zip(systems, res):
        assert r.converged and r.relres <= 1e-9 * 1.01, (s.name, r)
        single = amg.AMGSolver(s, smoother="BS-1-1", krylov="FGMRES")
        xd = torch.zeros(s.dofs, dtype=torch.float64, device=DEV)
        rr = single.solve(dev(s.rhs), xd, tol=1e-11)
        assert rr.converged
        assert rel(centre(xs[o:o + s.dofs], s), centre(host(xd), s)) < 1e-7, s.name
        o += s.dofs
        single.close()
    bsol.close()
