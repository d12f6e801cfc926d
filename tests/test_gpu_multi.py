"""amg_solve_multi (blocks of right-hand sides on one SPD hierarchy) through
the C ABI: every right-hand side reaches the tolerance in its true FP64
residual, in the iterations amg_solve takes for it alone (within one), at
the oracle's solution; zero right-hand sides, initial guesses, the FP64 and
the FP32/BF16 cycle, Jacobi and Gauss-Seidel, V- and W-cycles, the padding of
a block beyond the number of right-hand sides, and the rejected cases."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import scipy.sparse.linalg as spla  # noqa: E402

import paper_1503_01287_amd as amg  # noqa: E402
from oracle import workloads  # noqa: E402

DEV = torch.device("cuda:0")
TOL = 1e-10

CASES = {
    "laplace6": (lambda: amg.problems.laplace(6), lambda: workloads.laplace(6)),
    "elast5": (lambda: amg.problems.elasticity(5), lambda: workloads.elasticity(5)),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    hs, os_ = CASES[request.param]
    o = os_()
    return request.param, hs(), o, o.A.scipy().tocsc()


def _rhs(hsys, k, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((k, hsys.dofs))
    B[0] = hsys.rhs
    return B


@pytest.mark.parametrize("precision,krylov", [("FP64", "PCG"), ("MIXED", "FCG"), ("FP32", "FCG")])
@pytest.mark.parametrize("smoother", ["GS-1-1", "JA-1-1-0.5"])
@pytest.mark.parametrize("k", [1, 3, 8])
def test_block_matches_single_solves_and_oracle(case, precision, krylov, smoother, k):
    name, hsys, o, Asp = case
    s = amg.AMGSolver(hsys, smoother=smoother, krylov=krylov, precision=precision)
    B = _rhs(hsys, k, 40 + k)
    Bd = torch.from_numpy(B).to(DEV)
    Xd = torch.zeros_like(Bd)
    res = s.solve_multi(Bd, Xd, tol=TOL, maxit=300)
    torch.cuda.synchronize()
    X = Xd.cpu().numpy()
    for r in range(k):
        assert res[r].converged and res[r].relres <= TOL * 1.01, (name, r, res[r])
        x1 = torch.zeros(hsys.dofs, dtype=torch.float64, device=DEV)
        single = s.solve(Bd[r].contiguous(), x1, tol=TOL, maxit=300)
        assert abs(single.iters - res[r].iters) <= 1, (name, r, single.iters, res[r].iters)
        ref = spla.spsolve(Asp, B[r])
        assert np.linalg.norm(X[r] - ref) / np.linalg.norm(ref) < 1e-7, (name, r)
        true = np.linalg.norm(B[r] - Asp @ X[r]) / np.linalg.norm(B[r])
        assert true <= TOL * 1.01, (name, r, true)
    s.close()


def test_zero_rhs_initial_guess_and_w_cycle(case):
    name, hsys, o, Asp = case
    s = amg.AMGSolver(hsys, smoother="GS-1-1", krylov="PCG", nu=2)
    B = _rhs(hsys, 5, 7)
    B[2] = 0.0
    X0 = np.random.default_rng(8).standard_normal((5, hsys.dofs))
    X0[2] = 0.0
    Bd, Xd = torch.from_numpy(B).to(DEV), torch.from_numpy(X0).to(DEV)
    res = s.solve_multi(Bd, Xd, tol=TOL, maxit=300)
    torch.cuda.synchronize()
    X = Xd.cpu().numpy()
    assert res[2].converged and res[2].iters == 0 and np.all(X[2] == 0.0)
    for r in (0, 1, 3, 4):
        assert res[r].converged, res[r]
        ref = spla.spsolve(Asp, B[r])
        assert np.linalg.norm(X[r] - ref) / np.linalg.norm(ref) < 1e-7
        # the relative residual is measured against the initial guess's residual
        r0 = np.linalg.norm(B[r] - Asp @ X0[r])
        assert np.linalg.norm(B[r] - Asp @ X[r]) <= TOL * r0 * 1.01
    s.close()


def test_rejected_cases():
    hs = amg.problems.laplace(3)
    s = amg.AMGSolver(hs, smoother="GS-1-1", krylov="PCG")
    B = torch.zeros((9, hs.dofs), dtype=torch.float64, device=DEV)
    with pytest.raises(amg.AmgError):
        s.solve_multi(B, torch.zeros_like(B))
    s.close()
    s = amg.AMGSolver(hs, smoother="GS-1-1", krylov="NONE")
    B = torch.zeros((2, hs.dofs), dtype=torch.float64, device=DEV)
    with pytest.raises(amg.AmgError):
        s.solve_multi(B, torch.zeros_like(B))
    s.close()
    cav = amg.problems.stokes_cavity(3, 1.0)
    s = amg.AMGSolver(cav, smoother="BS-1-1", krylov="FGMRES")
    B = torch.zeros((2, cav.dofs), dtype=torch.float64, device=DEV)
    with pytest.raises(amg.AmgError):
        s.solve_multi(B, torch.zeros_like(B))
    s.close()
