"""Determinism through the C ABI: every kernel sums in a fixed order, so
solves on one hierarchy repeat bit for bit (with the setup-time tuners on),
and with the tuners off (autotune = 0: no setup choice depends on timing)
two setups of the same input give the same bits."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1503_01287_amd as amg  # noqa: E402

DEV = torch.device("cuda:0")

CASES = {
    "elasticity7-GS-FCG-MIXED": (lambda: amg.problems.elasticity(7),
                                 dict(smoother="GS-1-1", krylov="FCG", precision="MIXED")),
    "laplace6-JA-PCG": (lambda: amg.problems.laplace(6), dict(smoother="JA-1-1-0.5", krylov="PCG")),
    "mixed4-sGS-FGMRES-MIXED": (lambda: amg.problems.mixed_elasticity(4, nu=0.3),
                                dict(smoother="sGS-1-1", krylov="FGMRES", precision="MIXED")),
    "cavity5-BS-FGMRES": (lambda: amg.problems.stokes_cavity(5, 1.4), dict(smoother="BS-1-1", krylov="FGMRES")),
}


def _solve(s, hs):
    b = torch.from_numpy(np.ascontiguousarray(hs.rhs)).to(DEV)
    x = torch.zeros_like(b)
    r = s.solve(b, x, tol=1e-10, maxit=500)
    torch.cuda.synchronize()
    assert r.converged, r
    return r.iters, x.cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_repeated_solves_on_one_hierarchy_are_bitwise(name):
    hs = CASES[name][0]()
    s = amg.AMGSolver(hs, **CASES[name][1])
    it1, x1 = _solve(s, hs)
    it2, x2 = _solve(s, hs)
    s.close()
    assert it1 == it2 and np.array_equal(x1, x2), name


@pytest.mark.parametrize("name", list(CASES))
def test_two_setups_without_tuner_are_bitwise(name):
    hs = CASES[name][0]()
    out = []
    for _ in range(2):
        s = amg.AMGSolver(hs, autotune=False, **CASES[name][1])
        out.append(_solve(s, hs))
        s.close()
    assert out[0][0] == out[1][0] and np.array_equal(out[0][1], out[1][1]), name


def test_two_batch_setups_without_tuner_are_bitwise():
    systems = [amg.problems.stokes_cavity(5, 0.7), amg.problems.mixed_elasticity(3, nu=0.3),
               amg.problems.stokes_cavity(4, 1.2)]
    b = torch.from_numpy(np.concatenate([s.rhs for s in systems])).to(DEV)
    out = []
    for _ in range(2):
        bsol = amg.BatchedSolver(systems, smoother="BS-1-1", precision="FP32", autotune=False)
        x = torch.zeros_like(b)
        res = bsol.solve(b, x, tol=1e-9, maxit=400)
        torch.cuda.synchronize()
        assert all(r.converged for r in res), res
        out.append(([r.iters for r in res], x.cpu().numpy()))
        bsol.close()
    assert out[0][0] == out[1][0] and np.array_equal(out[0][1], out[1][1])
