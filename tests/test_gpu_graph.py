"""Recorded (HIP graph) preconditioner applications against the same
launches made one by one: identical bits for every replay, with eager work
and synchronisations between the replays, for every solver path."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1503_01287_amd as amg  # noqa: E402

DEV = torch.device("cuda:0")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


SPD = {
    "elast5-GS-PCG-FP64": (lambda: amg.problems.elasticity(5), dict(smoother="GS-1-1", krylov="PCG")),
    "laplace7-JA-FCG-MIXED": (lambda: amg.problems.laplace(7), dict(smoother="JA-1-1-0.5", krylov="FCG",
                                                                   precision="MIXED")),
    "elast4-GS-FGMRES-2cycles": (lambda: amg.problems.elasticity(4), dict(smoother="GS-1-1", krylov="FGMRES",
                                                                        cycles=2)),
    "cavity4-BS-FGMRES": (lambda: amg.problems.stokes_cavity(4, 1.1), dict(smoother="BS-1-1", krylov="FGMRES")),
    "mixed3-sGS-FGMRES": (lambda: amg.problems.mixed_elasticity(3, nu=0.3), dict(smoother="sGS-1-1",
                                                                               krylov="FGMRES")),
}


@pytest.mark.parametrize("name", list(SPD))
def test_recorded_solves_and_preconditioners_are_bitwise_eager(name):
    make, kw = SPD[name]
    hs = make()
    eager = amg.AMGSolver(hs, graph=False, autotune=False, **kw)
    rec = amg.AMGSolver(hs, graph=True, autotune=False, **kw)
    rng = np.random.default_rng(11)
    for rep in range(3):
        b = dev(hs.rhs * (1.0 + rep) + (rep > 0) * rng.standard_normal(hs.dofs))
        xe, xr = torch.zeros_like(b), torch.zeros_like(b)
        re = eager.solve(b, xe, tol=1e-9, maxit=300)
        torch.cuda.synchronize()
        rr = rec.solve(b, xr, tol=1e-9, maxit=300)
        torch.cuda.synchronize()
        assert re.iters == rr.iters and re.status == rr.status, (name, rep, re, rr)
        assert torch.equal(xe, xr), (name, rep)
        # single preconditioner applications between the solves
        r = dev(rng.standard_normal(hs.dofs))
        ze, zr = torch.zeros_like(r), torch.zeros_like(r)
        eager.precondition(r, ze)
        rec.precondition(r, zr)
        torch.cuda.synchronize()
        assert torch.equal(ze, zr), (name, rep)
    eager.close()
    rec.close()


def test_recorded_batch_is_bitwise_eager():
    systems = [amg.problems.stokes_cavity(4, 1.3), amg.problems.mixed_elasticity(3, nu=0.3),
               amg.problems.stokes_cavity(6, 0.6)]
    # (no setup tuner: two tuned setups may pick different launch shapes,
    # which changes rounding; the comparison is of graph against eager)
    eager = amg.BatchedSolver(systems, smoother="BS-1-1", graph=False, autotune=False)
    rec = amg.BatchedSolver(systems, smoother="BS-1-1", graph=True, autotune=False)
    b = dev(np.concatenate([s.rhs for s in systems]))
    for rep in range(2):
        xe, xr = torch.zeros_like(b), torch.zeros_like(b)
        re = eager.solve(b * (rep + 1), xe, tol=1e-9)
        rr = rec.solve(b * (rep + 1), xr, tol=1e-9)
        torch.cuda.synchronize()
        assert [q.iters for q in re] == [q.iters for q in rr]
        assert torch.equal(xe, xr)
    eager.close()
    rec.close()


def test_new_weights_drop_recorded_preconditioners():
    hs = amg.problems.laplace(6)
    rec = amg.AMGSolver(hs, smoother="JA-1-1-0.5", graph=True, autotune=False)
    b = dev(hs.rhs)
    x = torch.zeros_like(b)
    rec.solve(b, x, tol=1e-9)
    rec.set_level_omega([0.7, 0.8])
    x.zero_()
    r1 = rec.solve(b, x, tol=1e-9)
    ref = amg.AMGSolver(hs, smoother="JA-1-1-0.5", graph=False, autotune=False, level_omega=[0.7, 0.8])
    y = torch.zeros_like(b)
    r2 = ref.solve(b, y, tol=1e-9)
    torch.cuda.synchronize()
    assert r1.iters == r2.iters and torch.equal(x, y)
    rec.close()
    ref.close()
