"""Batches of independent SPD systems of different size and depth merged
into one hierarchy (amg_setup_batched / amg_solve_batched with every
n_pres = 0): the merged cycle equals each system's own cycle (FP64, and the
FP32 / BF16 cycles up to FP32 summation order), the lockstep PCG and FCG
reproduce each system's own solve (within one iteration) and the oracle's
solution, systems that are solved directly on the finest level, zero
right-hand sides and the rejected configurations."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1503_01287_amd as amg  # noqa: E402
from oracle import workloads  # noqa: E402

DEV = torch.device("cuda:0")
TOL = 1e-10


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


BATCHES = {
    # 3x3 blocks: elasticity of 1 (directly solved), 2 .. 4 levels
    "elasticity": lambda: [amg.problems.elasticity(4), amg.problems.elasticity(1), amg.problems.elasticity(6, i=1),
                           amg.problems.elasticity(3, i=2), amg.problems.elasticity(5, i=3)],
    # scalar operator applied per component
    "laplace": lambda: [amg.problems.laplace(5), amg.problems.laplace(2), amg.problems.laplace(7)],
}


@pytest.fixture(scope="module", params=list(BATCHES))
def batch(request):
    return request.param, BATCHES[request.param]()


def _single(sysm, smoother, nu=1):
    return amg.AMGSolver(sysm, smoother=smoother, krylov="PCG", nu=nu, fuse_coarse=False, autotune=False)


@pytest.mark.parametrize("smoother,nu", [("GS-1-1", 1), ("JA-1-1-0.5", 1), ("GS-2-2", 2)])
def test_merged_cycle_is_every_system_own_cycle(batch, smoother, nu):
    name, systems = batch
    bs = amg.BatchedSolver(systems, smoother=smoother, nu=nu, autotune=False)
    uoff, _ = bs.offsets()
    rng = np.random.default_rng(3)
    rs = [rng.standard_normal(s.dofs) for s in systems]
    merged = np.zeros(bs.n)
    for s, r, o in zip(systems, rs, uoff):
        merged[o:o + s.dofs] = r
    z = torch.zeros(bs.n, dtype=torch.float64, device=DEV)
    bs.precondition(dev(merged), z)
    zm = host(z)
    for s, r, o in zip(systems, rs, uoff):
        one = _single(s, smoother, nu)
        zo = torch.zeros(s.dofs, dtype=torch.float64, device=DEV)
        one.precondition(dev(r), zo)
        assert rel(zm[o:o + s.dofs], host(zo)) < 1e-11, (name, smoother, s.dofs)
        one.close()
    bs.close()


@pytest.mark.parametrize("smoother", ["GS-1-1", "JA-1-1-0.5"])
def test_batched_pcg_matches_single_solves_and_oracle(batch, smoother):
    name, systems = batch
    bs = amg.BatchedSolver(systems, smoother=smoother)
    b = np.concatenate([s.rhs for s in systems])
    x = torch.zeros(bs.n, dtype=torch.float64, device=DEV)
    res = bs.solve(dev(b), x, tol=TOL, maxit=300)
    X = host(x)
    o = 0
    for s, r in zip(systems, res):
        assert r.converged and r.relres <= TOL * 1.01, (name, s.dofs, r)
        one = amg.AMGSolver(s, smoother=smoother, krylov="PCG")
        x1 = torch.zeros(s.dofs, dtype=torch.float64, device=DEV)
        r1 = one.solve(dev(s.rhs), x1, tol=TOL, maxit=300)
        assert abs(r1.iters - r.iters) <= 1, (name, s.dofs, r1.iters, r.iters)
        xs = X[o:o + s.dofs]
        assert rel(xs, host(x1)) < 1e-8
        one.close()
        o += s.dofs
    bs.close()


def test_batched_solution_against_oracle():
    systems = BATCHES["elasticity"]()
    bs = amg.BatchedSolver(systems, smoother="GS-1-1")
    b = np.concatenate([s.rhs for s in systems])
    x = torch.zeros(bs.n, dtype=torch.float64, device=DEV)
    res = bs.solve(dev(b), x, tol=1e-11, maxit=300)
    X = host(x)
    oracles = [workloads.elasticity(4), workloads.elasticity(1), workloads.elasticity(6, i=1),
               workloads.elasticity(3, i=2), workloads.elasticity(5, i=3)]
    o = 0
    for s, r, ow in zip(systems, res, oracles):
        assert r.converged
        ref = spla.spsolve(ow.A.scipy().tocsc(), ow.b.ravel())
        assert rel(X[o:o + s.dofs], ref) < 1e-8, s.dofs
        o += s.dofs
    bs.close()


def test_zero_rhs_and_initial_guess():
    systems = BATCHES["laplace"]()
    bs = amg.BatchedSolver(systems, smoother="GS-1-1")
    b = [s.rhs.copy() for s in systems]
    b[1][:] = 0.0
    x0 = [np.random.default_rng(5 + k).standard_normal(s.dofs) for k, s in enumerate(systems)]
    x0[1][:] = 0.0
    x = dev(np.concatenate(x0))
    res = bs.solve(dev(np.concatenate(b)), x, tol=TOL, maxit=300)
    X = host(x)
    assert res[1].converged and res[1].iters == 0
    o = 0
    for k, (s, r) in enumerate(zip(systems, res)):
        assert r.converged, (k, r)
        if k == 1:
            assert np.all(X[o:o + s.dofs] == 0.0)
        o += s.dofs
    bs.close()


@pytest.mark.parametrize("precision", ["MIXED", "FP32"])
@pytest.mark.parametrize("smoother,nu", [("GS-1-1", 1), ("JA-1-1-0.5", 1), ("GS-1-1", 2)])
def test_merged_reduced_cycle_is_every_system_own_cycle(batch, precision, smoother, nu):
    """The FP32 / BF16 merged cycle against each system's own reduced cycle
    (no assembled coarse end, heuristic launch shapes): the same rounded
    operators, so they agree up to FP32 summation order (the merged levels'
    lane counts follow the batch's mean row, not each system's)."""
    name, systems = batch
    bs = amg.BatchedSolver(systems, smoother=smoother, nu=nu, precision=precision, autotune=False)
    uoff, _ = bs.offsets()
    rng = np.random.default_rng(4)
    rs = [rng.standard_normal(s.dofs) for s in systems]
    merged = np.zeros(bs.n)
    for s, r, o in zip(systems, rs, uoff):
        merged[o:o + s.dofs] = r
    z = torch.zeros(bs.n, dtype=torch.float64, device=DEV)
    bs.precondition(dev(merged), z)
    zm = host(z)
    for s, r, o in zip(systems, rs, uoff):
        one = amg.AMGSolver(s, smoother=smoother, krylov="FCG", nu=nu, precision=precision, fuse_coarse=False,
                            autotune=False)
        zo = torch.zeros(s.dofs, dtype=torch.float64, device=DEV)
        one.precondition(dev(r), zo)
        assert rel(zm[o:o + s.dofs], host(zo)) < 1e-5, (name, precision, smoother, s.dofs)
        one.close()
    bs.close()


@pytest.mark.parametrize("precision", ["MIXED", "FP32", "FP64"])
def test_batched_fcg_matches_single_solves(batch, precision):
    """Lockstep flexible CG (the default Krylov method of a reduced-precision
    batch): each system within one iteration of its own FCG solve with the
    same cycle, at its FP64 solution."""
    name, systems = batch
    bs = amg.BatchedSolver(systems, smoother="GS-1-1", precision=precision, krylov="FCG")
    b = np.concatenate([s.rhs for s in systems])
    x = torch.zeros(bs.n, dtype=torch.float64, device=DEV)
    res = bs.solve(dev(b), x, tol=TOL, maxit=300)
    X = host(x)
    o = 0
    for s, r in zip(systems, res):
        assert r.converged and r.relres <= TOL * 1.01, (name, precision, s.dofs, r)
        one = amg.AMGSolver(s, smoother="GS-1-1", krylov="FCG", precision=precision, fuse_coarse=False)
        x1 = torch.zeros(s.dofs, dtype=torch.float64, device=DEV)
        r1 = one.solve(dev(s.rhs), x1, tol=TOL, maxit=300)
        assert abs(r1.iters - r.iters) <= 1, (name, precision, s.dofs, r1.iters, r.iters)
        ref = amg.AMGSolver(s, smoother="GS-1-1", krylov="PCG")
        x2 = torch.zeros(s.dofs, dtype=torch.float64, device=DEV)
        ref.solve(dev(s.rhs), x2, tol=1e-12, maxit=300)
        assert rel(X[o:o + s.dofs], host(x2)) < 1e-7, (name, precision, s.dofs)
        one.close()
        ref.close()
        o += s.dofs
    bs.close()


def test_reduced_batch_default_krylov_and_zero_rhs():
    systems = BATCHES["elasticity"]()
    bs = amg.BatchedSolver(systems, precision="MIXED")
    assert bs.params.krylov == amg._lib.KRYLOV["FCG"]
    b = [s.rhs.copy() for s in systems]
    b[2][:] = 0.0
    x = torch.zeros(sum(s.dofs for s in systems), dtype=torch.float64, device=DEV)
    res = bs.solve(dev(np.concatenate(b)), x, tol=1e-8, maxit=300)
    X = host(x)
    assert res[2].converged and res[2].iters == 0
    o = sum(s.dofs for s in systems[:2])
    assert np.all(X[o:o + systems[2].dofs] == 0.0)
    assert all(r.converged for r in res)
    bs.close()


def test_rejected_configurations():
    el = [amg.problems.elasticity(3), amg.problems.elasticity(4)]
    for kw in (dict(krylov="FGMRES"), dict(smoother="sGS-1-1")):
        with pytest.raises(amg.AmgError):
            amg.BatchedSolver(el, **kw)
    with pytest.raises(amg.AmgError):
        amg.BatchedSolver([amg.problems.elasticity(3), amg.problems.laplace(3)])
    with pytest.raises(amg.AmgError):
        amg.BatchedSolver([amg.problems.elasticity(3), amg.problems.stokes_cavity(3, 1.0)])


def test_concurrent_setup_phases_and_repeatability():
    """The systems of a batch are set up on several host threads: the setup
    records the step's wall time and the systems' own phases summed, and two
    setups of one batch (no tuner) give the same preconditioner bit for bit."""
    systems = BATCHES["elasticity"]()
    a = amg.BatchedSolver(systems, smoother="GS-1-1", autotune=False)
    b = amg.BatchedSolver(systems, smoother="GS-1-1", autotune=False)
    wall = a.profile_read("setup.systems")
    assert wall["launches"] == 1 and wall["ms"] > 0.0
    for ph in ("upload", "coarsest"):  # once per system
        assert a.profile_read("setup.systems." + ph)["launches"] == len(systems), ph
    for ph in ("coarsen", "galerkin", "smoother"):  # per level of the systems that coarsen
        assert a.profile_read("setup.systems." + ph)["launches"] >= 1, ph
        assert a.profile_read("setup." + ph)["launches"] == 0, ph
    assert a.profile_read("setup.merge")["launches"] == 1
    single = amg.AMGSolver(systems[0], smoother="GS-1-1", krylov="PCG")
    assert single.profile_read("setup.systems")["launches"] == 0
    single.close()
    r = dev(np.random.default_rng(9).standard_normal(a.n))
    za, zb = torch.zeros_like(r), torch.zeros_like(r)
    a.precondition(r, za)
    b.precondition(r, zb)
    torch.cuda.synchronize()
    assert torch.equal(za, zb)
    a.close()
    b.close()
