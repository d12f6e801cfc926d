"""The saddle V-cycle's explicit coarse end: below the finest level the cycle
from a zero guess is a linear map of its right-hand side, assembled once per
system and applied as one GEMV. With it in place the preconditioner must be
the same map as the launch-by-launch cycle (up to rounding) and as the FP64
oracle's V-cycle, for every saddle smoother, in both precisions and in a
batch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1503_01287_amd as amg  # noqa: E402
from oracle import amg as oamg, workloads  # noqa: E402

DEV = torch.device("cuda:0")


def _fused_levels(s):
    return [l for l in range(s.num_levels) if s.level_info(l).fused]


def _apply(s, r):
    z = torch.zeros_like(r)
    s.precondition(r, z)
    torch.cuda.synchronize()
    return z.cpu().numpy()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("smoother,precision,tol", [
    ("sGS-1-1", "FP64", 1e-11), ("BS-1-1", "FP64", 1e-11), ("Vanka-1-1", "FP64", 1e-11),
    ("sGS-2-2", "FP64", 1e-11), ("sGS-1-1", "MIXED", 2e-4), ("BS-1-1", "FP32", 2e-4)])
@pytest.mark.parametrize("kind", ["mixed", "cavity"])
def test_tail_is_the_cycle(kind, smoother, precision, tol):
    # Vanka's cycle is the costliest to assemble (one cycle per column):
    # smaller systems keep its assembly inside the setup budget
    small = smoother.startswith("Vanka")
    if kind == "mixed":
        sysm = amg.problems.mixed_elasticity(5 if small else 8)
    else:
        sysm = amg.problems.stokes_cavity(4 if small else 6, 1.1)
    kw = dict(smoother=smoother, krylov="FGMRES", precision=precision)
    fused = amg.AMGSolver(sysm, fuse_coarse=True, **kw)
    plain = amg.AMGSolver(sysm, fuse_coarse=False, **kw)
    assert _fused_levels(fused), "the coarse end was not assembled"
    assert not _fused_levels(plain)
    rng = np.random.default_rng(7)
    r = torch.from_numpy(rng.standard_normal(sysm.dofs)).to(DEV)
    zf, zp = _apply(fused, r), _apply(plain, r)
    if sysm.pressure_kernel:
        nv = 3 * sysm.nodes
        zf[nv:] -= zf[nv:].mean()
        zp[nv:] -= zp[nv:].mean()
    assert _rel(zf, zp) < tol, (smoother, precision, _rel(zf, zp))
    # whole solves: same iteration counts up to one
    b = torch.from_numpy(sysm.rhs).to(DEV)
    xf, xp = torch.zeros_like(b), torch.zeros_like(b)
    rf = fused.solve(b, xf, tol=1e-8, maxit=300)
    rp = plain.solve(b, xp, tol=1e-8, maxit=300)
    assert rf.converged and rp.converged
    assert abs(rf.iters - rp.iters) <= 1, (rf.iters, rp.iters)
    fused.close()
    plain.close()


def test_tail_matches_oracle_vcycle():
    sysm = amg.problems.mixed_elasticity(6)
    s = amg.AMGSolver(sysm, smoother="sGS-1-1", krylov="FGMRES")
    assert 1 in _fused_levels(s)
    o = workloads.mixed_elasticity(6)
    h = oamg.setup(o.A, o.nlin, o.nquad, B=o.B, C=o.C, singular=o.singular)
    prec = oamg.preconditioner(h, oamg.Smoother.parse("sGS-1-1"))
    rng = np.random.default_rng(11)
    r = rng.standard_normal(sysm.dofs)
    z = _apply(s, torch.from_numpy(r).to(DEV))
    zo = prec(r)
    assert _rel(z, zo) < 1e-10, _rel(z, zo)
    s.close()


def test_batched_tail_is_each_systems_cycle():
    systems = [amg.problems.stokes_cavity(n, a) for n, a in ((6, 0.7), (4, 1.5), (7, 1.0), (5, 1.9))]
    fused = amg.BatchedSolver(systems, smoother="BS-1-1", fuse_coarse=True)
    plain = amg.BatchedSolver(systems, smoother="BS-1-1", fuse_coarse=False)
    assert _fused_levels(fused), "the coarse end was not assembled"
    assert not _fused_levels(plain)
    rng = np.random.default_rng(3)
    r = torch.from_numpy(rng.standard_normal(fused.n)).to(DEV)
    zf, zp = _apply(fused, r), _apply(plain, r)
    # merged layout [u of all systems; p of all systems]
    u, q = fused.offsets()
    nu_all = 3 * sum(s.nodes for s in systems)
    for s, uo, po in zip(systems, u, q):
        nu = 3 * s.nodes
        assert _rel(zf[uo:uo + nu], zp[uo:uo + nu]) < 1e-11, s.name
        pf = zf[nu_all + po:nu_all + po + s.n_pres]
        pp = zp[nu_all + po:nu_all + po + s.n_pres]
        assert _rel(pf, pp) < 1e-11, s.name
    fused.close()
    plain.close()
