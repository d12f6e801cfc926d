"""Batches of saddle point systems of different size and depth merged into
one hierarchy: the merged V-cycle equals each system's own V-cycle, the
batched FGMRES reproduces each system's own solve, and both agree with the
FP64 oracle."""
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


def mixed_batch():
    # cavities and a compressible mixed-elasticity system (with C), hierarchies of 2..4 levels
    return [amg.problems.stokes_cavity(5, 0.7), amg.problems.mixed_elasticity(3, nu=0.3),
            amg.problems.stokes_cavity(3, 1.2), amg.problems.stokes_cavity(7, 1.6),
            amg.problems.mixed_elasticity(5), amg.problems.stokes_cavity(4, 1.9)]


@pytest.fixture(scope="module")
def systems():
    return mixed_batch()


def _split(v, systems):
    out, o = [], 0
    for s in systems:
        out.append(v[o:o + s.dofs])
        o += s.dofs
    return out


def _centre(v, s):
    v = v.copy()
    if s.pressure_kernel:
        nu = 3 * s.nodes
        v[nu:] -= v[nu:].mean()
    return v


@pytest.mark.parametrize("smoother", ["BS-1-1", "sGS-1-1"])
def test_merged_cycle_is_each_systems_cycle(systems, smoother):
    bsol = amg.BatchedSolver(systems, smoother=smoother)
    singles = [amg.AMGSolver(s, smoother=smoother, krylov="FGMRES") for s in systems]
    depths = [s.num_levels for s in singles]
    assert len(set(depths)) > 1, depths        # the batch mixes depths
    assert bsol.num_levels == max(depths)
    uo, po = bsol.offsets()
    nu_all = 3 * sum(s.nodes for s in systems)
    rng = np.random.default_rng(5)
    rs = [rng.standard_normal(s.dofs) for s in systems]
    merged = np.zeros(bsol.n)
    for s, r, u, q in zip(systems, rs, uo, po):
        nu = 3 * s.nodes
        merged[u:u + nu] = r[:nu]
        merged[nu_all + q:nu_all + q + s.n_pres] = r[nu:]
    z = torch.zeros(bsol.n, dtype=torch.float64, device=DEV)
    bsol.precondition(dev(merged), z)
    zm = host(z)
    for s, r, u, q, single in zip(systems, rs, uo, po, singles):
        nu = 3 * s.nodes
        zs = torch.zeros(s.dofs, dtype=torch.float64, device=DEV)
        single.precondition(dev(r), zs)
        got = np.concatenate([zm[u:u + nu], zm[nu_all + q:nu_all + q + s.n_pres]])
        assert rel(got, host(zs)) < 1e-12, s.name
        single.close()
    bsol.close()


@pytest.mark.parametrize("smoother", ["BS-1-1", "sGS-1-1"])
def test_batched_solve_matches_single_solves(systems, smoother):
    tol = 1e-9
    bsol = amg.BatchedSolver(systems, smoother=smoother)
    b = dev(np.concatenate([s.rhs for s in systems]))
    x = torch.zeros_like(b)
    res = bsol.solve(b, x, tol=tol, maxit=300)
    xs = _split(host(x), systems)
    for s, r, xi in zip(systems, res, xs):
        assert r.converged and r.relres <= tol * 1.01, (s.name, r)
        single = amg.AMGSolver(s, smoother=smoother, krylov="FGMRES")
        xd = torch.zeros(s.dofs, dtype=torch.float64, device=DEV)
        rr = single.solve(dev(s.rhs), xd, tol=tol, maxit=300)
        assert abs(r.iters - rr.iters) <= 1, (s.name, r.iters, rr.iters)
        ref = _centre(host(xd), s)
        assert np.linalg.norm(_centre(xi, s) - ref) / np.linalg.norm(ref) < 1e-7, s.name
        single.close()
    bsol.close()


def test_batched_solve_matches_oracle():
    hs = [amg.problems.stokes_cavity(4, 1.3), amg.problems.mixed_elasticity(3, nu=0.3)]
    os_ = [workloads.stokes(4, 1.3), workloads.mixed_elasticity(3, nu=0.3)]
    bsol = amg.BatchedSolver(hs, smoother="BS-1-1")
    b = dev(np.concatenate([s.rhs for s in hs]))
    x = torch.zeros_like(b)
    res = bsol.solve(b, x, tol=1e-9)
    for s, o, r, xi in zip(hs, os_, res, _split(host(x), hs)):
        h = oamg.setup(o.A, o.nlin, o.nquad, B=o.B, C=o.C, singular=o.singular)
        oamg.prepare_bs(h)
        prec = oamg.preconditioner(h, oamg.Smoother.parse("BS-1-1"))
        A, B = o.A, o.B
        Bt = B.transpose()
        nv = 3 * A.nrows

        def mv(z, A=A, B=B, Bt=Bt, o=o, nv=nv):
            u, p = z[:nv].reshape(-1, 3), z[nv:]
            top = A.matvec(u).ravel() + Bt.matvec(p.reshape(-1, 1)).ravel()
            bot = B.matvec(u)[:, 0]
            if o.C is not None:
                bot = bot - o.C.matvec(p.reshape(-1, 1))[:, 0]
            return np.concatenate([top, bot])
        ref = krylov.fgmres(mv, prec, np.concatenate([o.f.ravel(), o.g]), tol=1e-9)
        assert abs(r.iters - ref.iters) <= 1, (s.name, r.iters, ref.iters)
        refx = _centre(ref.x, s)
        assert np.linalg.norm(_centre(xi, s) - refx) / np.linalg.norm(refx) < 1e-7
    bsol.close()


def test_batch_of_one_and_errors():
    s = amg.problems.stokes_cavity(4, 1.0)
    bsol = amg.BatchedSolver([s], smoother="BS-1-1")
    x = torch.zeros(s.dofs, dtype=torch.float64, device=DEV)
    res = bsol.solve(dev(s.rhs), x, tol=1e-8)
    single = amg.AMGSolver(s, smoother="BS-1-1", krylov="FGMRES")
    xd = torch.zeros_like(x)
    rr = single.solve(dev(s.rhs), xd, tol=1e-8)
    assert res[0].iters == rr.iters
    assert rel(_centre(host(x), s), _centre(host(xd), s)) < 1e-10
    # a batch handle refuses the single-system solve; SPD systems are not batched
    with pytest.raises(amg.AmgError):
        amg.lib()  # library loaded
        from paper_1503_01287_amd import _lib as C
        import ctypes
        r = C.AmgResult()
        C.check(C.lib().amg_solve(bsol.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(xd.data_ptr()), 1e-8, 10,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(r)),
                "amg_solve")
    with pytest.raises(amg.AmgError):
        amg.BatchedSolver([s, amg.problems.laplace(3)], smoother="BS-1-1")
    bsol.close()
    single.close()
