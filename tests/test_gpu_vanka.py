"""Parity of the multiplicative Vanka smoother (Section 3.3) with the FP64
oracle: one sweep, the saddle V-cycle with it, FGMRES."""
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
    "mixed4-nu0.49999": (lambda: amg.problems.mixed_elasticity(4), lambda: workloads.mixed_elasticity(4)),
    "cavity4": (lambda: amg.problems.stokes_cavity(4, 1.3), lambda: workloads.stokes(4, 1.3)),
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
    hs_, os_ = CASES[request.param]
    o = os_()
    h = oamg.setup(o.A, o.nlin, o.nquad, B=o.B, C=o.C, singular=o.singular)
    return request.param, hs_(), o, h


def _mv(o):
    Bt = o.B.transpose()
    nv = 3 * o.A.nrows

    def mv(z):
        u, p = z[:nv].reshape(-1, 3), z[nv:]
        top = o.A.matvec(u).ravel() + Bt.matvec(p.reshape(-1, 1)).ravel()
        bot = o.B.matvec(u)[:, 0]
        if o.C is not None:
            bot = bot - o.C.matvec(p.reshape(-1, 1))[:, 0]
        return np.concatenate([top, bot])
    return mv


def test_vanka_tiled_sweep_every_residual_width(case):
    """The spread-residual forms (2-D tiles and their sum; 64-row tiles)
    forced on every level with 16, 32 and 64 lanes per residual row: each
    sweep equals the oracle's."""
    name, hs, o, h = case
    s = amg.AMGSolver(hs, smoother="Vanka-1-1", krylov="FGMRES", autotune=False)
    sm = oamg.Smoother.parse("Vanka-1-1")
    rng = np.random.default_rng(52)
    for l in range(len(h.levels) - 1):
        lev = h.levels[l]
        nv = 3 * lev.n
        n = nv + lev.npres
        z, b = rng.standard_normal(n), rng.standard_normal(n)
        u, p = oamg.vanka_step(lev, sm, b[:nv].reshape(-1, 3), b[nv:], z[:nv].reshape(-1, 3), z[nv:])
        ref = np.concatenate([u.ravel(), p])
        for form in (1, 2):
            for lanes in (16, 32, 64):
                s.set_launch_shape(l, "vanka", lanes, form)
                for waves in ((4, 8, 16) if form == 2 else (None,)):
                    if waves:
                        s.set_launch_shape(l, "vanka_apply", waves)
                    xd = dev(z)
                    s.smooth(l, dev(b), xd)
                    assert rel(host(xd), ref) < 1e-11, (name, l, form, lanes, waves)
    with pytest.raises(amg.AmgError):
        s.set_launch_shape(0, "vanka", 8)
    with pytest.raises(amg.AmgError):
        s.set_launch_shape(0, "vanka", 32, 4)
    with pytest.raises(amg.AmgError):
        s.set_launch_shape(0, "vanka_apply", 32)
    with pytest.raises(amg.AmgError):
        s.set_launch_shape(len(h.levels) - 1, "vanka", 16)
    s.close()
    spd = amg.AMGSolver(amg.problems.elasticity(3), smoother="GS-1-1", krylov="PCG")
    with pytest.raises(amg.AmgError):
        spd.set_launch_shape(0, "vanka", 16)
    spd.close()


@pytest.mark.parametrize("autotune", [True, False])
def test_vanka_sweep(case, autotune):
    """Every level; without the tuner, patches above 256 unknowns take the
    two-kernel path and the others the fused one."""
    name, hs, o, h = case
    s = amg.AMGSolver(hs, smoother="Vanka-1-1", krylov="FGMRES", autotune=autotune)
    sm = oamg.Smoother.parse("Vanka-1-1")
    rng = np.random.default_rng(51)
    for l in range(len(h.levels) - 1):
        lev = h.levels[l]
        nv = 3 * lev.n
        n = nv + lev.npres
        z, b = rng.standard_normal(n), rng.standard_normal(n)
        xd = dev(z)
        s.smooth(l, dev(b), xd)
        u, p = oamg.vanka_step(lev, sm, b[:nv].reshape(-1, 3), b[nv:], z[:nv].reshape(-1, 3), z[nv:])
        assert rel(host(xd), np.concatenate([u.ravel(), p])) < 1e-11, (name, l)
    s.close()


@pytest.mark.parametrize("cycles", [1, 2])
def test_vanka_vcycle(case, cycles):
    name, hs, o, h = case
    s = amg.AMGSolver(hs, smoother="Vanka-1-1", krylov="FGMRES", cycles=cycles)
    prec = oamg.preconditioner(h, oamg.Smoother.parse("Vanka-1-1"), cycles=cycles)
    r = np.random.default_rng(52).standard_normal(hs.dofs)
    z = torch.zeros(hs.dofs, dtype=torch.float64, device=DEV)
    s.precondition(dev(r), z)
    assert rel(host(z), prec(r)) < 1e-10, name
    s.close()


def test_vanka_fgmres(case):
    name, hs, o, h = case
    tol = 1e-9
    s = amg.AMGSolver(hs, smoother="Vanka-1-1", krylov="FGMRES")
    b = dev(hs.rhs)
    x = torch.zeros_like(b)
    res = s.solve(b, x, tol=tol, maxit=300)
    assert res.converged and res.relres <= tol * 1.01, (name, res)
    prec = oamg.preconditioner(h, oamg.Smoother.parse("Vanka-1-1"))
    ref = krylov.fgmres(_mv(o), prec, np.concatenate([o.f.ravel(), o.g]), tol=tol, maxit=300)
    assert abs(res.iters - ref.iters) <= 1, (name, res.iters, ref.iters)
    xs, rx = host(x), ref.x.copy()
    nv = 3 * o.A.nrows
    if o.singular:
        xs[nv:] -= xs[nv:].mean()
        rx[nv:] -= rx[nv:].mean()
    assert np.linalg.norm(xs - rx) / np.linalg.norm(rx) < 1e-7
    s.close()


def test_vanka_damping_and_limits():
    hs, o = amg.problems.mixed_elasticity(3, nu=0.3), workloads.mixed_elasticity(3, nu=0.3)
    h = oamg.setup(o.A, o.nlin, o.nquad, B=o.B, C=o.C)
    s = amg.AMGSolver(hs, smoother="Vanka-1-1-0.6", krylov="FGMRES")
    lev = h.levels[0]
    nv = 3 * lev.n
    rng = np.random.default_rng(53)
    z, b = rng.standard_normal(hs.dofs), rng.standard_normal(hs.dofs)
    xd = dev(z)
    s.smooth(0, dev(b), xd)
    u, p = oamg.vanka_step(lev, oamg.Smoother.parse("Vanka-1-1-0.6"), b[:nv].reshape(-1, 3), b[nv:],
                           z[:nv].reshape(-1, 3), z[nv:])
    assert rel(host(xd), np.concatenate([u.ravel(), p])) < 1e-11
    s.close()
    with pytest.raises(amg.AmgError):
        amg.AMGSolver(hs, smoother="Vanka-1-1", krylov="FGMRES", precision="FP32")
    with pytest.raises(amg.AmgError):
        amg.BatchedSolver([hs], smoother="Vanka-1-1")
