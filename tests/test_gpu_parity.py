"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Element-by-element comparisons on seeded inputs at sizes the oracle handles
in seconds (several tiles and ragged tails: rows of 7..70 blocks, colour
groups of uneven length), plus the full-size elasticity workload checked
through properties that hold at any size.
"""
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


CASES = {
    "laplace4": (lambda: amg.problems.laplace(4), lambda: workloads.laplace(4)),
    "laplace6": (lambda: amg.problems.laplace(6), lambda: workloads.laplace(6)),
    "elast4": (lambda: amg.problems.elasticity(4), lambda: workloads.elasticity(4)),
    "elast7": (lambda: amg.problems.elasticity(7), lambda: workloads.elasticity(7)),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    hs, os_ = CASES[request.param]
    return request.param, hs(), os_()


def _oracle_hierarchy(o, smoother="GS-1-1"):
    return oamg.setup(o.A, o.nlin, o.nquad)


def test_spmv_level0(case):
    name, hsys, o = case
    s = amg.AMGSolver(hsys, smoother="GS-1-1")
    rng = np.random.default_rng(11)
    x = rng.standard_normal(hsys.dofs)
    y = torch.zeros(hsys.dofs, dtype=torch.float64, device=DEV)
    s.apply(0, dev(x), y)
    ref = o.A.matvec(x).ravel()
    assert rel(host(y), ref) < 1e-14, name


def test_hierarchy_matches_oracle(case):
    """Level sizes and prolongations bit-exact; Galerkin operators to 1e-13."""
    name, hsys, o = case
    s = amg.AMGSolver(hsys, smoother="GS-1-1")
    h = _oracle_hierarchy(o)
    assert s.num_levels == len(h.levels), name
    for l, lev in enumerate(h.levels):
        info = s.level_info(l)
        assert (info.n_lin, info.n_quad) == (lev.nlin, lev.nquad)
        rp, col, val = s.level_matrix(l, "A")
        assert np.array_equal(rp, lev.A.indptr) and np.array_equal(col, lev.A.indices)
        if hsys.bs == 1:
            blocks = np.zeros((col.shape[0], 3, 3))
            for c in range(3):
                blocks[:, c, c] = val[:, 0]
        else:
            blocks = val.reshape(-1, 3, 3)
        assert rel(blocks, lev.A.vals) < 1e-13, (name, l)
        if l < len(h.levels) - 1:
            prp, pcol, pval = s.level_matrix(l, "P")
            assert np.array_equal(prp, lev.P.indptr) and np.array_equal(pcol, lev.P.indices)
            assert np.array_equal(pval[:, 0], lev.P.data)
            assert np.array_equal(s.level_colors(l), lev.colors)


@pytest.mark.parametrize("smoother", ["GS-1-1", "JA-1-1-0.5"])
def test_smoother_step(case, smoother):
    name, hsys, o = case
    s = amg.AMGSolver(hsys, smoother=smoother)
    h = _oracle_hierarchy(o)
    sm = oamg.Smoother.parse(smoother)
    rng = np.random.default_rng(12)
    for l in range(len(h.levels) - 1):
        lev = h.levels[l]
        b = rng.standard_normal((lev.n, 3))
        x0 = rng.standard_normal((lev.n, 3))
        for fwd in (True, False):
            xd = dev(x0.ravel())
            s.smooth(l, dev(b.ravel()), xd, forward=fwd)
            if sm.kind == "GS":
                ref = oamg.gauss_seidel(lev, b, x0, forward=fwd)
            else:
                ref = oamg.jacobi(lev, b, x0, sm.omega)
            assert rel(host(xd), ref.ravel()) < 1e-12, (name, smoother, l, fwd)


@pytest.mark.parametrize("fuse", [True, False])
@pytest.mark.parametrize("smoother", ["GS-1-1", "JA-1-1-0.5", "GS-2-2", "JA-2-2-0.5"])
def test_vcycle(case, smoother, fuse):
    """One preconditioner application; fuse=True runs the smallest levels in
    the single-workgroup tail kernel, fuse=False launches every operation."""
    name, hsys, o = case
    s = amg.AMGSolver(hsys, smoother=smoother, fuse_coarse=fuse)
    h = _oracle_hierarchy(o)
    prec = oamg.preconditioner(h, oamg.Smoother.parse(smoother))
    r = np.random.default_rng(13).standard_normal(hsys.dofs)
    z = torch.zeros(hsys.dofs, dtype=torch.float64, device=DEV)
    s.precondition(dev(r), z)
    assert rel(host(z), prec(r).ravel()) < 1e-11, (name, smoother, fuse)


@pytest.mark.parametrize("cycles,nu", [(2, 1), (1, 2), (2, 2)])
def test_multiple_cycles_and_w_cycle(case, cycles, nu):
    """'2 V-cycles' per preconditioner application and the W-cycle (nu = 2)."""
    name, hsys, o = case
    s = amg.AMGSolver(hsys, smoother="GS-1-1", cycles=cycles, nu=nu)
    h = _oracle_hierarchy(o)
    prec = oamg.preconditioner(h, oamg.Smoother.parse("GS-1-1"), cycles=cycles, nu=nu)
    r = np.random.default_rng(14).standard_normal(hsys.dofs)
    z = torch.zeros(hsys.dofs, dtype=torch.float64, device=DEV)
    s.precondition(dev(r), z)
    assert rel(host(z), prec(r).ravel()) < 1e-11, (name, cycles, nu)


@pytest.mark.parametrize("fuse", [True, False])
@pytest.mark.parametrize("precision,tol", [("FP64", 1e-11), ("FP32", 2e-5)])
def test_vcycle_forward_post_smoothing(case, precision, tol, fuse):
    """gs_post='forward': the post-smoothing sweeps run forward like the
    pre-smoothing ones (the stand-alone form), level by level."""
    name, hsys, o = case
    s = amg.AMGSolver(hsys, smoother="GS-1-1", gs_post="forward", precision=precision, krylov="FCG",
                      fuse_coarse=fuse)
    assert not any(s.level_info(l).fused for l in range(s.num_levels))
    h = _oracle_hierarchy(o)
    sm = oamg.Smoother.parse("GS-1-1")
    sm.post_forward = True
    prec = oamg.preconditioner(h, sm)
    r = np.random.default_rng(15).standard_normal(hsys.dofs)
    z = torch.zeros(hsys.dofs, dtype=torch.float64, device=DEV)
    s.precondition(dev(r), z)
    assert rel(host(z), prec(r).ravel()) < tol, (name, precision, rel(host(z), prec(r).ravel()))


@pytest.mark.parametrize("smoother,kry,fuse,post", [("GS-1-1", "PCG", True, "auto"), ("GS-1-1", "PCG", False, "auto"),
                                                    ("JA-1-1-0.5", "PCG", True, "auto"),
                                                    ("GS-1-1", "FCG", True, "auto"),
                                                    ("GS-1-1", "NONE", True, "auto"),
                                                    ("GS-1-1", "NONE", True, "backward")])
def test_solve_matches_oracle(case, smoother, kry, fuse, post):
    name, hsys, o = case
    # the symmetric stand-alone iteration contracts by ~0.95 per cycle on elasticity
    tol = 1e-10 if kry != "NONE" else 1e-8
    s = amg.AMGSolver(hsys, smoother=smoother, krylov=kry, fuse_coarse=fuse, gs_post=post)
    b = dev(hsys.rhs)
    x = torch.zeros_like(b)
    res = s.solve(b, x, tol=tol, maxit=1000)
    assert res.converged and res.relres <= tol * 1.01, res
    h = _oracle_hierarchy(o)
    prec = oamg.preconditioner(h, oamg.Smoother.parse(smoother))
    mv = lambda v: o.A.matvec(v).ravel()
    if kry == "PCG":
        ref = krylov.pcg(mv, lambda r: prec(r).ravel(), o.b.ravel(), tol=tol)
    elif kry == "FCG":
        ref = krylov.fcg(mv, lambda r: prec(r).ravel(), o.b.ravel(), tol=tol)
    else:
        # the stand-alone solver sweeps forward after the coarse correction
        # too unless told otherwise
        ref = _stationary(o, h, smoother, tol, post_forward=post == "auto")
    assert abs(res.iters - ref.iters) <= 1, (name, res.iters, ref.iters)
    xs = host(x)
    assert np.linalg.norm(xs - ref.x) / np.linalg.norm(ref.x) < 1e-8


def _stationary(o, h, smoother, tol, post_forward=False):
    sm = oamg.Smoother.parse(smoother)
    sm.post_forward = post_forward
    b = o.b
    x = np.zeros_like(b)
    r0 = np.linalg.norm(b)
    it = 0
    while it < 1000:
        x = oamg.cycle(h, 0, sm, b, x)
        it += 1
        if np.linalg.norm(b - o.A.matvec(x)) / r0 <= tol:
            break
    return krylov.KrylovResult(x.ravel(), it, np.linalg.norm(b - o.A.matvec(x)) / r0, [], True)


def test_error_paths():
    hsys = amg.problems.laplace(3)
    s = amg.AMGSolver(hsys)
    b = dev(hsys.rhs)
    x = torch.zeros_like(b)
    res = s.solve(b, x, tol=1e-14, maxit=2)
    assert res.status == 1  # AMG_NOT_CONVERGED
    bad = b.clone()
    bad[5] = float("nan")
    x.zero_()
    res = s.solve(bad, x, tol=1e-8, maxit=50)
    assert res.status == 3  # AMG_DIVERGED
    with pytest.raises(amg.AmgError):
        s.apply(99, b, x)


def test_full_size_elasticity_properties():
    """32^3 elasticity (823,875 DOF): the hierarchy's level sizes equal the
    oracle's structural coarsening, PCG GS-1-1 reaches 1e-8 and the true
    FP64 residual of the returned solution, recomputed on the CPU from the
    assembled matrix, is below the tolerance."""
    from oracle import amg as oa, fem as ofem, mesh as omesh
    hsys = amg.problems.elasticity(32)
    s = amg.AMGSolver(hsys, smoother="GS-1-1")
    m = omesh.kuhn_mesh(32)
    sizes = oa.structural_sizes(ofem.structural_pattern(m), m.nv, m.ne)
    got = [(s.level_info(l).n_lin, s.level_info(l).n_quad) for l in range(s.num_levels)]
    assert got == sizes
    b = dev(hsys.rhs)
    x = torch.zeros_like(b)
    res = s.solve(b, x, tol=1e-8, maxit=300)
    assert res.converged, res
    xs = host(x)
    rows = np.repeat(np.arange(hsys.nodes), np.diff(hsys.A_rowptr))
    Ax = np.einsum("kij,kj->ki", hsys.A_val.reshape(-1, 3, 3), xs.reshape(-1, 3)[hsys.A_col])
    r = hsys.rhs.reshape(-1, 3).copy()
    for c in range(3):
        r[:, c] -= np.bincount(rows, weights=Ax[:, c], minlength=hsys.nodes)
    relres = np.linalg.norm(r) / np.linalg.norm(hsys.rhs)
    assert relres <= 1e-8 * 1.01 and abs(relres - res.relres) < 1e-10


# ---------------------------------------------------------------- mixed precision
@pytest.mark.parametrize("precision,tol_v", [("FP32", 1e-5), ("MIXED", 5e-2)])
def test_reduced_precision_vcycle(case, precision, tol_v):
    """FP32 / BF16-coarse V-cycle against the oracle's FP64 V-cycle: the
    difference is the rounding of the reduced formats (FP32 ~1e-7 per
    operation, BF16 ~4e-3 per stored coarse entry)."""
    name, hsys, o = case
    s = amg.AMGSolver(hsys, smoother="GS-1-1", precision=precision)
    h = _oracle_hierarchy(o)
    prec = oamg.preconditioner(h, oamg.Smoother.parse("GS-1-1"))
    r = np.random.default_rng(15).standard_normal(hsys.dofs)
    z = torch.zeros(hsys.dofs, dtype=torch.float64, device=DEV)
    s.precondition(dev(r), z)
    ref = prec(r).ravel()
    assert np.linalg.norm(host(z) - ref) / np.linalg.norm(ref) < tol_v, (name, precision)


@pytest.mark.parametrize("precision,kry", [("MIXED", "FCG"), ("FP32", "FCG"), ("MIXED", "PCG")])
def test_reduced_precision_solve(case, precision, kry):
    """The FP64 outer loop reaches the tolerance on the true FP64 residual;
    the solution matches the oracle's FP64 solution."""
    name, hsys, o = case
    tol = 1e-10
    s = amg.AMGSolver(hsys, smoother="GS-1-1", krylov=kry, precision=precision)
    b = dev(hsys.rhs)
    x = torch.zeros_like(b)
    res = s.solve(b, x, tol=tol, maxit=500)
    assert res.converged and res.relres <= tol * 1.01, res
    h = _oracle_hierarchy(o)
    prec = oamg.preconditioner(h, oamg.Smoother.parse("GS-1-1"))
    ref = krylov.pcg(lambda v: o.A.matvec(v).ravel(), lambda r: prec(r).ravel(), o.b.ravel(), tol=1e-13)
    err = np.linalg.norm(host(x) - ref.x) / np.linalg.norm(ref.x)
    assert err < 1e-7, (name, precision, err)
