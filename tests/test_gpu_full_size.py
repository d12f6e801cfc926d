"""The four benchmark workloads at their full sizes, in the solver
configurations the benchmark times, checked through the C ABI:

* against the oracle wherever it finishes in about a minute: the whole
  32^3 elasticity hierarchy element by element (sizes, prolongations and
  colours bit-exact, Galerkin operators to 1e-13) and one FP64 cycle of the
  elasticity and mixed elasticity workloads and of the 64-cavity batch (the
  merged cycle restricted to sampled cavities, each against the oracle's
  cycle of that cavity alone);
* through properties that hold at any size: the reduced-precision cycle
  within the bound of its arithmetic of the oracle's FP64 cycle, and each
  timed solve reaching 1e-8 in its true FP64 residual (recomputed on the
  host from the assembled matrices) and the FP64 solution to 1e-7.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import scipy.sparse as sps  # noqa: E402

import paper_1503_01287_amd as amg  # noqa: E402
import synth  # noqa: E402
from oracle import amg as oamg, krylov, reduced, workloads  # noqa: E402

DEV = torch.device("cuda:0")
TOL = 1e-8
# relative error of a solution against the FP64 solve to 1e-12
ERR = 1e-7
# one reduced-precision cycle against the FP64 cycle (2-norm): FP32 through
# the levels' smoothing and transfers, BF16 on the coarse velocity blocks
CYCLE_TOL = {"FP32": 2e-4, "MIXED": 5e-2}
# assembly plus the oracle's setup at these sizes takes about a minute
SLOW = pytest.mark.timeout(900)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def rel2(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def centre(v, s):
    """Pressure of a system whose pressure is fixed up to a constant, taken with zero mean."""
    v = v.copy()
    if s.pressure_kernel:
        v[3 * s.nodes:] -= v[3 * s.nodes:].mean()
    return v


def oracle_mv(o):
    """The oracle's operator (SPD, or [[A, B^T], [B, -C]])."""
    A, B = o.A, getattr(o, "B", None)
    nv = 3 * A.nrows
    if B is None:
        return lambda z: A.matvec(z.reshape(-1, 3)).ravel()
    Bt = B.transpose()

    def mv(z):
        u, p = z[:nv].reshape(-1, 3), z[nv:]
        top = A.matvec(u).ravel() + Bt.matvec(p.reshape(-1, 1)).ravel()
        bot = B.matvec(u)[:, 0]
        if o.C is not None:
            bot = bot - o.C.matvec(p.reshape(-1, 1))[:, 0]
        return np.concatenate([top, bot])
    return mv


def harness_mv(s):
    """The operator of a host system from its own arrays (scipy), for the
    48^3 Laplacian and the cavities of the batch, whose oracle assembly
    would take minutes."""
    N = s.nodes
    if s.bs == 1:
        A = sps.kron(sps.csr_matrix((s.A_val.ravel(), s.A_col, s.A_rowptr), shape=(N, N)), sps.eye(3),
                     format="csr")
    else:
        A = sps.bsr_matrix((s.A_val.reshape(-1, 3, 3), s.A_col, s.A_rowptr), shape=(3 * N, 3 * N)).tocsr()
    if not s.n_pres:
        return lambda z: A @ z
    B = sps.bsr_matrix((s.B_val.reshape(-1, 1, 3), s.B_col, s.B_rowptr), shape=(s.n_pres, 3 * N)).tocsr()
    C = None if s.C_val is None else sps.csr_matrix((s.C_val.ravel(), s.C_col, s.C_rowptr),
                                                   shape=(s.n_pres, s.n_pres))
    K = sps.bmat([[A, B.T], [B, None if C is None else -C]], format="csr")
    return lambda z: K @ z


def true_relres(mv, b, x):
    return np.linalg.norm(b - mv(x)) / np.linalg.norm(b)


def fp64_solution(hs, smoother, kry, b):
    ref = amg.AMGSolver(hs, smoother=smoother, krylov=kry)
    x = torch.zeros_like(b)
    r = ref.solve(b, x, tol=1e-12, maxit=1000)
    ref.close()
    assert r.converged, r
    return host(x)


# ---------------------------------------------------------------- elasticity 32^3
@pytest.fixture(scope="module")
def elast():
    hs = amg.problems.elasticity(32)
    o = workloads.elasticity(32)
    return hs, o, oamg.setup(o.A, o.nlin, o.nquad)


@SLOW
def test_elasticity32_hierarchy_and_cycle(elast):
    """823,875 DOF: every level of the GPU hierarchy equals the oracle's, and
    one FP64 GS-1-1 cycle equals the oracle's."""
    hs, o, h = elast
    s = amg.AMGSolver(hs, smoother="GS-1-1", krylov="FCG")
    assert s.num_levels == len(h.levels)
    for l, lev in enumerate(h.levels):
        info = s.level_info(l)
        assert (info.n_lin, info.n_quad) == (lev.nlin, lev.nquad), l
        rp, col, val = s.level_matrix(l, "A")
        assert np.array_equal(rp, lev.A.indptr) and np.array_equal(col, lev.A.indices), l
        assert relmax(val.reshape(-1, 3, 3), lev.A.vals) < 1e-13, l
        if l < len(h.levels) - 1:
            prp, pcol, pval = s.level_matrix(l, "P")
            assert np.array_equal(prp, lev.P.indptr) and np.array_equal(pcol, lev.P.indices), l
            assert np.array_equal(pval[:, 0], lev.P.data), l
            assert np.array_equal(s.level_colors(l), lev.colors), l
    prec = oamg.preconditioner(h, oamg.Smoother.parse("GS-1-1"))
    r = np.random.default_rng(71).standard_normal(hs.dofs)
    z = torch.zeros(hs.dofs, dtype=torch.float64, device=DEV)
    s.precondition(dev(r), z)
    assert relmax(host(z), prec(r).ravel()) < 1e-11
    s.close()


@SLOW
def test_elasticity32_reduced_fcg(elast):
    """The benchmark's solve: FP32 finest / BF16 coarse cycle in FP64 FCG."""
    hs, o, h = elast
    s = amg.AMGSolver(hs, smoother="GS-1-1", krylov="FCG", precision="MIXED")
    prec = oamg.preconditioner(h, oamg.Smoother.parse("GS-1-1"))
    r = np.random.default_rng(72).standard_normal(hs.dofs)
    z = torch.zeros(hs.dofs, dtype=torch.float64, device=DEV)
    s.precondition(dev(r), z)
    assert rel2(host(z), prec(r).ravel()) < CYCLE_TOL["MIXED"]
    b = dev(hs.rhs)
    x = torch.zeros_like(b)
    res = s.solve(b, x, tol=TOL, maxit=300)
    s.close()
    assert res.converged and res.relres <= TOL * 1.01, res
    xs = host(x)
    assert true_relres(oracle_mv(o), o.b.ravel(), xs) <= TOL * 1.01
    assert rel2(xs, fp64_solution(hs, "GS-1-1", "PCG", b)) < ERR


@SLOW
def test_elasticity32_reduced_cycle_vs_oracle_reading(elast):
    """The FP32/BF16 cycle launch by launch (no assembled coarse end) against
    the oracle's reduced-precision reading of the same cycle at full size
    (the assembled coarse end is compared at small sizes, where the oracle
    assembles its map in seconds)."""
    hs, o, h = elast
    s = amg.AMGSolver(hs, smoother="GS-1-1", krylov="FCG", precision="MIXED", fuse_coarse=False)
    r = np.random.default_rng(76).standard_normal(hs.dofs)
    z = torch.zeros(hs.dofs, dtype=torch.float64, device=DEV)
    s.precondition(dev(r), z)
    s.close()
    want = reduced.reduced_preconditioner(h, oamg.Smoother.parse("GS-1-1"), "MIXED")(r).ravel()
    assert relmax(host(z), want) < 1e-5


@SLOW
def test_elasticity32_solutions_vs_oracle_solution(elast):
    """The method's target at full size: the timed solve (FP32/BF16 cycle in
    FP64 FCG to 1e-8) within 1e-7 of the oracle's own FP64 solution (its
    AMG-PCG to 1e-12), and the GPU's FP64 PCG solution to 1e-12 within 1e-9."""
    hs, o, h = elast
    prec = oamg.preconditioner(h, oamg.Smoother.parse("GS-1-1"))
    ref = krylov.pcg(lambda v: o.A.matvec(v).ravel(), lambda r: prec(r).ravel(), o.b.ravel(), tol=1e-12,
                     maxit=300)
    assert ref.converged and ref.relres <= 1.01e-12, ref.relres
    b = dev(hs.rhs)
    for precision, kry, tol, bound in (("MIXED", "FCG", TOL, ERR), ("FP64", "PCG", 1e-12, 1e-9)):
        s = amg.AMGSolver(hs, smoother="GS-1-1", krylov=kry, precision=precision)
        x = torch.zeros_like(b)
        res = s.solve(b, x, tol=tol, maxit=300)
        s.close()
        assert res.converged, (precision, res)
        assert rel2(host(x), ref.x) < bound, (precision, rel2(host(x), ref.x))


# ---------------------------------------------------------------- mixed elasticity 24^3
@pytest.fixture(scope="module")
def mixed():
    hs = amg.problems.mixed_elasticity(24)
    o = workloads.mixed_elasticity(24)
    return hs, o, oamg.setup(o.A, o.nlin, o.nquad, B=o.B, C=o.C, singular=o.singular)


@SLOW
def test_mixed24_cycles(mixed):
    """368,572 DOF, sGS-1-1: the FP64 cycle equals the oracle's, the
    FP32/BF16 cycle is within its bound of it."""
    hs, o, h = mixed
    prec = oamg.preconditioner(h, oamg.Smoother.parse("sGS-1-1"))
    r = np.random.default_rng(73).standard_normal(hs.dofs)
    ref = prec(r)
    for precision in ("FP64", "MIXED"):
        s = amg.AMGSolver(hs, smoother="sGS-1-1", krylov="FGMRES", precision=precision)
        z = torch.zeros(hs.dofs, dtype=torch.float64, device=DEV)
        s.precondition(dev(r), z)
        if precision == "FP64":
            assert relmax(host(z), ref) < 1e-11
        else:
            assert rel2(host(z), ref) < CYCLE_TOL["MIXED"]
        s.close()


@SLOW
def test_mixed24_reduced_fgmres(mixed):
    """The benchmark's solve: FP32/BF16 cycle in FP64 flexible GMRES."""
    hs, o, h = mixed
    s = amg.AMGSolver(hs, smoother="sGS-1-1", krylov="FGMRES", precision="MIXED")
    b = dev(hs.rhs)
    x = torch.zeros_like(b)
    res = s.solve(b, x, tol=TOL, maxit=1000)
    s.close()
    assert res.converged and res.relres <= TOL * 1.01, res
    xs = host(x)
    rhs = np.concatenate([o.f.ravel(), o.g])
    assert true_relres(oracle_mv(o), rhs, xs) <= TOL * 1.01
    assert rel2(xs, fp64_solution(hs, "sGS-1-1", "FGMRES", b)) < ERR


@SLOW
def test_mixed24_solution_vs_oracle_solution(mixed):
    """The timed solve (FP32/BF16 sGS cycle in FP64 FGMRES to 1e-8) within
    1e-7 of the oracle's own FP64 solution (its FGMRES with the FP64 sGS
    cycle to 1e-12)."""
    hs, o, h = mixed
    prec = oamg.preconditioner(h, oamg.Smoother.parse("sGS-1-1"))
    rhs = np.concatenate([o.f.ravel(), o.g])
    ref = krylov.fgmres(oracle_mv(o), prec, rhs, tol=1e-12, maxit=400, restart=200)
    assert ref.converged, ref.relres
    s = amg.AMGSolver(hs, smoother="sGS-1-1", krylov="FGMRES", precision="MIXED")
    b = dev(hs.rhs)
    x = torch.zeros_like(b)
    res = s.solve(b, x, tol=TOL, maxit=1000)
    s.close()
    assert res.converged, res
    assert rel2(host(x), ref.x) < ERR, rel2(host(x), ref.x)


# ---------------------------------------------------------------- vector Laplacian 48^3
@SLOW
def test_laplace48_learned_reduced_fcg():
    """2,738,019 DOF, the benchmark's solves: one setup with the learned
    per-level weights and the FP32/BF16 cycle in FCG, then one solve per
    Dirichlet data set, each reaching 1e-8 in its true residual (from the
    assembled matrix, on the host) and the FP64 solution to 1e-7, in no more
    iterations than the fixed-weight reduced-precision solve. (The oracle's
    own assembly of this size takes minutes; its cycle is compared at the
    other three full sizes and at small sizes.)"""
    from paper_1503_01287_amd import learned
    hs = amg.problems.laplace(48, workload=synth.LAPLACE_LARGE, i=0)
    s = amg.AMGSolver(hs, smoother="JA-1-1-0.5", krylov="FCG", precision="MIXED",
                      omega_model=learned.DampingModel.load())
    fixed = amg.AMGSolver(hs, smoother="JA-1-1-0.5", krylov="FCG", precision="MIXED")
    mv = harness_mv(hs)
    rhs = amg.problems.laplace_rhs_many(hs, synth.LAPLACE_LARGE, [0, 1])
    assert relmax(rhs[0], hs.rhs) < 1e-13
    for k, r in enumerate(rhs):
        b = dev(r)
        x = torch.zeros_like(b)
        res = s.solve(b, x, tol=TOL, maxit=300)
        assert res.converged and res.relres <= TOL * 1.01, (k, res)
        xs = host(x)
        assert true_relres(mv, r, xs) <= TOL * 1.01, k
        assert rel2(xs, fp64_solution(hs, "JA-1-1-0.5", "PCG", b)) < ERR, k
        x.zero_()
        rf = fixed.solve(b, x, tol=TOL, maxit=300)
        assert rf.converged and res.iters <= rf.iters, (k, res.iters, rf.iters)
    s.close()
    fixed.close()


# ---------------------------------------------------------------- 64 Stokes cavities
@pytest.fixture(scope="module")
def cavities():
    cfg = synth.stokes_batch()
    return cfg, [amg.problems.stokes_cavity(n, sp) for n, sp in cfg]


def _offsets(systems):
    """Start of every system in the vectors of BatchedSolver.solve."""
    return np.cumsum([0] + [s.dofs for s in systems])


@SLOW
def test_stokes_batch_sampled_cycles(cavities):
    """The merged BS-1-1 cycle of all 64 cavities (one preconditioner
    application in the merged layout: every cavity's velocity, then every
    cavity's pressure), restricted to the smallest and the largest cavity,
    equals the oracle's cycle of that cavity alone (FP64), and the FP32
    merged cycle is within its bound of it."""
    cfg, systems = cavities
    ns = [n for n, _ in cfg]
    rng = np.random.default_rng(75)
    rs = [rng.standard_normal(s.dofs) for s in systems]
    nu_all = 3 * sum(s.nodes for s in systems)
    z = {}
    for precision in ("FP64", "FP32"):
        bsol = amg.BatchedSolver(systems, smoother="BS-1-1", precision=precision)
        uo, po = bsol.offsets()
        merged = np.zeros(bsol.n)
        for s, r, u, q in zip(systems, rs, uo, po):
            merged[u:u + 3 * s.nodes] = r[:3 * s.nodes]
            merged[nu_all + q:nu_all + q + s.n_pres] = r[3 * s.nodes:]
        zd = torch.zeros(bsol.n, dtype=torch.float64, device=DEV)
        bsol.precondition(dev(merged), zd)
        zm = host(zd)
        z[precision] = [np.concatenate([zm[u:u + 3 * s.nodes], zm[nu_all + q:nu_all + q + s.n_pres]])
                        for s, u, q in zip(systems, uo, po)]
        bsol.close()
    for i in sorted({ns.index(min(ns)), ns.index(max(ns))}):
        n, sp = cfg[i]
        o = workloads.stokes(n, sp)
        h = oamg.setup(o.A, o.nlin, o.nquad, B=o.B, C=o.C, singular=o.singular)
        oamg.prepare_bs(h)
        prec = oamg.preconditioner(h, oamg.Smoother.parse("BS-1-1"))
        ref = prec(rs[i])
        assert relmax(z["FP64"][i], ref) < 1e-10, (i, n)
        assert rel2(z["FP32"][i], ref) < CYCLE_TOL["FP32"], (i, n)


@SLOW
def test_stokes_batch_fp32_fgmres(cavities):
    """The benchmark's solve: all 64 cavities as one merged hierarchy, FP32
    cycle in FP64 flexible GMRES; every cavity reaches 1e-8 in its true
    residual and its FP64 solution to 1e-7."""
    cfg, systems = cavities
    off = _offsets(systems)
    b = dev(np.concatenate([s.rhs for s in systems]))
    out = {}
    for precision, tol in (("FP32", TOL), ("FP64", 1e-12)):
        bsol = amg.BatchedSolver(systems, smoother="BS-1-1", precision=precision)
        x = torch.zeros_like(b)
        res = bsol.solve(b, x, tol=tol, maxit=1000)
        bsol.close()
        assert all(q.converged and q.relres <= tol * 1.01 for q in res), (precision, res)
        out[precision] = host(x)
    for i, s in enumerate(systems):
        sl = slice(off[i], off[i + 1])
        assert true_relres(harness_mv(s), s.rhs, out["FP32"][sl]) <= TOL * 1.01, i
        assert rel2(centre(out["FP32"][sl], s), centre(out["FP64"][sl], s)) < ERR, i
    # the smallest and the largest cavity against the oracle's own FP64
    # solution of that cavity alone (its FGMRES with the BS-1-1 cycle to 1e-12)
    ns = [n for n, _ in cfg]
    for i in sorted({ns.index(min(ns)), ns.index(max(ns))}):
        n, sp = cfg[i]
        o = workloads.stokes(n, sp)
        h = oamg.setup(o.A, o.nlin, o.nquad, B=o.B, C=o.C, singular=o.singular)
        oamg.prepare_bs(h)
        prec = oamg.preconditioner(h, oamg.Smoother.parse("BS-1-1"))
        ref = krylov.fgmres(oracle_mv(o), prec, np.concatenate([o.f.ravel(), o.g]), tol=1e-12, maxit=400,
                            restart=200)
        assert ref.converged, (i, n, ref.relres)
        sl = slice(off[i], off[i + 1])
        assert rel2(centre(out["FP32"][sl], systems[i]), centre(ref.x, systems[i])) < ERR, (i, n)
