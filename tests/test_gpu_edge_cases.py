"""Edge cases through the C ABI: a zero right-hand side, a nonzero initial
guess, one-cube meshes whose hierarchy is a single (coarsest, directly
solved) level, and malformed systems that the host-side checks reject before
anything reaches the device."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1503_01287_amd as amg  # noqa: E402
from oracle import workloads  # noqa: E402

DEV = torch.device("cuda:0")

SOLVERS = {
    "laplace3-PCG": (lambda: amg.problems.laplace(3), dict(smoother="GS-1-1", krylov="PCG")),
    "elasticity3-FCG-MIXED": (lambda: amg.problems.elasticity(3),
                              dict(smoother="GS-1-1", krylov="FCG", precision="MIXED")),
    "mixed3-FGMRES": (lambda: amg.problems.mixed_elasticity(3, nu=0.3), dict(smoother="sGS-1-1", krylov="FGMRES")),
    "cavity3-BS-stand-alone": (lambda: amg.problems.stokes_cavity(3, 1.0), dict(smoother="BS-1-1", krylov="NONE")),
}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def dense_operator(o):
    """The oracle's assembled operator as a dense matrix (SPD or saddle)."""
    A = o.A.scipy().toarray()
    if getattr(o, "B", None) is None:
        return A
    B = o.B.scipy().toarray()
    C = o.C.scipy().toarray() if o.C is not None else np.zeros((B.shape[0], B.shape[0]))
    return np.block([[A, B.T], [B, -C]])


@pytest.mark.parametrize("name", list(SOLVERS))
def test_zero_rhs_gives_zero_without_iterations(name):
    hs = SOLVERS[name][0]()
    s = amg.AMGSolver(hs, **SOLVERS[name][1])
    b = torch.zeros(hs.dofs, dtype=torch.float64, device=DEV)
    x = torch.zeros_like(b)
    res = s.solve(b, x, tol=1e-8, maxit=50)
    s.close()
    assert res.status == 0 and res.iters == 0, res
    assert not host(x).any()


def test_zero_rhs_batch():
    systems = [amg.problems.stokes_cavity(3, 1.0), amg.problems.mixed_elasticity(2, nu=0.3)]
    bsol = amg.BatchedSolver(systems, smoother="BS-1-1")
    b = torch.zeros(bsol.n, dtype=torch.float64, device=DEV)
    x = torch.zeros_like(b)
    res = bsol.solve(b, x, tol=1e-8, maxit=50)
    bsol.close()
    assert all(r.status == 0 and r.iters == 0 for r in res), res
    assert not host(x).any()


@pytest.mark.parametrize("name", ["laplace3-PCG", "elasticity3-FCG-MIXED", "mixed3-FGMRES"])
def test_nonzero_initial_guess(name):
    """x is the initial guess on entry: from a random x0 the solve reaches the
    solution it reaches from zero, and the reported residual is relative to
    the initial one."""
    hs = SOLVERS[name][0]()
    s = amg.AMGSolver(hs, **SOLVERS[name][1])
    b = dev(hs.rhs)
    x = torch.zeros_like(b)
    r0 = s.solve(b, x, tol=1e-12, maxit=500)
    ref = host(x)
    x = dev(np.random.default_rng(3).standard_normal(hs.dofs))
    r1 = s.solve(b, x, tol=1e-12, maxit=500)
    s.close()
    assert r0.converged and r1.converged, (r0, r1)
    got = host(x)
    if hs.pressure_kernel:
        nv = 3 * hs.nodes
        got[nv:] -= got[nv:].mean()
        ref[nv:] -= ref[nv:].mean()
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-9


@pytest.mark.parametrize("which", ["laplace", "elasticity", "mixed"])
def test_one_cube_mesh_is_a_single_direct_level(which):
    """27 velocity nodes: below the coarsening threshold, so the hierarchy is
    one level solved by its explicit inverse, and the Krylov method converges
    in one iteration to the oracle's dense solution."""
    if which == "laplace":
        hs, o, kw = amg.problems.laplace(1), workloads.laplace(1), dict(smoother="GS-1-1", krylov="PCG")
        rhs = o.b.ravel()
    elif which == "elasticity":
        hs, o, kw = amg.problems.elasticity(1), workloads.elasticity(1), dict(smoother="GS-1-1", krylov="PCG")
        rhs = o.b.ravel()
    else:
        hs, o = amg.problems.mixed_elasticity(1, nu=0.3), workloads.mixed_elasticity(1, nu=0.3)
        kw = dict(smoother="sGS-1-1", krylov="FGMRES")
        rhs = np.concatenate([o.f.ravel(), o.g])
    s = amg.AMGSolver(hs, **kw)
    assert s.num_levels == 1 and s.level_info(0).is_coarsest == 1
    b = dev(hs.rhs)
    x = torch.zeros_like(b)
    res = s.solve(b, x, tol=1e-10, maxit=10)
    s.close()
    assert res.converged and res.iters == 1, res
    want = np.linalg.solve(dense_operator(o), rhs)
    assert np.linalg.norm(host(x) - want) / np.linalg.norm(want) < 1e-10


@pytest.mark.parametrize("case", ["no nodes", "column out of range", "unsorted columns", "missing diagonal",
                                  "rowptr start", "bad block size"])
def test_malformed_systems_are_rejected(case):
    hs = amg.problems.laplace(2)
    col = hs.A_col.copy()
    rp = hs.A_rowptr.copy()
    if case == "no nodes":
        bad = dataclasses.replace(hs, n_lin=0, n_quad=0)
    elif case == "column out of range":
        col[rp[3]] = hs.nodes
        bad = dataclasses.replace(hs, A_col=col)
    elif case == "unsorted columns":
        a, b = rp[4], rp[4] + 1
        col[a], col[b] = col[b], col[a]
        bad = dataclasses.replace(hs, A_col=col)
    elif case == "missing diagonal":
        row = 5
        k = rp[row] + int(np.nonzero(col[rp[row]:rp[row + 1]] == row)[0][0])
        # replace the diagonal by a column that keeps the row sorted and unique
        left = col[k - 1] if k > rp[row] else -1
        right = col[k + 1] if k + 1 < rp[row + 1] else hs.nodes
        cand = [c for c in range(left + 1, right) if c != row]
        if not cand:
            pytest.skip("no free column next to the diagonal")
        col[k] = cand[0]
        bad = dataclasses.replace(hs, A_col=col)
    elif case == "rowptr start":
        bad = dataclasses.replace(hs, A_rowptr=rp + 1)
    else:
        bad = dataclasses.replace(hs, bs=2)
    with pytest.raises(amg.AmgError):
        amg.AMGSolver(bad, smoother="GS-1-1")


def test_malformed_system_in_a_batch_is_rejected():
    """The systems of a batch are set up concurrently; the error reported is
    the one of the lowest-numbered failing system, as in a sequential setup."""
    good = [amg.problems.laplace(3, i=k) for k in range(6)]
    rp, col = good[1].A_rowptr, good[1].A_col.copy()
    col[rp[3]] = good[1].nodes  # column out of range in system 1
    out_of_range = dataclasses.replace(good[1], A_col=col)
    rp, col = good[4].A_rowptr, good[4].A_col.copy()
    for row in range(good[4].nodes):  # a row whose diagonal can move to a free column
        k = rp[row] + int(np.nonzero(col[rp[row]:rp[row + 1]] == row)[0][0])
        left = col[k - 1] if k > rp[row] else -1
        right = col[k + 1] if k + 1 < rp[row + 1] else good[4].nodes
        cand = [c for c in range(left + 1, right) if c != row]
        if cand:
            break
    assert cand
    col[k] = cand[0]  # the row stays sorted and unique, without its diagonal
    no_diag = dataclasses.replace(good[4], A_col=col)
    for systems, want in (([good[0], out_of_range, good[2], good[3], no_diag, good[5]], "column index out of range"),
                          ([good[0], good[2], good[3], no_diag, good[5]], "missing diagonal")):
        with pytest.raises(amg.AmgError, match=want):
            amg.BatchedSolver(systems, smoother="GS-1-1")
    # the well-formed ones still set up and solve afterwards
    bs = amg.BatchedSolver(good, smoother="GS-1-1")
    x = torch.zeros(bs.n, dtype=torch.float64, device=DEV)
    res = bs.solve(dev(np.concatenate([s.rhs for s in good])), x, tol=1e-8)
    assert all(r.converged for r in res)
    bs.close()
