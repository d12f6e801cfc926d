"""amg_setup / amg_setup_batched with the system in device memory
(memory = AMG_MEM_DEVICE): the same hierarchy and, with the launch shapes
fixed (no tuner), the same solutions bit for bit as from host arrays; host
pointers under AMG_MEM_DEVICE and unknown memory kinds are rejected."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1503_01287_amd as amg  # noqa: E402
from paper_1503_01287_amd import _lib as C  # noqa: E402
from paper_1503_01287_amd import solver as S  # noqa: E402

DEV = torch.device("cuda:0")


def _levels(s):
    return [(i.n_lin, i.n_quad, i.n_pres, i.nnz_A, i.nnz_B, i.nnz_C)
            for i in (s.level_info(l) for l in range(s.num_levels))]


def _solve(s, hsys, tol=1e-10):
    b = torch.from_numpy(hsys.rhs).to(DEV)
    x = torch.zeros_like(b)
    r = s.solve(b, x, tol=tol, maxit=300)
    torch.cuda.synchronize()
    return r, x.cpu().numpy()


@pytest.mark.parametrize("case", ["elasticity", "laplace"])
@pytest.mark.parametrize("precision,krylov", [("FP64", "PCG"), ("MIXED", "FCG")])
def test_spd_device_system_matches_host(case, precision, krylov):
    hsys = amg.problems.elasticity(4) if case == "elasticity" else amg.problems.laplace(5)
    kw = dict(smoother="GS-1-1", krylov=krylov, precision=precision, autotune=False)
    a = amg.AMGSolver(hsys, **kw)
    d = amg.AMGSolver(hsys, device_system=True, **kw)
    assert _levels(a) == _levels(d)
    ra, xa = _solve(a, hsys)
    rd, xd = _solve(d, hsys)
    assert ra.converged and rd.converged and ra.iters == rd.iters
    assert np.array_equal(xa, xd)
    a.close()
    d.close()


def test_saddle_device_system_matches_host():
    hsys = amg.problems.stokes_cavity(3, 1.0)
    kw = dict(smoother="BS-1-1", krylov="FGMRES", autotune=False)
    a = amg.AMGSolver(hsys, **kw)
    d = amg.AMGSolver(hsys, device_system=True, **kw)
    assert _levels(a) == _levels(d)
    ra, xa = _solve(a, hsys)
    rd, xd = _solve(d, hsys)
    assert ra.converged and ra.iters == rd.iters and np.array_equal(xa, xd)
    a.close()
    d.close()


def test_batched_device_systems_match_host():
    systems = [amg.problems.stokes_cavity(n, sp) for n, sp in ((3, 1.0), (4, 0.7))]
    a = amg.BatchedSolver(systems, autotune=False)
    d = amg.BatchedSolver(systems, autotune=False, device_system=True)
    b = torch.from_numpy(np.concatenate([s.rhs for s in systems])).to(DEV)
    xa, xd = torch.zeros_like(b), torch.zeros_like(b)
    ra = a.solve(b, xa, tol=1e-10)
    rd = d.solve(b, xd, tol=1e-10)
    torch.cuda.synchronize()
    assert [r.iters for r in ra] == [r.iters for r in rd]
    assert all(r.converged for r in ra)
    assert torch.equal(xa, xd)
    a.close()
    d.close()


def test_rejected_memory_arguments():
    hsys = amg.problems.laplace(3)
    p = C.default_params()
    h = ctypes.c_void_p()
    stream = S._stream_handle(None)
    keep = []
    s = S._marshal(hsys, keep)          # host arrays ...
    s.memory = C.AMG_MEM_DEVICE          # ... declared as device memory
    assert C.lib().amg_setup(ctypes.byref(s), ctypes.byref(p), stream, ctypes.byref(h)) == C.AMG_EINVAL
    assert not h.value
    s.memory = 7
    assert C.lib().amg_setup(ctypes.byref(s), ctypes.byref(p), stream, ctypes.byref(h)) == C.AMG_EINVAL
    arr = (C.AmgSystem * 1)()
    arr[0] = S._marshal(amg.problems.stokes_cavity(3, 1.0), keep)
    arr[0].memory = C.AMG_MEM_DEVICE
    pb = C.default_params()
    pb.smoother, pb.krylov = C.SMOOTH["BS"], C.KRYLOV["FGMRES"]
    assert C.lib().amg_setup_batched(1, arr, ctypes.byref(pb), stream, ctypes.byref(h)) == C.AMG_EINVAL
