"""The reduced-precision cycles (FP32 finest / BF16 with row scales below,
and all-FP32) against the oracle's reduced-precision reading of the cycle
(reading R18: the same rounded operators, the FP64 cycle's diagonal block
inverses, FP64 arithmetic), so that only the rounding of the FP32 vectors and
accumulations separates them: bound 1e-5 of the largest entry. Also every
launch shape of the row kernels (lanes per row, two entries per trip,
per-XCD placement), forced through the C ABI, against the oracle: FP64 cycle
to 1e-12, reduced cycles to 1e-5.
"""
import itertools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1503_01287_amd as amg  # noqa: E402
from oracle import amg as oamg, reduced, workloads  # noqa: E402

DEV = torch.device("cuda:0")
RP_TOL = 1e-5     # reduced-precision cycle vs its FP64 reading (FP32 vectors and sums)
FP64_TOL = 1e-12


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


CASES = {
    "laplace6": (lambda: amg.problems.laplace(6), lambda: workloads.laplace(6)),
    "elast4": (lambda: amg.problems.elasticity(4), lambda: workloads.elasticity(4)),
    "elast7": (lambda: amg.problems.elasticity(7), lambda: workloads.elasticity(7)),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    hs, os_ = CASES[request.param]
    o = os_()
    return request.param, hs(), o, oamg.setup(o.A, o.nlin, o.nquad)


def _coarse_map_level(s):
    for l in range(s.num_levels):
        if s.level_info(l).coarse_map:
            return l
    return None


def _gpu_cycle(s, r):
    z = torch.zeros(r.shape[0], dtype=torch.float64, device=DEV)
    s.precondition(dev(r), z)
    return host(z)


@pytest.mark.parametrize("precision", ["MIXED", "FP32"])
@pytest.mark.parametrize("smoother", ["GS-1-1", "JA-1-1-0.5", "GS-2-2"])
@pytest.mark.parametrize("fuse", [False, True])
def test_reduced_cycle_matches_oracle_reading(case, precision, smoother, fuse):
    name, hsys, o, h = case
    s = amg.AMGSolver(hsys, smoother=smoother, krylov="FCG", precision=precision, fuse_coarse=fuse)
    d = _coarse_map_level(s)
    assert (d is not None) == (fuse and s.num_levels > 2), (name, d)
    prec = reduced.reduced_preconditioner(h, oamg.Smoother.parse(smoother), precision, tail_level=d)
    r = np.random.default_rng(31).standard_normal(hsys.dofs)
    got = _gpu_cycle(s, r)
    want = prec(r).ravel()
    assert relmax(got, want) < RP_TOL, (name, precision, smoother, fuse, relmax(got, want))
    # the reading is sharper than the FP64 cycle: BF16 moves the cycle by far more
    if precision == "MIXED":
        fp64 = oamg.preconditioner(h, oamg.Smoother.parse(smoother))(r).ravel()
        assert relmax(want, fp64) > 20 * relmax(got, want)
    s.close()


@pytest.mark.parametrize("cycles,nu", [(2, 1), (1, 2)])
def test_reduced_two_cycles_and_w_cycle(case, cycles, nu):
    name, hsys, o, h = case
    s = amg.AMGSolver(hsys, smoother="GS-1-1", krylov="FCG", precision="MIXED", cycles=cycles, nu=nu)
    d = _coarse_map_level(s)
    prec = reduced.reduced_preconditioner(h, oamg.Smoother.parse("GS-1-1"), "MIXED", tail_level=d,
                                          cycles=cycles, nu=nu)
    r = np.random.default_rng(32).standard_normal(hsys.dofs)
    assert relmax(_gpu_cycle(s, r), prec(r).ravel()) < RP_TOL, name
    s.close()


SHAPES = list(itertools.product([4, 8, 16, 32, 64], [1, 2, 4]))


@pytest.mark.parametrize("precision", ["FP64", "MIXED"])
def test_every_launch_shape_matches_oracle(case, precision):
    """Every lanes / loop-form / placement variant of the natural-order and
    colour-sweep kernels, forced on every level, gives the oracle's cycle
    (FP64: 1e-12; reduced precision: its reading to 1e-5) and the oracle's
    operator on the finest level."""
    name, hsys, o, h = case
    sm = oamg.Smoother.parse("GS-1-1")
    s = amg.AMGSolver(hsys, smoother="GS-1-1", krylov="FCG", precision=precision, autotune=False)
    nat, swp = ("natural", "sweep") if precision == "FP64" else ("natural_rp", "sweep_rp")
    r = np.random.default_rng(33).standard_normal(hsys.dofs)
    if precision == "FP64":
        want = oamg.preconditioner(h, sm)(r).ravel()
        tol = FP64_TOL
    else:
        want = reduced.reduced_preconditioner(h, sm, "MIXED", tail_level=_coarse_map_level(s))(r).ravel()
        tol = RP_TOL
    Ax = o.A.matvec(r).ravel()
    levels = [l for l in range(s.num_levels) if not s.level_info(l).is_coarsest]
    for (lanes, trip), xcd in itertools.product(SHAPES, [False, True]):
        for l in levels:
            s.set_launch_shape(l, nat, lanes, trip)
            s.set_launch_shape(l, swp, lanes, trip, xcd)
            if precision != "FP64":
                s.set_launch_shape(l, "natural", lanes, trip)
        got = _gpu_cycle(s, r)
        assert relmax(got, want) < tol, (name, precision, lanes, trip, xcd, relmax(got, want))
        y = torch.zeros(hsys.dofs, dtype=torch.float64, device=DEV)
        s.apply(0, dev(r), y)
        assert relmax(host(y), Ax) < 1e-14, (name, lanes, trip)
    s.close()


def test_launch_shape_rejects_bad_arguments():
    hsys = amg.problems.elasticity(3)
    s = amg.AMGSolver(hsys, smoother="GS-1-1")
    for args in [(0, "natural", 12), (99, "natural", 16), (0, "natural_rp", 16)]:
        with pytest.raises(amg.AmgError):
            s.set_launch_shape(*args)
    with pytest.raises(amg.AmgError):
        s.set_launch_shape(0, "natural", 16, 1, True)   # xcd is for colour sweeps
    for trip in (0, 3, 8):
        with pytest.raises(amg.AmgError):
            s.set_launch_shape(0, "sweep", 16, trip)
    s.close()


@pytest.mark.parametrize("precision", ["FP64", "MIXED"])
def test_entries_per_trip_do_not_change_the_bits(case, precision):
    """A lane adds its entries in the same order for 1, 2 or 4 entries per
    trip, so at fixed lanes the cycle is the same bit for bit."""
    name, hsys, o, h = case
    s = amg.AMGSolver(hsys, smoother="GS-1-1", krylov="FCG", precision=precision, autotune=False)
    nat, swp = ("natural", "sweep") if precision == "FP64" else ("natural_rp", "sweep_rp")
    r = np.random.default_rng(34).standard_normal(hsys.dofs)
    levels = [l for l in range(s.num_levels) if not s.level_info(l).is_coarsest]
    for lanes in (8, 32):
        outs = []
        for trip in (1, 2, 4):
            for l in levels:
                s.set_launch_shape(l, nat, lanes, trip)
                s.set_launch_shape(l, swp, lanes, trip)
            outs.append(_gpu_cycle(s, r))
        assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2]), (name, precision, lanes)
    s.close()
