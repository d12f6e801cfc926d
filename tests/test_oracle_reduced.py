"""Pins of the oracle's reduced-precision reading of the cycle (addition X1,
reading R18): the BF16 rounding against its definition, the rounded
operators against their error bounds, and the cycle against the FP64
cycle when nothing is rounded."""
import math

import numpy as np
import pytest

from oracle import amg, reduced, workloads


def _bf16_definition(v):
    """Nearest value with 8 significant bits, ties to an even 8-bit
    significand (Python's round() on an exact float is half-to-even)."""
    if v == 0.0 or not math.isfinite(v):
        return v
    m, e = math.frexp(v)                 # v = m 2^e, 0.5 <= |m| < 1
    return math.ldexp(round(m * 256.0), e - 8)


def test_bf16_rounding_is_nearest_even():
    rng = np.random.default_rng(21)
    vals = list(rng.standard_normal(2000) * 10.0 ** rng.integers(-20, 20, 2000))
    # exact ties: 8 significant bits plus a half unit, both parities
    for sig in (129, 130, 255, 200, 201):
        for e in (-30, 0, 7):
            vals.append(math.ldexp(sig + 0.5, e))
            vals.append(-math.ldexp(sig + 0.5, e))
    vals += [0.0, -0.0, 1.0, -1.0, 1.0 + 2.0 ** -9, 1.0 + 2.0 ** -8 + 2.0 ** -9]
    v = np.array(vals)
    got = reduced.bf16_round(v)
    want = np.array([_bf16_definition(x) for x in vals])
    assert np.array_equal(got, want)
    # and the result fits in BF16: its FP32 image has 16 zero low bits
    f = got.astype(np.float32)
    assert np.all((f.view(np.uint32) & 0xFFFF) == 0) and np.array_equal(f.astype(np.float64), got)


def test_rounded_operator_bounds_and_unit_diagonal():
    s = workloads.elasticity(3)
    h = amg.setup(s.A, s.nlin, s.nquad, coarse_max=30)
    A = h.levels[1].A
    Ah = reduced.round_operator(A, "bf16")
    sc = reduced.row_scales(A)
    # every stored value within half a BF16 unit of the scaled value
    err = np.abs(Ah.vals - A.vals) / sc[A.row_of()][:, :, None]
    assert err.max() <= 2.0 ** -8 * (1 + 1e-7)
    # the scaled diagonal is exactly +-1: the stored diagonal is +-fp32(|a_ii|)
    dA, dH = np.einsum("nii->ni", A.diag_blocks()), np.einsum("nii->ni", Ah.diag_blocks())
    assert np.array_equal(np.abs(dH), sc) and np.array_equal(np.sign(dH), np.sign(dA))
    A32 = reduced.round_operator(A, "fp32")
    assert np.abs(A32.vals - A.vals).max() <= 2.0 ** -24 * np.abs(A.vals).max()


def test_zero_diagonal_row_scale_falls_back_to_row_maximum():
    s = workloads.elasticity(2)
    A = s.A
    vals = A.vals.copy()
    rows = A.row_of()
    on = np.nonzero(rows == A.indices)[0]
    vals[on[3], 1, 1] = 0.0
    Z = type(A)(A.indptr, A.indices, vals, A.ncols)
    sc = reduced.row_scales(Z)
    sel = rows == 3
    assert sc[3, 1] == np.float32(np.abs(vals[sel, 1, :]).max())


@pytest.mark.parametrize("name", ["GS-1-1", "JA-1-1-0.5", "GS-2-2"])
def test_unrounded_reduced_cycle_equals_fp64_cycle(name):
    """With no rounding the correction-form sweeps are the sweeps of the FP64
    cycle and the explicit coarse-end map is the cycle it replaces."""
    s = workloads.elasticity(3)
    h = amg.setup(s.A, s.nlin, s.nquad, coarse_max=30)
    sm = amg.Smoother.parse(name)
    r = np.random.default_rng(22).standard_normal(3 * s.A.nrows)
    want = amg.preconditioner(h, sm)(r).ravel()
    for tail in (None, 1, 2):
        got = reduced.reduced_preconditioner(h, sm, "FP64", tail_level=tail)(r).ravel()
        assert np.abs(got - want).max() < 1e-12 * np.abs(want).max(), tail
    w2 = amg.preconditioner(h, sm, nu=2)(r).ravel()
    g2 = reduced.reduced_preconditioner(h, sm, "FP64", tail_level=1, nu=2)(r).ravel()
    assert np.abs(g2 - w2).max() < 1e-12 * np.abs(w2).max()


def test_mixed_cycle_close_to_fp64_cycle():
    """The MIXED cycle differs from the FP64 one by about BF16's precision
    (a few 1e-3), the FP32 one by about FP32's."""
    s = workloads.elasticity(4)
    h = amg.setup(s.A, s.nlin, s.nquad)
    sm = amg.Smoother.parse("GS-1-1")
    r = np.random.default_rng(23).standard_normal(3 * s.A.nrows)
    ref = amg.preconditioner(h, sm)(r).ravel()
    mixed = reduced.reduced_preconditioner(h, sm, "MIXED")(r).ravel()
    f32 = reduced.reduced_preconditioner(h, sm, "FP32")(r).ravel()
    dm = np.linalg.norm(mixed - ref) / np.linalg.norm(ref)
    d32 = np.linalg.norm(f32 - ref) / np.linalg.norm(ref)
    assert 1e-5 < dm < 2e-2 and d32 < 1e-5, (dm, d32)
