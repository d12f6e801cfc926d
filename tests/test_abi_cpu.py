"""CPU checks of the boundary: the library loads and exports every symbol the
header declares; the harness's problem generator agrees with the oracle's
assembly; host-side argument checks of the binding."""
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1503_01287_amd as amg
from paper_1503_01287_amd import _lib
from oracle import fem, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            text = open(os.path.join(ROOT, "include", f)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(amg_\w+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    L = amg.lib()
    decl = declared_functions()
    assert decl, "no declarations found"
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (amg_\w+)", out))
    assert decl <= exported, decl - exported
    for name in decl:
        assert hasattr(L, name)
    assert set(_lib.SIGNATURES) == decl


def test_status_strings_and_defaults():
    assert _lib.status_string(0) == "converged"
    p = _lib.default_params()
    assert p.pre == 1 and p.post == 1 and abs(p.omega - 0.5) < 1e-15
    assert abs(p.sgs_omega - 0.125) < 1e-15 and p.coarse_max == 300 and p.separate == 1
    for name, parsed in [("JA-2-2-0.5", dict(smoother="JA", pre=2, post=2, omega=0.5)),
                         ("GS-1-1", dict(smoother="GS", pre=1, post=1)),
                         ("sGS-1-1", dict(smoother="SGS", pre=1, post=1)),
                         ("Braess-Sarazin-2-2", dict(smoother="BS", pre=2, post=2))]:
        assert amg.parse_smoother(name) == parsed


def _oracle_blocks(A):
    return A.vals


@pytest.mark.parametrize("n", [2, 5])
def test_harness_matches_oracle_assembly(n):
    """Quadrature assembly (harness) vs closed-form assembly (oracle)."""
    h = amg.problems.laplace(n)
    o = workloads.laplace(n)
    assert np.array_equal(h.A_rowptr, o.A.indptr) and np.array_equal(h.A_col, o.A.indices)
    v = np.zeros((h.A_col.shape[0], 3, 3))
    for c in range(3):
        v[:, c, c] = h.A_val
    assert np.abs(v - o.A.vals).max() <= 1e-14 * np.abs(o.A.vals).max()
    assert np.abs(h.rhs - o.b.ravel()).max() <= 1e-14 * max(1.0, np.abs(o.b).max())
    he = amg.problems.elasticity(n)
    oe = workloads.elasticity(n)
    assert np.array_equal(he.A_col, oe.A.indices)
    assert np.abs(he.A_val.reshape(-1, 3, 3) - oe.A.vals).max() <= 1e-14 * np.abs(oe.A.vals).max()
    assert np.abs(he.rhs - oe.b.ravel()).max() <= 1e-14 * np.abs(oe.b).max()


def test_laplace_rhs_many_matches_assembly():
    """The right-hand sides of several Dirichlet data sets from one operator
    equal those of separate assemblies, and data set 0 equals the oracle's."""
    import synth
    n = 4
    h = amg.problems.laplace(n, workload=synth.LAPLACE_LARGE, i=0)
    many = amg.problems.laplace_rhs_many(h, synth.LAPLACE_LARGE, [0, 1, 2])
    o = workloads.laplace(n, workload=synth.LAPLACE_LARGE, i=0)
    scale = max(1.0, np.abs(o.b).max())
    assert np.abs(many[0] - o.b.ravel()).max() <= 1e-13 * scale
    for i in (1, 2):
        ref = amg.problems.laplace(n, workload=synth.LAPLACE_LARGE, i=i).rhs
        assert np.abs(many[i] - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
        assert np.abs(many[i] - many[0]).max() > 1e-3 * scale   # distinct data sets


def test_harness_paper_cube_matches_oracle():
    h = amg.problems.paper_cube(3, "laplace")
    o = fem.paper_spd(3, "laplace")
    assert np.abs(h.rhs - o.b.ravel()).max() < 1e-14


def test_harness_paper_mixed_matches_oracle():
    """Section 4.4's mixed system: quadrature assembly (harness) vs closed
    form (oracle), blocks and right-hand side."""
    h = amg.problems.paper_cube(3, "mixed")
    o = fem.paper_mixed(3)
    assert h.n_pres == o.B.nrows and h.dofs == 3 * o.A.nrows + o.B.nrows
    assert np.array_equal(h.A_col, o.A.indices) and np.array_equal(h.B_col, o.B.indices)
    assert np.abs(h.A_val.reshape(-1, 3, 3) - o.A.vals).max() <= 1e-14 * np.abs(o.A.vals).max()
    assert np.abs(h.B_val.reshape(-1, 1, 3) - o.B.vals.reshape(-1, 1, 3)).max() <= 1e-14 * np.abs(o.B.vals).max()
    assert np.abs(h.C_val - o.C.vals.ravel()).max() <= 1e-14 * np.abs(o.C.vals).max()
    rhs = np.concatenate([o.f.ravel(), o.g])
    assert np.abs(h.rhs - rhs).max() <= 1e-14 * np.abs(rhs).max()


def test_sizes_match_paper_table():
    h = amg.problems.elasticity(8)
    assert h.dofs == 14739
