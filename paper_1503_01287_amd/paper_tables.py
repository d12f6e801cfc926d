"""The paper's iteration tables (Section 4, meshes L1-L4 = 4^3 ... 32^3
cubes, its boundary data u = 0 on z = 0, u = (0, 0, 1) on z = 1, FP64)
rerun on the GPU. SPD (vector Laplacian, elasticity in pure displacement
form; relative residual 1e-11): stand-alone AMG and AMG-preconditioned CG,
V-cycle (nu = 1) and W-cycle (nu = 2), smoothers JA-1-1-0.5, JA-2-2-0.5,
GS-1-1, GS-2-2. Mixed elasticity (Section 4.4; relative residual 1e-9 of the
whole residual): stand-alone AMG with sGS-k-k and Braess-Sarazin-k-k, and
GMRES with one or two V-cycles of sGS-1-1, Braess-Sarazin-1-1 and
Vanka-1-1 (flexible GMRES here). Non-separating coarsening (the black-box
comparison of Section 4.2, vector Laplacian, two W-cycles per iteration).
The paper's counts are printed beside ours;
'-' marks a run that does not converge (within MAXIT).

    python -m paper_1503_01287_amd.paper_tables [--levels 1 2 3 4] [--out table.md]
"""
from __future__ import annotations

import argparse
import sys
import time

SIZES = {1: 4, 2: 8, 3: 16, 4: 32}
SMOOTHERS = ["JA-1-1-0.5", "JA-2-2-0.5", "GS-1-1", "GS-2-2"]
MAXIT = 400
X = None  # no count in the paper (the solver fails there)

# (table label, problem, Krylov method, nu) -> smoother -> counts at L1..L4
PAPER = {
    ("tab:amglapv", "laplace", "NONE", 1): {
        "JA-1-1-0.5": [129, 125, 124, 128], "JA-2-2-0.5": [65, 65, 65, 66],
        "GS-1-1": [43, 46, 47, 47], "GS-2-2": [23, 24, 24, 24]},
    ("tab:amglapw", "laplace", "NONE", 2): {
        "JA-1-1-0.5": [128, 124, 121, 123], "JA-2-2-0.5": [65, 64, 63, 64],
        "GS-1-1": [43, 46, 47, 47], "GS-2-2": [23, 24, 24, 24]},
    ("tab:amglapvpcg", "laplace", "PCG", 1): {
        "JA-1-1-0.5": [30, 30, 30, 30], "JA-2-2-0.5": [21, 22, 22, 22],
        "GS-1-1": [26, 29, 29, 30], "GS-2-2": [17, 19, 19, 19]},
    ("tab:amglapwpcg", "laplace", "PCG", 2): {
        "JA-1-1-0.5": [30, 30, 30, 29], "JA-2-2-0.5": [21, 21, 21, 21],
        "GS-1-1": [26, 29, 29, 29], "GS-2-2": [17, 18, 18, 18]},
    ("tab:amgelasv", "elastic", "NONE", 1): {
        "JA-1-1-0.5": [X, X, X, X], "JA-2-2-0.5": [X, X, X, X],
        "GS-1-1": [80, 78, 76, 75], "GS-2-2": [44, 40, 39, 39]},
    ("tab:amgelasw", "elastic", "NONE", 2): {
        "JA-1-1-0.5": [X, X, X, X], "JA-2-2-0.5": [X, X, X, X],
        "GS-1-1": [80, 78, 75, 73], "GS-2-2": [44, 40, 39, 44]},
    ("tab:amgelasvpcg", "elastic", "PCG", 1): {
        "JA-1-1-0.5": [50, 81, X, X], "JA-2-2-0.5": [32, 63, X, X],
        "GS-1-1": [40, 43, 43, 42], "GS-2-2": [28, 27, 27, 27]},
    ("tab:amgelaswpcg", "elastic", "PCG", 2): {
        "JA-1-1-0.5": [47, 80, X, X], "JA-2-2-0.5": [32, 62, X, X],
        "GS-1-1": [39, 44, 42, 41], "GS-2-2": [28, 27, 27, 26]},
}


# mixed elasticity: (table label, Krylov method, V-cycles per preconditioner, smoother, counts at L1..L4)
PAPER_MIXED = [
    ("tab:amgelasamguzawanotay", "NONE", 1, "sGS-1-1", [107, 104, 99, 93]),
    ("tab:amgelasamguzawanotay", "NONE", 1, "sGS-2-2", [54, 53, 53, 59]),
    ("tab:amgelasgmresuzawanotay", "FGMRES", 1, "sGS-1-1", [14, 18, 19, 21]),
    ("tab:amgelasgmresuzawanotay", "FGMRES", 2, "sGS-1-1", [12, 15, 15, 15]),
    ("tab:amgelasamgBS", "NONE", 1, "BS-1-1", [135, 133, 125, 117]),
    ("tab:amgelasamgBS", "NONE", 1, "BS-2-2", [71, 70, 66, 62]),
    ("tab:amgelasgmresBS", "FGMRES", 1, "BS-1-1", [27, 27, 27, 27]),
    ("tab:amgelasgmresBS", "FGMRES", 2, "BS-1-1", [18, 19, 19, 19]),
    ("tab:amgelasgmresvanka", "FGMRES", 1, "Vanka-1-1", [60, 45, 49, 69]),
    ("tab:amgelasgmresvanka", "FGMRES", 2, "Vanka-1-1", [42, 30, 32, 45]),
]


# non-separating ("black-box") coarsening, vector Laplacian, 2 W-cycles per
# iteration with one smoothing step each way (smoother read as GS-1-1);
# None = the paper's "> 200"
PAPER_NONSEP = [
    ("tab:nonsepamg", "NONE", [90, 158, None, None]),
    ("tab:nonsepamg", "PCG", [22, 25, 36, 64]),
]


def _run(systems, kind, l, dev, tol, **kw):
    import torch
    from . import problems, AMGSolver
    key = (kind, l)
    if key not in systems:
        systems[key] = problems.paper_cube(SIZES[l], kind)
    sysm = systems[key]
    s = AMGSolver(sysm, **kw)
    b = torch.from_numpy(sysm.rhs).to(dev)
    x = torch.zeros_like(b)
    t0 = time.perf_counter()
    r = s.solve(b, x, tol=tol, maxit=MAXIT)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0)
    s.close()
    return sysm, (str(r.iters) if r.converged else "-"), ms


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--levels", type=int, nargs="+", default=[1, 2, 3, 4])
    ap.add_argument("--out", default=None)
    ap.add_argument("--only", choices=["spd", "mixed", "nonsep"], default=None)
    args = ap.parse_args()
    import torch
    dev = torch.device("cuda:0")
    systems = {}
    lines = ["| table | smoother | " + " | ".join(f"L{l} (ours / paper)" for l in args.levels) + " |",
             "|---|---|" + "---|" * len(args.levels)]
    for (label, kind, kry, nu), rows in (PAPER.items() if args.only in (None, "spd") else []):
        for sm in SMOOTHERS:
            cells = []
            for l in args.levels:
                sysm, ours, ms = _run(systems, kind, l, dev, 1e-11, smoother=sm, krylov=kry, nu=nu)
                ref = rows[sm][l - 1]
                cells.append(f"{ours} / {'-' if ref is None else ref}")
                print(f"{label} {sm} L{l} ({sysm.dofs} DOF): {ours} iterations ({ms:.0f} ms), paper "
                      f"{'-' if ref is None else ref}", file=sys.stderr, flush=True)
            lines.append(f"| {label} | {sm} | " + " | ".join(cells) + " |")
    for label, kry, cyc, sm, ref in (PAPER_MIXED if args.only in (None, "mixed") else []):
        cells = []
        for l in args.levels:
            sysm, ours, ms = _run(systems, "mixed", l, dev, 1e-9, smoother=sm, krylov=kry, cycles=cyc)
            cells.append(f"{ours} / {ref[l - 1]}")
            print(f"{label} {sm} {cyc} V L{l} ({sysm.dofs} DOF): {ours} iterations ({ms:.0f} ms), paper "
                  f"{ref[l - 1]}", file=sys.stderr, flush=True)
        name = sm if kry == "NONE" else f"{sm}, {cyc} V-cycle{'s' if cyc > 1 else ''}"
        lines.append(f"| {label} | {name} | " + " | ".join(cells) + " |")
    for label, kry, ref in (PAPER_NONSEP if args.only in (None, "nonsep") else []):
        cells = []
        for l in args.levels:
            sysm, ours, ms = _run(systems, "laplace", l, dev, 1e-11, smoother="GS-1-1", krylov=kry, nu=2,
                                  cycles=2, separate=False)
            r = "> 200" if ref[l - 1] is None else ref[l - 1]
            cells.append(f"{ours} / {r}")
            print(f"{label} {kry} L{l} ({sysm.dofs} DOF): {ours} iterations ({ms:.0f} ms), paper {r}",
                  file=sys.stderr, flush=True)
        lines.append(f"| {label} | non-separating, {'AMG' if kry == 'NONE' else 'PCG'}, 2 W-cycles | "
                     + " | ".join(cells) + " |")
    text = "\n".join(lines) + "\n"
    print(text)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
