#!/usr/bin/env python3
"""Throughput of the AMG-preconditioned Krylov solve on one MI355X.

One step = one amg_solve of the workload to a relative residual of 1e-8
(every kernel of the hot path: smoothing, residuals, restriction,
prolongation, coarsest solve and the outer Krylov loop), starting from
x = 0 with the right-hand side resident in HBM. The hierarchy is built once
by amg_setup (timed separately and reported as setup_ms).

Prints ONE JSON line. `value` is DOF-solves/s of the timed steps. The
`roofline` object reports the dominant kernel's algorithmic bytes per launch
over its mean launch time (HIP events on the library's stream during the
timed steps). `cpu_baseline` times the FP64 CPU oracle on a bounded sample
of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published

WORKLOADS = {
    "elasticity-32": dict(desc="linear elasticity, pure displacement, unit cube 32^3 cubes x 6 Kuhn tets, "
                               "hierarchical P2, E=1 nu=0.3, clamped x=0, random traction x=1",
                          smoother="GS-1-1"),
    "laplace-48": dict(desc="vector Laplacian, unit cube 48^3 cubes x 6 Kuhn tets, hierarchical P2, "
                            "trigonometric Dirichlet data on x=0", smoother="JA-1-1-0.5"),
    "laplace-4": dict(desc="vector Laplacian 4^3 cubes (2187 DOF)", smoother="GS-1-1"),
}


def build_system(name: str):
    from paper_1503_01287_amd import problems
    if name == "elasticity-32":
        return problems.elasticity(32)
    if name == "laplace-48":
        import synth
        return problems.laplace(48, workload=synth.LAPLACE_LARGE, i=0)
    if name == "laplace-4":
        return problems.laplace(4)
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(name: str, iters_full: int, tol: float, budget_s: float = 20.0) -> dict:
    """Time the CPU oracle's preconditioned CG iterations on the same
    workload (its own assembly and hierarchy, untimed) for about budget_s
    seconds and scale to one full solve."""
    import numpy as np
    from oracle import amg as oamg, krylov, workloads
    import synth
    if name == "elasticity-32":
        o = workloads.elasticity(32)
        sm = "GS-1-1"
    elif name == "laplace-48":
        o = workloads.laplace(48, workload=synth.LAPLACE_LARGE, i=0)
        sm = "JA-1-1-0.5"
    else:
        o = workloads.laplace(4)
        sm = "GS-1-1"
    h = oamg.setup(o.A, o.nlin, o.nquad)
    prec = oamg.preconditioner(h, oamg.Smoother.parse(sm))
    mv = lambda v: o.A.matvec(v).ravel()
    pc = lambda r: prec(r).ravel()
    # a short first run measures the cost of one iteration, then a run sized to the budget
    t0 = time.perf_counter()
    krylov.pcg(mv, pc, o.b.ravel(), tol=0.0, maxit=1)
    t1 = max(time.perf_counter() - t0, 1e-3)
    k = int(max(1, min(iters_full, budget_s / t1)))
    t0 = time.perf_counter()
    krylov.pcg(mv, pc, o.b.ravel(), tol=0.0, maxit=k)
    per_iter = (time.perf_counter() - t0) / (k + 1)   # k iterations + the initial preconditioning
    solve_s = per_iter * (iters_full + 1)
    dofs = 3 * o.A.nrows
    return {"value": dofs / solve_s, "unit": "DOF-solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} PCG iterations of the oracle on the same {dofs}-DOF system "
                      f"({per_iter * 1e3:.0f} ms/iteration, single-threaded numpy/scipy + C loops), "
                      f"scaled to the {iters_full} iterations one solve to tol {tol:g} takes; "
                      f"host has {os.cpu_count()} logical CPUs"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="elasticity-32", choices=sorted(WORKLOADS))
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the event-timed pass")
    ap.add_argument("--precision", default="MIXED", choices=["MIXED", "FP32", "FP64"],
                    help="cycle arithmetic of the timed solve (FP64 outer loop always); "
                         "the FP64 PCG solve is timed beside it for comparison")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(one MI355X per process; sharding is a design note only)", file=sys.stderr)
        return 2

    import torch
    import paper_1503_01287_amd as amg

    wl = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    sysm = build_system(args.workload)
    t_asm = time.perf_counter() - t0
    print(f"# assembled {sysm.name}: {sysm.dofs} DOF in {t_asm:.1f}s", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    b = torch.from_numpy(sysm.rhs).to(dev)
    x = torch.zeros_like(b)

    def run_variant(precision: str, krylov: str, profile: bool) -> dict:
        """amg_setup (timed once), W warm-up and K timed solves; optionally
        the same K solves again with HIP events on the finest level."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver = amg.AMGSolver(sysm, smoother=wl["smoother"], krylov=krylov, precision=precision)
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
        levels = []
        for l in range(solver.num_levels):
            i = solver.level_info(l)
            levels.append(dict(nodes=i.n_lin + i.n_quad, nnz=int(i.nnz_A), colors=int(i.n_colors),
                               lanes=[int(i.lanes_A), int(i.lanes_gs)], fused=bool(i.fused)))
        print(f"# {precision}/{krylov} setup {setup_ms:.0f} ms, levels {levels}", file=sys.stderr, flush=True)

        def step():
            x.zero_()
            return solver.solve(b, x, tol=args.tol, maxit=1000)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        results = [step() for _ in range(args.steps)]
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        bad = [r for r in results if not (r.converged and r.relres <= args.tol * 1.0001)]
        if bad:
            raise SystemExit(f"# {precision}/{krylov}: solve did not converge: {bad[0]}")
        ms = elapsed * 1e3 / args.steps
        sol = x.clone()
        out = dict(precision=precision, krylov=krylov, setup_ms=round(setup_ms, 1), ms_per_step=round(ms, 3),
                   value=sysm.dofs * args.steps / elapsed, iterations=results[-1].iters,
                   relres=results[-1].relres, levels=levels, solution=sol)
        print(f"# {precision}/{krylov}: {args.steps} solves, {ms:.2f} ms/solve, {results[-1].iters} iterations, "
              f"relres {results[-1].relres:.2e}", file=sys.stderr, flush=True)
        if profile:
            solver.profile(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                step()
            torch.cuda.synchronize()
            prof_ms = (time.perf_counter() - t0) * 1e3 / args.steps
            classes = ["gs.L0", "resid.L0", "spmv.L0", "jacobi.L0", "jacobi0.L0", "restrict.L0", "prolong.L0"]
            stats = {c: solver.profile_read(c) for c in classes}
            solver.profile(0)
            stats = {c: v for c, v in stats.items() if v["launches"] > 0}
            dom = max(stats, key=lambda c: stats[c]["ms"])
            st = stats[dom]
            per_launch_bytes = st["bytes"] / st["launches"]
            per_launch_ms = st["ms"] / st["launches"]
            achieved = per_launch_bytes / (per_launch_ms * 1e-3) / 1e9
            out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                               "kernel": dom, "launches_per_step": st["launches"] // args.steps,
                               "bytes_per_launch": per_launch_bytes,
                               "mean_launch_us": round(per_launch_ms * 1e3, 2),
                               "profiled_ms_per_step": round(prof_ms, 2)}
            tot_b = sum(v["bytes"] for v in stats.values())
            tot_ms = sum(v["ms"] for v in stats.values())
            out["vcycle_bandwidth"] = {
                "finest_level_GBps": round(tot_b / (tot_ms * 1e-3) / 1e9, 1),
                "finest_level_ms_per_step": round(tot_ms / args.steps, 3),
                "per_class": {c: {"launches_per_step": v["launches"] // args.steps,
                                  "ms_per_step": round(v["ms"] / args.steps, 3),
                                  "GBps": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)}
                              for c, v in stats.items()}}
        solver.close()
        return out

    primary_kry = "PCG" if args.precision == "FP64" else "FCG"
    prim = run_variant(args.precision, primary_kry, not args.no_profile)
    comp = run_variant("FP64", "PCG", False) if args.precision != "FP64" else None
    # reference solution for the error of each variant: FP64 PCG to 1e-12 (untimed)
    ref_solver = amg.AMGSolver(sysm, smoother=wl["smoother"], krylov="PCG", precision="FP64")
    x.zero_()
    ref_res = ref_solver.solve(b, x, tol=1e-12, maxit=2000)
    ref = x.clone()
    ref_solver.close()

    def err(v):
        return float(torch.linalg.norm(v["solution"] - ref) / torch.linalg.norm(ref))

    prim["error_vs_fp64_reference"] = err(prim)
    if comp:
        comp["error_vs_fp64_reference"] = err(comp)
    ms, value, iters = prim["ms_per_step"], prim["value"], prim["iterations"]
    roofline = prim.get("roofline")
    vcycle = prim.get("vcycle_bandwidth")
    setup_ms, levels = prim["setup_ms"], prim["levels"]
    results_relres = prim["relres"]

    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        cpu = cpu_baseline(args.workload, comp["iterations"] if comp else iters, args.tol)
        print(f"# cpu baseline {time.perf_counter() - t0:.0f}s: {cpu['value']:.3g} DOF-solves/s",
              file=sys.stderr, flush=True)

    out = {
        "metric": "DOF-solves/s to 1e-8 rel. residual (mixed/learned vs plain FP64); V-cycle HBM GB/s",
        "value": round(value, 1),
        "unit": "DOF-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "FP64" else
                 ("f32 cycle, f64 outer" if args.precision == "FP32" else "f32/bf16 cycle, f64 outer"),
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl['desc']}", "dofs": sysm.dofs,
                   "smoother": wl["smoother"], "krylov": primary_kry, "precision": args.precision,
                   "tol": args.tol, "iterations": iters, "relres": results_relres,
                   "error_vs_fp64_reference": prim["error_vs_fp64_reference"],
                   "setup_ms": round(setup_ms, 1), "levels": levels, "parallelism": "single GPU"},
        "fp64_comparison": None if comp is None else {
            k: (float(f"{v:.6g}") if isinstance(v, float) else v) for k, v in comp.items()
            if k in ("precision", "krylov", "ms_per_step", "value", "iterations", "relres", "setup_ms",
                     "error_vs_fp64_reference")},
        "reference": {"krylov": "PCG", "precision": "FP64", "tol": 1e-12, "iterations": ref_res.iters},
        "roofline": roofline,
        "vcycle_bandwidth": vcycle,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
