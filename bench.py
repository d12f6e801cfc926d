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
PROFILES = os.path.join(ROOT, "profiles")


def measured_traffic(workload: str, precision: str, kernel_class: str, lanes: int, pair: int, xcd: int):
    """HBM bytes per launch of the dominant kernel from a committed rocprofv3
    --pmc summary of this workload (profiles/<workload>_*_traffic.md:
    FETCH_SIZE + WRITE_SIZE, copy-calibrated), if one covers this kernel
    class, precision and launch shape; else None."""
    if not os.path.isdir(PROFILES):
        return None
    for name in sorted(os.listdir(PROFILES)):
        if not (name.startswith(workload + "_") and name.endswith("_traffic.md")):
            continue
        with open(os.path.join(PROFILES, name)) as f:
            for line in f:
                if not line.startswith("traffic:"):
                    continue
                kv = dict(t.split("=", 1) for t in line.split()[1:])
                if (kv.get("class") == kernel_class and kv.get("precision") == precision
                        and int(kv.get("lanes", -1)) == lanes and int(kv.get("pair", 0)) == pair
                        and int(kv.get("xcd", 0)) == xcd):
                    return int(kv["bytes_per_launch"])
    return None


WORKLOADS = {
    "elasticity-32": dict(desc="linear elasticity, pure displacement, unit cube 32^3 cubes x 6 Kuhn tets, "
                               "hierarchical P2, E=1 nu=0.3, clamped x=0, random traction x=1",
                          smoother="GS-1-1"),
    "laplace-48": dict(desc="vector Laplacian, unit cube 48^3 cubes x 6 Kuhn tets, hierarchical P2, "
                            "one setup, then one solve per seeded trigonometric Dirichlet data set on x=0",
                   smoother="JA-1-1-0.5"),
    "laplace-4": dict(desc="vector Laplacian 4^3 cubes (2187 DOF)", smoother="GS-1-1"),
    "mixed-elasticity-24": dict(desc="mixed displacement-pressure elasticity, unit cube 24^3 cubes x 6 Kuhn tets, "
                                     "P2 displacement / P1 pressure, E=1 nu=0.49999, clamped x=0, random traction x=1",
                                smoother="sGS-1-1", saddle=True),
    "stokes-batch-64": dict(desc="64 lid-driven Stokes cavities (Taylor-Hood, mirrored Kuhn split), n^3 cubes with "
                                 "n ~ U{8..20}, lid speed ~ U[0.5, 2], mu=0.5, one merged hierarchy",
                            smoother="BS-1-1", saddle=True, batch=True, precision="FP32"),
}


class _Batch:
    """The 64 cavities as one right-hand side (systems one after another)."""

    def __init__(self, systems):
        import numpy as np
        self.systems = systems
        self.dofs = sum(s.dofs for s in systems)
        self.rhs = np.concatenate([s.rhs for s in systems])
        self.name = f"stokes-batch-{len(systems)}"


def build_system(name: str):
    from paper_1503_01287_amd import problems
    if name == "elasticity-32":
        return problems.elasticity(32)
    if name == "mixed-elasticity-24":
        return problems.mixed_elasticity(24)
    if name == "stokes-batch-64":
        import synth
        return _Batch([problems.stokes_cavity(n, sp) for n, sp in synth.stokes_batch()])
    if name == "laplace-48":
        import synth
        return problems.laplace(48, workload=synth.LAPLACE_LARGE, i=0)
    if name == "laplace-4":
        return problems.laplace(4)
    raise SystemExit(f"unknown workload {name}")


def _oracle_saddle_mv(o):
    import numpy as np
    A, B = o.A, o.B
    Bt = B.transpose()
    nv = 3 * A.nrows

    def mv(z):
        u, p = z[:nv].reshape(-1, 3), z[nv:]
        top = A.matvec(u).ravel() + Bt.matvec(p.reshape(-1, 1)).ravel()
        bot = B.matvec(u)[:, 0]
        if o.C is not None:
            bot = bot - o.C.matvec(p.reshape(-1, 1))[:, 0]
        return np.concatenate([top, bot])
    return mv, np.concatenate([o.f.ravel(), o.g])


def cpu_baseline(name: str, iters_full: int, tol: float, budget_s: float = 20.0) -> dict:
    """Time the CPU oracle's preconditioned Krylov iterations on the same
    workload (its own assembly and hierarchy, untimed) for about budget_s
    seconds and scale to one full solve (for the batch: to all systems)."""
    from oracle import amg as oamg, krylov, workloads
    import synth
    saddle = WORKLOADS[name].get("saddle", False)
    scale_dofs = None
    if name == "elasticity-32":
        o, sm = workloads.elasticity(32), "GS-1-1"
    elif name == "laplace-48":
        o, sm = workloads.laplace(48, workload=synth.LAPLACE_LARGE, i=0), "JA-1-1-0.5"
    elif name == "mixed-elasticity-24":
        o, sm = workloads.mixed_elasticity(24), "sGS-1-1"
    elif name == "stokes-batch-64":
        # one system of the batch (the median size), scaled by the batch's DOF
        cfg = synth.stokes_batch()
        n, sp = sorted(cfg)[len(cfg) // 2]
        o, sm = workloads.stokes(n, sp), "BS-1-1"
        scale_dofs = sum(3 * (2 * m + 1) ** 3 + (m + 1) ** 3 for m, _ in cfg)
    else:
        o, sm = workloads.laplace(4), "GS-1-1"
    print(f"# cpu baseline: oracle system assembled ({o.A.nrows} nodes)", file=sys.stderr, flush=True)
    if saddle:
        h = oamg.setup(o.A, o.nlin, o.nquad, B=o.B, C=o.C, singular=o.singular)
        if sm.startswith("BS"):
            oamg.prepare_bs(h)
        prec = oamg.preconditioner(h, oamg.Smoother.parse(sm))
        mv, rhs = _oracle_saddle_mv(o)
        run = lambda k: krylov.fgmres(mv, prec, rhs, tol=0.0, maxit=k)
        dofs = rhs.shape[0]
        method = "FGMRES"
    else:
        h = oamg.setup(o.A, o.nlin, o.nquad)
        prec = oamg.preconditioner(h, oamg.Smoother.parse(sm))
        mv = lambda v: o.A.matvec(v).ravel()
        pc = lambda r: prec(r).ravel()
        run = lambda k: krylov.pcg(mv, pc, o.b.ravel(), tol=0.0, maxit=k)
        dofs = 3 * o.A.nrows
        method = "PCG"
    print(f"# cpu baseline: oracle hierarchy built ({len(h.levels)} levels)", file=sys.stderr, flush=True)
    # a short first run measures the cost of one iteration, then a run sized to the budget
    t0 = time.perf_counter()
    run(1)
    t1 = max(time.perf_counter() - t0, 1e-3)
    k = int(max(1, min(iters_full, budget_s / t1)))
    t0 = time.perf_counter()
    run(k)
    per_iter = (time.perf_counter() - t0) / (k + 1)   # k iterations + the initial preconditioning
    solve_s = per_iter * (iters_full + 1)
    value = dofs / solve_s
    what = f"the same {dofs}-DOF system"
    if scale_dofs:
        value = dofs / solve_s   # DOF-solves/s of one system; the batch runs them one after another
        what = (f"one {dofs}-DOF cavity of the batch (median size), the batch's systems being solved one "
                f"after another at the same rate")
    return {"value": value, "unit": "DOF-solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} {method} iterations of the oracle on {what} "
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
    ap.add_argument("--only-timed", action="store_true",
                    help="for profiler runs: only the timed variant (no FP64 or unbatched comparison, no "
                         "reference solve, so no error figures)")
    ap.add_argument("--precision", default="MIXED", choices=["MIXED", "FP32", "FP64"],
                    help="cycle arithmetic of the timed solve (FP64 outer loop always; the Stokes batch "
                         "uses FP32 unless FP64 is asked for); the plain FP64 solve is timed beside it")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(one MI355X per process; sharding is a design note only)", file=sys.stderr)
        return 2

    import torch
    import paper_1503_01287_amd as amg
    from paper_1503_01287_amd import learned

    wl = WORKLOADS[args.workload]
    saddle, batch = wl.get("saddle", False), wl.get("batch", False)
    precision = wl.get("precision", args.precision) if args.precision != "FP64" else "FP64"
    t0 = time.perf_counter()
    sysm = build_system(args.workload)
    t_asm = time.perf_counter() - t0
    print(f"# assembled {sysm.name}: {sysm.dofs} DOF in {t_asm:.1f}s", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    b = torch.from_numpy(sysm.rhs).to(dev)
    x = torch.zeros_like(b)
    # right-hand sides: the vector Laplacian workload is one setup and many
    # solves, each with its own seeded Dirichlet data set (solve k uses data
    # set k); the others solve their one right-hand side repeatedly
    bs = [b]
    if args.workload == "laplace-48":
        import synth
        from paper_1503_01287_amd import problems
        t0 = time.perf_counter()
        bs = [torch.from_numpy(r).to(dev) for r in
              problems.laplace_rhs_many(sysm, synth.LAPLACE_LARGE, range(args.warmup + args.steps))]
        print(f"# {len(bs)} Dirichlet data sets in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    use_model = args.workload == "laplace-48" and os.path.exists(learned.MODEL_PATH)
    model = learned.DampingModel.load() if use_model else None

    def make(precision: str, krylov: str, with_model: bool):
        if batch:
            return amg.BatchedSolver(sysm.systems, smoother=wl["smoother"], precision=precision)
        kw = {"omega_model": model} if (with_model and model is not None) else {}
        return amg.AMGSolver(sysm, smoother=wl["smoother"], krylov=krylov, precision=precision, **kw)

    def solve_once(solver, tol, k=-1):
        x.zero_()
        r = solver.solve(bs[k % len(bs)], x, tol=tol, maxit=1000)
        if batch:
            ok = all(q.converged and q.relres <= tol * 1.0001 for q in r)
            return ok, max(q.iters for q in r), max(q.relres for q in r)
        return r.converged and r.relres <= tol * 1.0001, r.iters, r.relres

    def run_variant(precision: str, krylov: str, profile: bool, with_model: bool = False) -> dict:
        """amg_setup (timed once), W warm-up and K timed solves; optionally
        the same K solves again with HIP events on the finest level."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver = make(precision, krylov, with_model)
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
        levels = []
        for l in range(solver.num_levels):
            i = solver.level_info(l)
            levels.append(dict(nodes=i.n_lin + i.n_quad, pressure=i.n_pres, nnz=int(i.nnz_A), kept=int(i.kept_A), colors=int(i.n_colors),
                               lanes=[int(i.lanes_A), int(i.lanes_gs)], pair=[int(i.pair_A), int(i.pair_gs)],
                               fp64=[int(i.lanes64_A), int(i.pair64_A)],
                               gs_xcd=int(i.gs_xcd), fused=bool(i.fused),
                               omega=round(float(i.omega), 4)))
        print(f"# {precision}/{krylov} setup {setup_ms:.0f} ms, levels {levels}", file=sys.stderr, flush=True)
        for k in range(args.warmup):
            solve_once(solver, args.tol, k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        results = [solve_once(solver, args.tol, args.warmup + k) for k in range(args.steps)]
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        if not all(r[0] for r in results):
            raise SystemExit(f"# {precision}/{krylov}: solve did not converge: {results}")
        ms = elapsed * 1e3 / args.steps
        sol = x.clone()
        out = dict(precision=precision, krylov=krylov, setup_ms=round(setup_ms, 1), ms_per_step=round(ms, 3),
                   value=sysm.dofs * args.steps / elapsed, iterations=results[-1][1],
                   relres=results[-1][2], levels=levels, solution=sol, learned_omega=bool(with_model and model))
        print(f"# {precision}/{krylov}{' learned-omega' if out['learned_omega'] else ''}: {args.steps} solves, "
              f"{ms:.2f} ms/solve, {results[-1][1]} iterations, relres {results[-1][2]:.2e}",
              file=sys.stderr, flush=True)
        if profile:
            solver.profile(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(args.steps):
                solve_once(solver, args.tol, args.warmup + k)
            torch.cuda.synchronize()
            prof_ms = (time.perf_counter() - t0) * 1e3 / args.steps
            classes = ["gs.L0", "resid.L0", "spmv.L0", "jacobi.L0", "jacobi0.L0", "restrict.L0", "prolong.L0"]
            stats = {c: solver.profile_read(c) for c in classes}
            solver.profile(0)
            stats = {c: v for c, v in stats.items() if v["launches"] > 0}
            if stats:
                dom = max(stats, key=lambda c: stats[c]["ms"])
                st = stats[dom]
                per_launch_bytes = st["bytes"] / st["launches"]
                per_launch_ms = st["ms"] / st["launches"]
                achieved = per_launch_bytes / (per_launch_ms * 1e-3) / 1e9
                # the outer operator is the FP64 kernel; the cycle's kernels
                # are the reduced-precision copies unless the cycle is FP64
                if dom.startswith("spmv."):
                    lanes, pair, xcd = levels[0]["fp64"][0], levels[0]["fp64"][1], 0
                else:
                    which = 1 if dom.startswith("gs.") else 0
                    lanes, pair = levels[0]["lanes"][which], levels[0]["pair"][which]
                    xcd = levels[0]["gs_xcd"] if which else 0
                traffic = measured_traffic(args.workload, precision, dom, lanes, pair, xcd)
                out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
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

    full = not args.only_timed
    if saddle:
        prim = run_variant(precision, "FGMRES", not args.no_profile)
        comp = run_variant("FP64", "FGMRES", False) if precision != "FP64" and full else None
    else:
        primary_kry = "PCG" if precision == "FP64" else "FCG"
        prim = run_variant(precision, primary_kry, not args.no_profile, with_model=use_model)
        comp = run_variant("FP64", "PCG", False) if (precision != "FP64" or use_model) and full else None
    # the same systems solved one after another (batch only), once
    unbatched = None
    if batch and full:
        t_all, its = 0.0, []
        for s_ in sysm.systems:
            single = amg.AMGSolver(s_, smoother=wl["smoother"], krylov="FGMRES", precision=precision)
            bb = torch.from_numpy(s_.rhs).to(dev)
            xx = torch.zeros_like(bb)
            single.solve(bb, xx, tol=args.tol, maxit=1000)
            xx.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = single.solve(bb, xx, tol=args.tol, maxit=1000)
            torch.cuda.synchronize()
            t_all += time.perf_counter() - t0
            its.append(r.iters)
            single.close()
        unbatched = {"ms_per_step": round(t_all * 1e3, 2), "value": round(sysm.dofs / t_all, 1),
                     "iterations_max": max(its), "iterations_min": min(its),
                     "note": "the same systems, one amg_solve after another (warm, FGMRES, same smoother "
                             "and precision)"}
        print(f"# unbatched: {t_all * 1e3:.1f} ms for all systems", file=sys.stderr, flush=True)

    # reference solution for the error of each variant: FP64 to 1e-12 (untimed)
    ref_iters = None
    prim["error_vs_fp64_reference"] = None
    if full:
        ref_solver = make("FP64", "FGMRES" if saddle else "PCG", False)
        # the same right-hand side as the variants' last timed solve
        last = args.warmup + args.steps - 1
        solve_once(ref_solver, 1e-12, last)
        ref = x.clone()
        ref_res = solve_once(ref_solver, 1e-12, last)
        ref_solver.close()
        ref_iters = ref_res[1]

        def centred(v):
            """Pressure of systems with constants in the pressure kernel taken with zero mean."""
            if not saddle:
                return v
            v = v.clone()
            systems = sysm.systems if batch else [sysm]
            o = 0
            for s_ in systems:
                if s_.pressure_kernel:
                    nu = 3 * s_.nodes
                    p_ = v[o + nu:o + s_.dofs]
                    p_ -= p_.mean()
                o += s_.dofs
            return v

        refc = centred(ref)

        def err(v):
            return float(torch.linalg.norm(centred(v["solution"]) - refc) / torch.linalg.norm(refc))

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

    kry = prim["krylov"]
    dtype = "f64" if precision == "FP64" else (
        "f32 cycle, f64 outer" if precision == "FP32" else "f32/bf16 cycle, f64 outer")
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
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl['desc']}", "dofs": sysm.dofs,
                   "smoother": wl["smoother"], "krylov": kry, "precision": precision,
                   "learned_omega": prim["learned_omega"],
                   "tol": args.tol, "iterations": iters, "relres": results_relres,
                   "error_vs_fp64_reference": prim["error_vs_fp64_reference"],
                   "setup_ms": round(setup_ms, 1), "levels": levels, "parallelism": "single GPU",
                   "rhs_data_sets": len(bs)},
        "fp64_comparison": None if comp is None else {
            k: (float(f"{v:.6g}") if isinstance(v, float) else v) for k, v in comp.items()
            if k in ("precision", "krylov", "ms_per_step", "value", "iterations", "relres", "setup_ms",
                     "error_vs_fp64_reference")},
        "unbatched_comparison": unbatched,
        "reference": {"krylov": "FGMRES" if saddle else "PCG", "precision": "FP64", "tol": 1e-12,
                      "iterations": ref_iters},
        "roofline": roofline,
        "vcycle_bandwidth": vcycle,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
