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


def measured_traffic(workload: str, precision: str, kernel_class: str, lanes: int, trip: int, xcd: int):
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
                        and int(kv.get("lanes", -1)) == lanes and int(kv.get("trip", 0)) == trip
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
    from oracle import threaded
    # a short first run measures the cost of one iteration, then a run sized to the budget
    t0 = time.perf_counter()
    run(1)
    t1 = max(time.perf_counter() - t0, 1e-3)
    k = int(max(1, min(iters_full, budget_s / t1)))
    t0 = time.perf_counter()
    run(k)
    per_iter = (time.perf_counter() - t0) / (k + 1)   # k iterations + the initial preconditioning
    # the same k iterations with the oracle's order-independent loops on every host core
    want = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    with threaded.on_threads(h, want):
        cores = threaded.threads()
        run(1)
        t0 = time.perf_counter()
        run(k)
        per_iter_mt = (time.perf_counter() - t0) / (k + 1)
    print(f"# cpu baseline: {per_iter * 1e3:.0f} ms/iteration on 1 thread, {per_iter_mt * 1e3:.0f} on {cores}",
          file=sys.stderr, flush=True)
    what = f"the same {dofs}-DOF system"
    if scale_dofs:
        # DOF-solves/s of one system; the batch runs them one after another
        what = (f"one {dofs}-DOF cavity of the batch (median size), the batch's systems being solved one "
                f"after another at the same rate")
    model = _cpu_model()
    scaled = f"scaled to the {iters_full} iterations one solve to tol {tol:g} takes"
    single = {"value": dofs / (per_iter * (iters_full + 1)), "unit": "DOF-solves/s", "cores": 1,
              "ms_per_iteration": round(per_iter * 1e3, 1),
              "sample": f"the same {k} iterations on one thread (numpy/scipy + sequential C loops), {scaled}"}
    return {"value": dofs / (per_iter_mt * (iters_full + 1)), "unit": "DOF-solves/s", "cores": cores,
            "kind": "oracle", "ms_per_iteration": round(per_iter_mt * 1e3, 1),
            "sample": f"{k} {method} iterations of the oracle on {what}, its block and transfer products, "
                      f"Gauss-Seidel colours and Jacobi steps on {cores} OpenMP threads (dot products and "
                      f"vector updates numpy's), {scaled}; host: {os.cpu_count()} logical CPUs, {model}",
            "single_thread": single}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "CPU model unknown"


# kernel classes of the library's profiler (amg_profile_read): one launch of
# one kernel per event pair, except "blas" (a partial-sum kernel and its
# reduction), which the roofline leaves out
CYCLE_OPS = ("gs", "resid", "jacobi", "jacobi0", "restrict", "prolong", "vanka", "spmv")
SINGLE_CLASSES = ("coarse", "dense_tail", "saddle_tail", "tail")


SETUP_PHASES = ("upload", "coarsen", "galerkin", "omega_network", "drop_zeros", "smoother", "autotune", "coarsest",
                "omega_bound", "schur", "schur_map", "vanka", "coarse_map", "reduced_copies", "saddle_map", "merge")


def setup_breakdown(solver) -> dict:
    """Wall ms per setup phase (the library records them at every setup) and
    the Galerkin numeric kernels' rate. A batch sets its systems up on
    several host threads: "systems" is that step's wall ms, and
    "systems_summed" its systems' own phases summed over them."""
    out = {}
    for ph in SETUP_PHASES:
        r = solver.profile_read("setup." + ph)
        if r["launches"]:
            out[ph] = round(r["ms"], 1)
    r = solver.profile_read("setup.systems")
    if r["launches"]:
        out["systems"] = round(r["ms"], 1)
        summed = {}
        for ph in SETUP_PHASES:
            q = solver.profile_read("setup.systems." + ph)
            if q["launches"]:
                summed[ph] = round(q["ms"], 1)
        out["systems_summed"] = summed
    g = solver.profile_read("setup.spgemm_numeric")
    if g["launches"]:
        gbps = g["bytes"] / max(g["ms"] * 1e-3, 1e-12) / 1e9
        out["spgemm_numeric"] = {"launches": g["launches"], "ms": round(g["ms"], 2),
                                 "algorithmic_bytes": int(g["bytes"]), "GBps": round(gbps, 1),
                                 "frac": round(gbps / HBM_PEAK_GBS, 4)}
    return out


def _profile_classes(nlevels: int) -> list:
    return [f"{op}.L{l}" for l in range(nlevels) for op in CYCLE_OPS] + list(SINGLE_CLASSES) + ["blas"]


def _class_shape(cls: str, levels: list):
    """(lanes, entries per trip, xcd) of the kernel a class launches, for the traffic lookup."""
    if "." not in cls:
        return -1, 0, 0
    op, lv = cls.split(".")
    lv = levels[int(lv[1:])]
    if op == "spmv":
        return lv["fp64"][0], lv["fp64"][1], 0
    which = 1 if op == "gs" else 0
    return lv["lanes"][which], lv["trip"][which], (lv["gs_xcd"] if which else 0)


# ---------------------------------------------------------------- assembly
def _assemble_cavity(args):
    from paper_1503_01287_amd import problems
    n, sp = args
    return problems.stokes_cavity(n, sp)


class _Grid:
    def __init__(self, n):
        self.n = n


def _laplace_rhs_chunk(args):
    import synth
    from paper_1503_01287_amd import problems
    n, ids = args
    return problems.laplace_rhs_many(_Grid(n), synth.LAPLACE_LARGE, ids)


def _pool(workers: int):
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    # spawn: the workers start clean (no GPU runtime state from this process)
    return ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"))


def assemble(name: str, n_rhs: int, workers: int):
    """The workload's system (host arrays) and its right-hand sides, the
    independent pieces assembled in parallel on the host cores."""
    import synth
    from paper_1503_01287_amd import problems
    if name == "stokes-batch-64":
        with _pool(workers) as ex:
            systems = list(ex.map(_assemble_cavity, synth.stokes_batch()))
        b = _Batch(systems)
        return b, [b.rhs]
    sysm = build_system(name)
    if name != "laplace-48":
        return sysm, [sysm.rhs]
    ids = list(range(n_rhs))
    k = max(1, min(workers, 8, len(ids)))
    chunks = [(sysm.n, ids[i::k]) for i in range(k)]
    with _pool(k) as ex:
        parts = list(ex.map(_laplace_rhs_chunk, chunks))
    rhs = [None] * len(ids)
    for (_, cid), part in zip(chunks, parts):
        for i, r in zip(cid, part):
            rhs[i] = r
    return sysm, rhs


# ---------------------------------------------------------------- measurement
def measure(name: str, sysm, rhs, steps: int, warmup: int, tol: float, precision: str, profile: bool,
            variants: list, reference: bool = True) -> dict:
    """Time each variant (setup once, `warmup` untimed and `steps` timed
    solves, right-hand side k for solve k), optionally profile the first one
    (HIP events around every launch of every level), and measure every
    variant's error against an FP64 solve of the last right-hand side to
    1e-12 (run by the FP64 variant's own hierarchy)."""
    import torch
    import paper_1503_01287_amd as amg
    from paper_1503_01287_amd import learned
    wl = WORKLOADS[name]
    saddle, batch = wl.get("saddle", False), wl.get("batch", False)
    dev = torch.device("cuda:0")
    bs = [torch.from_numpy(r).to(dev) for r in rhs]
    x = torch.zeros_like(bs[0])
    model = learned.DampingModel.load() if os.path.exists(learned.MODEL_PATH) else None

    def make(prec: str, krylov: str, with_model: bool, omega=None, smoother=None):
        sm = smoother or wl["smoother"]
        if batch:
            return amg.BatchedSolver(sysm.systems, smoother=sm, precision=prec)
        kw = {"omega_model": model} if (with_model and model is not None) else {}
        if omega is not None:
            kw["level_omega"] = [omega]
        return amg.AMGSolver(sysm, smoother=sm, krylov=krylov, precision=prec, **kw)

    def solve_once(solver, t, k=-1):
        x.zero_()
        r = solver.solve(bs[k % len(bs)], x, tol=t, maxit=1000)
        if batch:
            return all(q.converged and q.relres <= t * 1.0001 for q in r), max(q.iters for q in r), \
                max(q.relres for q in r)
        return r.converged and r.relres <= t * 1.0001, r.iters, r.relres

    def levels_of(solver):
        out = []
        for l in range(solver.num_levels):
            i = solver.level_info(l)
            out.append(dict(nodes=i.n_lin + i.n_quad, pressure=i.n_pres, nnz=int(i.nnz_A), kept=int(i.kept_A),
                            colors=int(i.n_colors), lanes=[int(i.lanes_A), int(i.lanes_gs)],
                            trip=[int(i.trip_A), int(i.trip_gs)], fp64=[int(i.lanes64_A), int(i.trip64_A)],
                            gs_xcd=int(i.gs_xcd), fused=bool(i.fused), coarse_map=bool(i.coarse_map),
                            omega=round(float(i.omega), 4)))
        return out

    def run_variant(v: dict) -> dict:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver = make(v["precision"], v["krylov"], v.get("model", False), v.get("omega"), v.get("smoother"))
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
        levels = levels_of(solver)
        phases = setup_breakdown(solver)
        print(f"# {name} {v['label']}: setup {setup_ms:.0f} ms {phases}", file=sys.stderr, flush=True)
        for k in range(warmup):
            solve_once(solver, tol, k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        results = [solve_once(solver, tol, warmup + k) for k in range(steps)]
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        if not all(r[0] for r in results):
            raise SystemExit(f"# {name} {v['label']}: solve did not converge: {results}")
        ms = elapsed * 1e3 / steps
        out = dict(label=v["label"], smoother=v.get("smoother") or wl["smoother"], precision=v["precision"],
                   krylov=v["krylov"], setup_ms=round(setup_ms, 1),
                   setup_phases_ms=phases,
                   ms_per_step=round(ms, 3), value=sysm.dofs * steps / elapsed, iterations=results[-1][1],
                   relres=results[-1][2], levels=levels, solution=x.clone(),
                   learned_omega=bool(v.get("model") and model is not None))
        if v.get("omega") is not None:
            out["omega"] = v["omega"]
        print(f"# {name} {v['label']}: {steps} solves, {ms:.2f} ms/solve, {results[-1][1]} iterations, "
              f"relres {results[-1][2]:.2e}", file=sys.stderr, flush=True)
        if v.get("profile"):
            out.update(profile_pass(solver, levels))
        if v.get("reference"):
            last = warmup + steps - 1
            ok, its, _ = solve_once(solver, 1e-12, last)
            out["reference"] = (x.clone(), its)
        solver.close()
        return out

    def profile_pass(solver, levels) -> dict:
        """The same solves again with HIP events around every launch."""
        solver.profile(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            solve_once(solver, tol, warmup + k)
        torch.cuda.synchronize()
        prof_ms = (time.perf_counter() - t0) * 1e3 / steps
        stats = {c: solver.profile_read(c) for c in _profile_classes(len(levels))}
        solver.profile(0)
        stats = {c: v for c, v in stats.items() if v["launches"] > 0}
        res = {}
        kern = {c: v for c, v in stats.items() if c != "blas"}
        if kern:
            dom = max(kern, key=lambda c: kern[c]["ms"])
            st = kern[dom]
            per_launch_bytes = st["bytes"] / st["launches"]
            per_launch_ms = st["ms"] / st["launches"]
            achieved = per_launch_bytes / (per_launch_ms * 1e-3) / 1e9
            lanes, trip, xcd = _class_shape(dom, levels)
            traffic = measured_traffic(name, precision, dom, lanes, trip, xcd)
            res["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                               "kernel": dom, "launch_shape": {"lanes": lanes, "trip": trip, "xcd": xcd},
                               "launches_per_step": st["launches"] // steps,
                               "bytes_per_launch": per_launch_bytes,
                               "mean_launch_us": round(per_launch_ms * 1e3, 2),
                               "profiled_ms_per_step": round(prof_ms, 2)}

            def agg(sel):
                b_ = sum(v["bytes"] for c, v in sel.items())
                m_ = sum(v["ms"] for c, v in sel.items())
                return round(b_ / max(m_ * 1e-3, 1e-12) / 1e9, 1), round(m_ / steps, 3)
            cyc = {c: v for c, v in kern.items() if c != "spmv.L0"}
            fin = {c: v for c, v in cyc.items() if c.endswith(".L0")}
            all_gbps, all_ms = agg(cyc)
            fin_gbps, fin_ms = agg(fin)
            per_level = {}
            for l in range(len(levels)):
                lv = {c: v for c, v in cyc.items() if c.endswith(f".L{l}")}
                if lv:
                    g_, m_ = agg(lv)
                    per_level[f"L{l}"] = {"GBps": g_, "ms_per_step": m_}
            ce = {c: v for c, v in cyc.items() if c in SINGLE_CLASSES}
            if ce:
                g_, m_ = agg(ce)
                per_level["coarse_end"] = {"GBps": g_, "ms_per_step": m_}
            res["vcycle_bandwidth"] = {
                "all_levels_GBps": all_gbps, "all_levels_ms_per_step": all_ms,
                "all_levels_frac": round(all_gbps / HBM_PEAK_GBS, 4),
                "finest_level_GBps": fin_gbps, "finest_level_ms_per_step": fin_ms,
                "per_level": per_level,
                "per_class": {c: {"launches_per_step": v["launches"] // steps,
                                  "ms_per_step": round(v["ms"] / steps, 3),
                                  "GBps": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)}
                              for c, v in sorted(kern.items(), key=lambda kv: -kv[1]["ms"])},
                "note": "algorithmic bytes over HIP-event time per launch, every launch of every level; "
                        "all_levels: the V-cycle's kernels (the outer FP64 operator spmv.L0 and the Krylov "
                        "vector kernels excluded)"}
        return res

    out = {"workload": f"{name}: {wl['desc']}", "dofs": sysm.dofs, "rhs_data_sets": len(bs), "variants": {}}
    ref = None
    for v in variants:
        r = run_variant(v)
        if "reference" in r:
            ref, out["reference_iterations"] = r.pop("reference")
        out["variants"][v["label"]] = r
    if ref is not None:
        def centred(t):
            if not saddle:
                return t
            t = t.clone()
            o = 0
            for s_ in (sysm.systems if batch else [sysm]):
                if s_.pressure_kernel:
                    p_ = t[o + 3 * s_.nodes:o + s_.dofs]
                    p_ -= p_.mean()
                o += s_.dofs
            return t
        refc = centred(ref)
        for r in out["variants"].values():
            r["error_vs_fp64_reference"] = float(torch.linalg.norm(centred(r["solution"]) - refc)
                                                 / torch.linalg.norm(refc))
    for r in out["variants"].values():
        r.pop("solution", None)
    return out


def measure_blocks(name: str, sysm, rhs, K: int, precision: str, krylov: str, with_model: bool, tol: float,
                   passes: int = 1) -> dict:
    """Every right-hand side of `rhs` solved in blocks of K by amg_solve_multi
    (one setup; one untimed warm-up block, then `passes` timed passes over all
    blocks); DOF-solves/s over the timed blocks, and each block's first
    right-hand side against an FP64 solve to 1e-12 of it alone."""
    import numpy as np
    import torch
    import paper_1503_01287_amd as amg
    from paper_1503_01287_amd import learned
    wl = WORKLOADS[name]
    dev = torch.device("cuda:0")
    model = learned.DampingModel.load() if (with_model and os.path.exists(learned.MODEL_PATH)) else None
    kw = {"omega_model": model} if model is not None else {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = amg.AMGSolver(sysm, smoother=wl["smoother"], krylov=krylov, precision=precision, **kw)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    blocks = [torch.from_numpy(np.ascontiguousarray(np.stack(rhs[i:i + K]))).to(dev) for i in range(0, len(rhs), K)]
    X = torch.zeros_like(blocks[0])
    s.solve_multi(blocks[0], X, tol=tol, maxit=1000)
    iters, rel, sols = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(passes):
        sols = []
        for Bk in blocks:
            Xk = torch.zeros_like(Bk)
            res = s.solve_multi(Bk, Xk, tol=tol, maxit=1000)
            if not all(r.converged and r.relres <= tol * 1.0001 for r in res):
                raise SystemExit(f"# {name} block solve did not converge: {res}")
            iters += [r.iters for r in res]
            rel += [r.relres for r in res]
            sols.append(Xk[0].clone())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s.close()
    nsolves = passes * len(rhs)
    # error of each block's first right-hand side against an FP64 solve of it
    ref = amg.AMGSolver(sysm, smoother=wl["smoother"], krylov="PCG", precision="FP64")
    errs = []
    for Bk, xk in zip(blocks, sols):
        xr = torch.zeros_like(Bk[0])
        ref.solve(Bk[0].contiguous(), xr, tol=1e-12, maxit=1000)
        errs.append(float(torch.linalg.norm(xk - xr) / torch.linalg.norm(xr)))
    ref.close()
    out = {"rhs_per_block": K, "rhs": len(rhs), "blocks": len(blocks), "precision": precision, "krylov": krylov,
           "learned_omega": model is not None, "setup_ms": round(setup_ms, 1),
           "ms_per_block": round(elapsed * 1e3 / (passes * len(blocks)), 3),
           "ms_per_rhs": round(elapsed * 1e3 / nsolves, 3),
           "value": float(f"{sysm.dofs * nsolves / elapsed:.6g}"),
           "iterations_max": max(iters), "iterations_min": min(iters), "relres_max": max(rel),
           "error_vs_fp64_reference_max": max(errs)}
    print(f"# {name} blocks of {K}: {out['ms_per_rhs']:.2f} ms per right-hand side, iterations "
          f"{min(iters)}-{max(iters)}", file=sys.stderr, flush=True)
    return out


def variants_for(name: str, precision: str, profile: bool, extras: bool) -> list:
    wl = WORKLOADS[name]
    saddle = wl.get("saddle", False)
    prec = wl.get("precision", precision) if precision != "FP64" else "FP64"
    kry = "FGMRES" if saddle else ("PCG" if prec == "FP64" else "FCG")
    fp64_kry = "FGMRES" if saddle else "PCG"
    if name == "laplace-48":
        v = [dict(label="learned_mixed", precision=prec, krylov=kry, model=True, profile=profile)]
        if extras:
            v.append(dict(label="fixed_mixed", precision=prec, krylov=kry))
        v.append(dict(label="fixed_fp64", precision="FP64", krylov=fp64_kry, reference=True))
        return v
    v = [dict(label="primary", precision=prec, krylov=kry, profile=profile)]
    if prec != "FP64":
        v.append(dict(label="fp64", precision="FP64", krylov=fp64_kry, reference=True))
    else:
        v[0]["reference"] = True
    if name == "mixed-elasticity-24" and extras:
        # the other two saddle smoothers of Section 3.3 on the same system (FP64)
        v.append(dict(label="bs_fp64", smoother="BS-1-1", precision="FP64", krylov="FGMRES"))
        v.append(dict(label="vanka_fp64", smoother="Vanka-1-1", precision="FP64", krylov="FGMRES"))
    return v


def best_global_omega(name: str, sysm, rhs, tol: float, grid=None) -> dict:
    """The best single damping weight for every level (JA, reduced-precision
    cycle in FCG): fewest iterations on the first right-hand side over a grid,
    ties broken by time; the baseline the learned per-level weights are
    compared with beside the paper's fixed 0.5."""
    import torch
    import paper_1503_01287_amd as amg
    dev = torch.device("cuda:0")
    b = torch.from_numpy(rhs[0]).to(dev)
    x = torch.zeros_like(b)
    s = amg.AMGSolver(sysm, smoother="JA-1-1-0.5", krylov="FCG", precision="MIXED")
    # up to the smallest level bound 0.95 * 2 / lambda_max(D^-1 A_l): beyond
    # it the cycle need not be positive definite
    top = min(s.level_info(l).omega_max for l in range(s.num_levels - 1))
    grid = grid or [round(0.30 + 0.05 * i, 2) for i in range(40) if 0.30 + 0.05 * i <= top + 1e-9]
    rows = []
    for w in grid:
        s.set_level_omega([w])
        x.zero_()
        r = s.solve(b, x, tol=tol, maxit=300)
        torch.cuda.synchronize()
        x.zero_()
        t0 = time.perf_counter()
        r = s.solve(b, x, tol=tol, maxit=300)
        torch.cuda.synchronize()
        rows.append((r.iters if r.converged else 10 ** 6, time.perf_counter() - t0, w))
    s.close()
    its, t, w = min(rows)
    print(f"# {name}: best global omega {w} ({its} iterations)", file=sys.stderr, flush=True)
    return {"omega": w, "iterations": its, "grid": [g[2] for g in rows], "grid_iterations": [g[0] for g in rows]}


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
                    help="for profiler runs: only the timed variant (no FP64 comparison, no reference "
                         "solve, so no error figures, no other workloads)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads' lines (learned damping on the 48^3 Laplacian, the "
                         "64-cavity Stokes batch) that the default elasticity run adds")
    ap.add_argument("--precision", default="MIXED", choices=["MIXED", "FP32", "FP64"],
                    help="cycle arithmetic of the timed solve (FP64 outer loop always; the Stokes batch "
                         "uses FP32 unless FP64 is asked for); the plain FP64 solve is timed beside it")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="host processes for assembling independent systems and right-hand sides")
    ap.add_argument("--rhs-block", type=int, default=0,
                    help="laplace-48: solve --rhs-count Dirichlet data sets in blocks of this many right-hand "
                         "sides (amg_solve_multi); one step = one block")
    ap.add_argument("--rhs-count", type=int, default=256)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(one MI355X per process; sharding is a design note only)", file=sys.stderr)
        return 2

    name = args.workload
    if args.rhs_block:
        return block_main(args)
    full = not args.only_timed
    extras = full and not args.no_extras and name == "elasticity-32"
    extra_steps, extra_warmup = min(args.steps, 5), 1
    # host assembly first, before this process touches the GPU
    t0 = time.perf_counter()
    sysm, rhs = assemble(name, args.warmup + args.steps, args.workers)
    print(f"# assembled {sysm.name}: {sysm.dofs} DOF, {len(rhs)} right-hand side(s) in "
          f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    other = {}
    other_block_rhs = []
    if extras:
        for xn in ("laplace-48", "stokes-batch-64"):
            t0 = time.perf_counter()
            # the Laplacian: the single-solve data sets, then 10 more (16 in all, two blocks of 8)
            other[xn] = assemble(xn, extra_warmup + extra_steps + (10 if xn == "laplace-48" else 0), args.workers)
            if xn == "laplace-48":
                xs_, xr_ = other[xn]
                other_block_rhs = xr_[extra_warmup + extra_steps:]
                other[xn] = (xs_, xr_[:extra_warmup + extra_steps])
            print(f"# assembled {xn} in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)

    precision = WORKLOADS[name].get("precision", args.precision) if args.precision != "FP64" else "FP64"
    vs = variants_for(name, args.precision, not args.no_profile,
                      full and not args.no_extras and name == "mixed-elasticity-24")
    if not full:
        vs = [dict(v, reference=False) for v in vs[:1]]
    prim_all = measure(name, sysm, rhs, args.steps, args.warmup, args.tol, precision, not args.no_profile, vs)
    labels = list(prim_all["variants"])
    prim = prim_all["variants"][labels[0]]
    comp = prim_all["variants"].get("fp64") if len(labels) > 1 else None
    smoothers = {lab: {k: (float(f"{v:.6g}") if isinstance(v, float) else v) for k, v in r.items()
                       if k in ("smoother", "precision", "krylov", "ms_per_step", "iterations", "relres", "setup_ms",
                                "error_vs_fp64_reference")}
                 for lab, r in prim_all["variants"].items() if lab in ("bs_fp64", "vanka_fp64")}

    others = None
    if extras:
        others = {}
        for xn, (xs, xr) in other.items():
            xprec = WORKLOADS[xn].get("precision", "MIXED")
            res = measure(xn, xs, xr, extra_steps, extra_warmup, args.tol, xprec, False,
                          variants_for(xn, args.precision, False, True))
            if xn == "laplace-48":
                best = best_global_omega(xn, xs, xr, args.tol)
                bw = measure(xn, xs, xr, extra_steps, extra_warmup, args.tol, "MIXED", False,
                             [dict(label="best_global_omega_mixed", precision="MIXED", krylov="FCG",
                                   omega=best["omega"]),
                              dict(label="fixed_fp64", precision="FP64", krylov="PCG", reference=True)])
                res["variants"]["best_global_omega_mixed"] = bw["variants"]["best_global_omega_mixed"]
                res["best_global_omega_search"] = best
                res["blocks_of_rhs"] = measure_blocks(xn, xs, xr + other_block_rhs, 8, "MIXED", "FCG", True,
                                                      args.tol)
            for r in res["variants"].values():
                r.pop("levels", None)
                for k in ("value", "relres"):
                    r[k] = float(f"{r[k]:.6g}")
            others[xn] = res

    ms, value, iters = prim["ms_per_step"], prim["value"], prim["iterations"]
    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        cpu = cpu_baseline(name, comp["iterations"] if comp else iters, args.tol)
        print(f"# cpu baseline {time.perf_counter() - t0:.0f}s: {cpu['value']:.3g} DOF-solves/s",
              file=sys.stderr, flush=True)

    wl = WORKLOADS[name]
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
        "config": {"workload": prim_all["workload"], "dofs": sysm.dofs,
                   "smoother": wl["smoother"], "krylov": prim["krylov"], "precision": precision,
                   "learned_omega": prim["learned_omega"],
                   "tol": args.tol, "iterations": iters, "relres": prim["relres"],
                   "error_vs_fp64_reference": prim.get("error_vs_fp64_reference"),
                   "setup_ms": prim["setup_ms"], "setup_phases_ms": prim["setup_phases_ms"],
                   "levels": prim["levels"], "parallelism": "single GPU",
                   "rhs_data_sets": prim_all["rhs_data_sets"]},
        "fp64_comparison": None if comp is None else {
            k: (float(f"{v:.6g}") if isinstance(v, float) else v) for k, v in comp.items()
            if k in ("precision", "krylov", "ms_per_step", "value", "iterations", "relres", "setup_ms",
                     "error_vs_fp64_reference", "learned_omega")},
        "reference": {"krylov": "FGMRES" if wl.get("saddle") else "PCG", "precision": "FP64", "tol": 1e-12,
                      "iterations": prim_all.get("reference_iterations")},
        "roofline": prim.get("roofline"),
        "vcycle_bandwidth": prim.get("vcycle_bandwidth"),
        "cpu_baseline": cpu,
        "other_workloads": others,
    }
    if smoothers:
        out["other_saddle_smoothers"] = smoothers
    print(json.dumps(out))
    return 0


def block_main(args) -> int:
    """--rhs-block K: every Dirichlet data set of the 48^3 Laplacian workload
    in blocks of K right-hand sides; one JSON line like main()'s, one step =
    one block of K solves, value = DOF-solves/s of the timed blocks."""
    if args.workload != "laplace-48":
        raise SystemExit("--rhs-block applies to the laplace-48 workload")
    K = args.rhs_block
    t0 = time.perf_counter()
    sysm, rhs = assemble("laplace-48", args.rhs_count, args.workers)
    print(f"# assembled {sysm.name}: {args.rhs_count} data sets in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    learned_ = measure_blocks("laplace-48", sysm, rhs, K, "MIXED", "FCG", True, args.tol)
    fixed64 = measure_blocks("laplace-48", sysm, rhs, K, "FP64", "PCG", False, args.tol)
    out = {
        "metric": "DOF-solves/s to 1e-8 rel. residual (mixed/learned vs plain FP64); V-cycle HBM GB/s",
        "value": learned_["value"], "unit": "DOF-solves/s", "n_gpus": 1, "steps": learned_["blocks"],
        "warmup": 1, "ms_per_step": learned_["ms_per_block"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32/bf16 cycle, f64 outer", "data": "synthetic",
        "config": {"workload": f"laplace-48: {WORKLOADS['laplace-48']['desc']}", "dofs": sysm.dofs,
                   "rhs_data_sets": args.rhs_count, "rhs_per_block": K, "smoother": "JA-1-1",
                   "learned_omega": learned_["learned_omega"], "tol": args.tol},
        "learned_mixed_blocks": learned_, "fixed_fp64_blocks": fixed64,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
