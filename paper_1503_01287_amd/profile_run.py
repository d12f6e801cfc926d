"""A short, fixed run for hardware-counter profiles (rocprofv3 --pmc).

amg_setup of one workload in the configuration bench.py times (same
smoother, Krylov method, precision and, for the Laplacian, the learned
damping), then - inside a roctx profiler region, so that rocprofv3
--selected-regions collects only there and the setup and its tuners run
unprofiled - a plain device-to-device copy of a known size (the calibration
for the HBM traffic counters) and a few solves.

    rocprofv3 --pmc FETCH_SIZE --selected-regions ... -- python3 -m paper_1503_01287_amd.profile_run --workload elasticity-32
"""
from __future__ import annotations

import argparse
import ctypes
import os
import sys
import time


def _roctx():
    """roctxProfilerResume / roctxProfilerPause of the profiler SDK (no-ops
    without a profiler); None if the library is absent."""
    for name in ("librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so"):
        try:
            lib = ctypes.CDLL(name)
            lib.roctxProfilerResume.argtypes = [ctypes.c_uint64]
            lib.roctxProfilerPause.argtypes = [ctypes.c_uint64]
            return lib
        except (OSError, AttributeError):
            continue
    return None


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="elasticity-32",
                    choices=["elasticity-32", "mixed-elasticity-24", "laplace-48", "stokes-batch-64"])
    ap.add_argument("--precision", default=None, choices=["FP64", "MIXED", "FP32"],
                    help="default: MIXED, FP32 for the Stokes batch")
    ap.add_argument("--smoother", default=None,
                    help="default: the workload's (GS-1-1, JA-1-1-0.5, sGS-1-1, BS-1-1)")
    ap.add_argument("--solves", type=int, default=1)
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--fuse-coarse", type=int, default=1, choices=[0, 1],
                    help="0: no assembled coarse-end maps (the 64-cavity batch's map assembly issues"
                         " some 10^5-10^6 small dispatches, which the counter profiler does not survive;"
                         " the finest-level kernels and operators are the same)")
    ap.add_argument("--shape", action="append", default=[],
                    help="LEVEL:KERNELS:LANES:TRIP[:XCD] fixes a launch shape after the setup (kernels natural,"
                         " sweep, natural_rp or sweep_rp), so that the runs of the two counters time the same"
                         " kernel whatever the tuner picked")
    args = ap.parse_args()

    import torch
    import synth
    from . import problems, AMGSolver, BatchedSolver, learned
    dev = torch.device("cuda:0")

    wl = args.workload
    prec = args.precision or ("FP32" if wl == "stokes-batch-64" else "MIXED")
    if wl == "stokes-batch-64":
        systems = [problems.stokes_cavity(n, sp) for n, sp in synth.stokes_batch()]
        s = BatchedSolver(systems, smoother=args.smoother or "BS-1-1", precision=prec,
                          fuse_coarse=bool(args.fuse_coarse))
        rhs = __import__("numpy").concatenate([q.rhs for q in systems])
        kry = "FGMRES"
    else:
        kw = {}
        if wl == "elasticity-32":
            sysm, kw["smoother"] = problems.elasticity(32), "GS-1-1"
        elif wl == "laplace-48":
            sysm, kw["smoother"] = problems.laplace(48, workload=synth.LAPLACE_LARGE, i=0), "JA-1-1-0.5"
            if prec != "FP64" and os.path.exists(learned.MODEL_PATH):
                kw["omega_model"] = learned.DampingModel.load()
        else:
            sysm, kw["smoother"] = problems.mixed_elasticity(24), "sGS-1-1"
        saddle = sysm.n_pres > 0
        kry = "FGMRES" if saddle else ("PCG" if prec == "FP64" else "FCG")
        if args.smoother:
            kw["smoother"] = args.smoother
        s = AMGSolver(sysm, krylov=kry, precision=prec, fuse_coarse=bool(args.fuse_coarse), **kw)
        rhs = sysm.rhs
    for spec in args.shape:
        f = spec.split(":")
        s.set_launch_shape(int(f[0]), f[1], int(f[2]), int(f[3]), bool(int(f[4])) if len(f) > 4 else False)
    i0 = s.level_info(0)
    print(f"level 0: lanes {i0.lanes_A}/{i0.lanes_gs}, entries per trip {i0.trip_A}/{i0.trip_gs}, "
          f"per-XCD rows {i0.gs_xcd}, FP64 kernels lanes {i0.lanes64_A} entries per trip {i0.trip64_A}",
          file=sys.stderr, flush=True)
    b = torch.from_numpy(rhs).to(dev)
    x = torch.zeros_like(b)
    src = torch.ones(args.copy_mib * 2**20 // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    rt = _roctx()
    if rt is not None:
        rt.roctxProfilerResume(0)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"calibration copy: 3 x {args.copy_mib} MiB read + written", file=sys.stderr, flush=True)
    time.sleep(0.01)  # an idle gap between the copies and the solve phase
    for _ in range(args.solves):
        x.zero_()
        t0 = time.perf_counter()
        r = s.solve(b, x, tol=1e-8)
        torch.cuda.synchronize()
        its = max(q.iters for q in r) if isinstance(r, list) else r.iters
        print(f"{wl} {prec}/{kry}: {its} iterations, {1e3 * (time.perf_counter() - t0):.1f} ms",
              file=sys.stderr, flush=True)
    if rt is not None:
        rt.roctxProfilerPause(0)
    s.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
