"""A short, fixed run for hardware-counter profiles (rocprofv3 --pmc).

First a plain device-to-device copy of a known size (the calibration for the
HBM traffic counters), then amg_setup and a few solves of one workload.

    python -m paper_1503_01287_amd.profile_run --workload elasticity-32 --precision MIXED --solves 1
"""
from __future__ import annotations

import argparse
import sys
import time


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="elasticity-32",
                    choices=["elasticity-32", "mixed-elasticity-24", "laplace-48"])
    ap.add_argument("--precision", default="MIXED", choices=["FP64", "MIXED", "FP32"])
    ap.add_argument("--solves", type=int, default=1)
    ap.add_argument("--copy-mib", type=int, default=256)
    args = ap.parse_args()

    import torch
    from . import problems, AMGSolver
    dev = torch.device("cuda:0")
    src = torch.ones(args.copy_mib * 2**20 // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"calibration copy: 3 x {args.copy_mib} MiB read + written", file=sys.stderr, flush=True)

    if args.workload == "elasticity-32":
        sysm, kw = problems.elasticity(32), dict(smoother="GS-1-1")
    elif args.workload == "laplace-48":
        import synth
        sysm, kw = problems.laplace(48, workload=synth.LAPLACE_LARGE, i=0), dict(smoother="JA-1-1-0.5")
    else:
        sysm, kw = problems.mixed_elasticity(24), dict(smoother="sGS-1-1")
    saddle = sysm.n_pres > 0
    prec = "FP64" if saddle else args.precision
    kry = "FGMRES" if saddle else ("PCG" if prec == "FP64" else "FCG")
    s = AMGSolver(sysm, krylov=kry, precision=prec, **kw)
    i0 = s.level_info(0)
    print(f"level 0: lanes {i0.lanes_A}/{i0.lanes_gs}, two entries per trip {i0.pair_A}/{i0.pair_gs}, "
          f"per-XCD rows {i0.gs_xcd}", file=sys.stderr, flush=True)
    b = torch.from_numpy(sysm.rhs).to(dev)
    x = torch.zeros_like(b)
    for _ in range(args.solves):
        x.zero_()
        t0 = time.perf_counter()
        r = s.solve(b, x, tol=1e-8)
        torch.cuda.synchronize()
        print(f"{args.workload} {prec}/{kry}: {r.iters} iterations, {1e3 * (time.perf_counter() - t0):.1f} ms",
              file=sys.stderr, flush=True)
    s.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
