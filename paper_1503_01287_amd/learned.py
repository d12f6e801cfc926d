"""Learned per-level damping of the Jacobi smoother: binding of the network
calls of libamgp2 (amg_mlp_*, amg_level_features) and the procedure that
produces its training data from the method's own solves.

Training data: for each training system (vector Laplacian, n^3 Kuhn cubes,
n in [16, 32], trigonometric Dirichlet data) and each non-coarsest level l,
the damping of level l is swept over a grid with the other levels at their
current best, and the mean convergence factor of JA-1-1 V-cycle PCG (the
geometric mean residual reduction per iteration to 1e-8) is recorded. The
grid runs from 0.3 to 1.8 and stops at the level's bound
0.95 * 2 / lambda_max(D^{-1} A_l) (amg_level_info.omega_max), above which
the symmetric cycle need not be positive definite. The target for level l
is the minimiser of a parabola through the best grid point and its
neighbours, kept under the bound. The network then regresses target
weights on the level's row features.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _lib as C

NF = 8
NPARAM = 1377
MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "omega_mlp.npy")


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


class DampingModel:
    """The network on the GPU (amg_mlp_handle)."""

    def __init__(self, params, stream=None):
        from .solver import _stream_handle
        p = _f32(params)
        if p.shape != (NPARAM,):
            raise ValueError(f"expected {NPARAM} parameters, got {p.shape}")
        h = ctypes.c_void_p()
        C.check(C.lib().amg_mlp_create(C._ptr(p, ctypes.c_float), _stream_handle(stream), ctypes.byref(h)),
                "amg_mlp_create")
        self.h = h

    @classmethod
    def load(cls, path: str = MODEL_PATH, stream=None) -> "DampingModel":
        return cls(np.load(path, allow_pickle=False), stream)

    def save(self, path: str = MODEL_PATH) -> None:
        np.save(path, self.params())

    def params(self) -> np.ndarray:
        out = np.zeros(NPARAM, dtype=np.float32)
        C.check(C.lib().amg_mlp_get_params(self.h, C._ptr(out, ctypes.c_float)), "amg_mlp_get_params")
        return out

    def forward(self, X) -> np.ndarray:
        X = _f32(X).reshape(-1, NF)
        out = np.zeros(X.shape[0], dtype=np.float32)
        C.check(C.lib().amg_mlp_forward(self.h, C._ptr(X, ctypes.c_float), X.shape[0],
                                        C._ptr(out, ctypes.c_float)), "amg_mlp_forward")
        return out

    def gradient(self, X, y) -> tuple[float, np.ndarray]:
        X, y = _f32(X).reshape(-1, NF), _f32(y)
        loss = np.zeros(1, dtype=np.float32)
        g = np.zeros(NPARAM, dtype=np.float32)
        C.check(C.lib().amg_mlp_gradient(self.h, C._ptr(X, ctypes.c_float), C._ptr(y, ctypes.c_float), X.shape[0],
                                         C._ptr(loss, ctypes.c_float), C._ptr(g, ctypes.c_float)),
                "amg_mlp_gradient")
        return float(loss[0]), g

    def train(self, X, y, steps: int, lr: float = 1e-2) -> np.ndarray:
        X, y = _f32(X).reshape(-1, NF), _f32(y)
        hist = np.zeros(max(1, steps), dtype=np.float32)
        C.check(C.lib().amg_mlp_train(self.h, C._ptr(X, ctypes.c_float), C._ptr(y, ctypes.c_float), X.shape[0],
                                      int(steps), float(lr), C._ptr(hist, ctypes.c_float)), "amg_mlp_train")
        return hist[:steps]

    def close(self) -> None:
        if getattr(self, "h", None):
            C.lib().amg_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- training data
OMEGA_GRID = np.round(np.arange(0.3, 1.801, 0.05), 4)


def _rate(res) -> float:
    """Mean residual reduction per iteration of a converged solve."""
    return float(res.relres) ** (1.0 / max(res.iters, 1))


def sweep_targets(system, rhs_list, omega_grid=OMEGA_GRID, rounds: int = 2, log=None):
    """Per-level target weights of one training system (see the module
    docstring). Returns (features [L x 8], targets [L], solves)."""
    import torch
    from .solver import AMGSolver
    dev = torch.device("cuda:0")
    bs = [torch.from_numpy(np.ascontiguousarray(r)).to(dev) for r in rhs_list]
    s = AMGSolver(system, smoother="JA-1-1-0.5", krylov="PCG")
    L = s.num_levels - 1
    feats = np.array([s.level_features(l) for l in range(L)])
    caps = np.array([s.level_info(l).omega_max for l in range(L)])
    omega = np.minimum(np.full(L + 1, 0.5), np.append(caps, caps[-1]))
    solves = 0

    def score(om):
        nonlocal solves
        s.set_level_omega(om)
        rates = []
        for b in bs:
            x = torch.zeros_like(b)
            r = s.solve(b, x, tol=1e-8, maxit=400)
            solves += 1
            rates.append(_rate(r) if r.converged else 1.0)
        return float(np.mean(rates))

    for _ in range(rounds):
        for l in range(L):
            grid = np.array([w for w in omega_grid if w <= caps[l]] or [caps[l]])
            vals = []
            for w in grid:
                om = omega.copy()
                om[l] = w
                if l == L - 1:
                    om[L] = w
                vals.append(score(om))
            vals = np.array(vals)
            k = int(np.argmin(vals))
            best = float(grid[k])
            if 0 < k < len(grid) - 1:
                y0, y1, y2 = vals[k - 1], vals[k], vals[k + 1]
                den = y0 - 2 * y1 + y2
                if den > 0:
                    h = grid[1] - grid[0]
                    best = float(grid[k] + 0.5 * h * (y0 - y2) / den)
            best = min(best, float(caps[l]))
            omega[l] = best
            if l == L - 1:
                omega[L] = best
            if log:
                log(f"level {l}: best omega {best:.3f} (rate {vals[k]:.4f})")
    s.close()
    return feats, omega[:L].copy(), solves


def evaluate(sizes, tol: float = 1e-8, log=None) -> list:
    """Learned per-level weights against the paper's fixed 0.5 and against
    the best single weight for every level (grid up to the smallest level
    bound, fewest iterations, ties broken by time), on vector Laplacians
    with Dirichlet data from a workload id of their own (not the training
    one); JA-1-1, FP64 PCG and the FP32/BF16 cycle in FCG; warm solves."""
    import time
    import torch
    import synth
    from . import problems
    from .solver import AMGSolver
    model = DampingModel.load()
    dev = torch.device("cuda:0")
    rows = []

    def timed(s, b, x):
        x.zero_()
        s.solve(b, x, tol=tol, maxit=500)
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.solve(b, x, tol=tol, maxit=500)
        torch.cuda.synchronize()
        return r.iters if r.converged else -1, round((time.perf_counter() - t0) * 1e3, 2)

    for n in sizes:
        sysm = problems.laplace(n, workload=synth.LAPLACE_SMALL, i=7)
        b = torch.from_numpy(sysm.rhs).to(dev)
        x = torch.zeros_like(b)
        row = {"n": n, "dofs": sysm.dofs}
        for prec, kry in (("FP64", "PCG"), ("MIXED", "FCG")):
            fixed = AMGSolver(sysm, smoother="JA-1-1-0.5", krylov=kry, precision=prec)
            row[f"fixed_{prec}"] = timed(fixed, b, x)
            top = min(fixed.level_info(l).omega_max for l in range(fixed.num_levels - 1))
            best = None
            for w in [round(0.30 + 0.05 * i, 2) for i in range(40) if 0.30 + 0.05 * i <= top + 1e-9]:
                fixed.set_level_omega([w])
                it, ms = timed(fixed, b, x)
                if it > 0 and (best is None or (it, ms) < (best[0], best[1])):
                    best = (it, ms, w)
            row[f"best_single_{prec}"] = best
            fixed.close()
            lw = AMGSolver(sysm, smoother="JA-1-1-0.5", krylov=kry, precision=prec, omega_model=model)
            row[f"learned_{prec}"] = timed(lw, b, x)
            row["learned_weights"] = [round(lw.level_info(l).omega, 3) for l in range(lw.num_levels - 1)]
            lw.close()
        if log:
            log(str(row))
        rows.append(row)
    return rows


def main() -> None:
    """Generate the training set, train the network on the GPU, save it."""
    import argparse
    import json
    import sys
    import time

    import synth
    from . import problems

    ap = argparse.ArgumentParser()
    ap.add_argument("--systems", type=int, default=8, help="training meshes (n drawn from [16, 32])")
    ap.add_argument("--rhs", type=int, default=2, help="Dirichlet data sets per mesh")
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--out", default=MODEL_PATH)
    ap.add_argument("--data-out", default=None, help="also write the training set (.npz)")
    ap.add_argument("--evaluate", type=int, nargs="*", default=None,
                    help="no training: compare the stored network with the fixed and the best single weight "
                         "on Laplacians of these sizes")
    args = ap.parse_args()

    def log(m):
        print(m, file=sys.stderr, flush=True)

    if args.evaluate is not None:
        print(json.dumps(evaluate(args.evaluate, log=log)))
        return

    sizes = sorted(set(synth.training_sizes(args.systems)))
    X, y = [], []
    total = 0
    t0 = time.time()
    for k, n in enumerate(sizes):
        sysm = problems.laplace(n, workload=synth.LAPLACE_TRAIN, i=1000 * k)
        rhs = [sysm.rhs] + [problems.laplace_rhs(sysm, synth.LAPLACE_TRAIN, 1000 * k + j)
                            for j in range(1, args.rhs)]
        f, w, s = sweep_targets(sysm, rhs, log=log)
        total += s
        log(f"n={n}: targets {np.round(w, 3).tolist()} ({s} solves, {time.time() - t0:.0f}s)")
        X.append(f)
        y.append(w)
    X = np.concatenate(X)
    y = np.concatenate(y)
    model = DampingModel(synth.mlp_init(0))
    hist = model.train(X, y, args.steps, args.lr)
    pred = model.forward(X)
    model.save(args.out)
    if args.data_out:
        np.savez(args.data_out, X=X, y=y)
    log(f"trained on {len(y)} levels from {total} solves: loss {hist[0]:.4g} -> {hist[-1]:.4g}, "
        f"max |pred - target| {np.abs(pred - y).max():.3f}")
    print(json.dumps({"solves": total, "levels": int(len(y)), "sizes": sizes, "loss_first": float(hist[0]),
                      "loss_last": float(hist[-1]), "targets": np.round(y, 4).tolist(),
                      "pred": np.round(pred, 4).tolist()}))


if __name__ == "__main__":
    main()
