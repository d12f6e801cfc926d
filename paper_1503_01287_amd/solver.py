"""Python handle around the C ABI: setup, solve and the introspection calls.

Vectors are torch CUDA float64 tensors; the library runs on the caller's
current torch stream unless another stream is given.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _lib as C
from .problems import LinearSystem


def parse_smoother(name: str) -> dict:
    """The paper's smoother names: 'JA-1-1-0.5', 'GS-2-2', 'sGS-1-1',
    'Braess-Sarazin-1-1' (alias 'BS-1-1'), 'Vanka-1-1' (optionally with its
    damping, 'Vanka-1-1-0.8')."""
    parts = name.split("-")
    if parts[0] == "Braess":
        parts = ["BS"] + parts[2:]
    kind = {"JA": "JA", "GS": "GS", "sGS": "SGS", "SGS": "SGS", "BS": "BS", "Vanka": "VANKA"}[parts[0]]
    out = dict(smoother=kind, pre=int(parts[1]), post=int(parts[2]))
    if kind == "JA" and len(parts) > 3:
        out["omega"] = float(parts[3])
    if kind == "VANKA" and len(parts) > 3:
        out["vanka_omega"] = float(parts[3])
    return out


@dataclass
class SolveResult:
    iters: int
    status: int
    relres: float
    solve_ms: float

    @property
    def converged(self) -> bool:
        return self.status == C.AMG_OK


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, n: int, name: str):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name}: expected a contiguous float64 CUDA tensor")
    if t.numel() != n:
        raise ValueError(f"{name}: expected {n} values, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _marshal(system: LinearSystem, keep: list, device: bool = False) -> "C.AmgSystem":
    """amg_system over host copies of the arrays, or over device copies
    (CUDA tensors, memory = AMG_MEM_DEVICE) when `device`; the copies are
    kept alive in `keep`."""
    def arr(a, dtype, ctype):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dtype)
        if device:
            import torch
            t = torch.from_numpy(a).to("cuda")
            keep.append(t)
            return ctypes.cast(ctypes.c_void_p(t.data_ptr()), ctypes.POINTER(ctype))
        keep.append(a)
        return C._ptr(a, ctype)

    s = C.AmgSystem()
    s.n_lin, s.n_quad, s.n_pres, s.bs = system.n_lin, system.n_quad, system.n_pres, system.bs
    s.A_rowptr = arr(system.A_rowptr, np.int32, ctypes.c_int32)
    s.A_col = arr(system.A_col, np.int32, ctypes.c_int32)
    s.A_val = arr(system.A_val, np.float64, ctypes.c_double)
    s.B_rowptr = arr(system.B_rowptr, np.int32, ctypes.c_int32)
    s.B_col = arr(system.B_col, np.int32, ctypes.c_int32)
    s.B_val = arr(system.B_val, np.float64, ctypes.c_double)
    s.C_rowptr = arr(system.C_rowptr, np.int32, ctypes.c_int32)
    s.C_col = arr(system.C_col, np.int32, ctypes.c_int32)
    s.C_val = arr(system.C_val, np.float64, ctypes.c_double)
    s.pressure_kernel = 1 if system.pressure_kernel else 0
    s.memory = 1 if device else 0
    return s


class AMGSolver:
    """amg_setup on construction; amg_solve / amg_precondition / ... on call."""

    def __init__(self, system: LinearSystem, smoother: str = "GS-1-1", krylov: str = "PCG",
                 precision: str = "FP64", cycles: int = 1, nu: int = 1, coarse_max: int = 300,
                 max_levels: int = 10, separate: bool = True, level_omega=None,
                 sgs_omega: float = 0.125, sgs_damping: float = 0.5, restart: int = 100,
                 omega: float | None = None, fuse_coarse: bool = True, autotune: bool = True,
                 omega_model=None, graph: bool = True, gs_post: str = "auto", stream=None,
                 device_system: bool = False):
        L = C.lib()
        p = C.default_params()
        sm = parse_smoother(smoother)
        p.gs_post = {"auto": 0, "backward": 1, "forward": 2}[gs_post]
        p.smoother = C.SMOOTH[sm["smoother"]]
        p.pre, p.post = sm["pre"], sm["post"]
        p.omega = omega if omega is not None else sm.get("omega", 0.5)
        p.sgs_omega, p.sgs_damping = sgs_omega, sgs_damping
        if "vanka_omega" in sm:
            p.vanka_omega = sm["vanka_omega"]
        p.cycles, p.nu = cycles, nu
        p.coarse_max, p.max_levels = coarse_max, max_levels
        p.separate = 1 if separate else 0
        p.krylov = C.KRYLOV[krylov]
        p.restart = restart
        p.precision = C.PREC[precision]
        p.fuse_coarse = 1 if fuse_coarse else 0
        p.autotune = 1 if autotune else 0
        if omega_model is not None:
            p.omega_model = omega_model.h
        p.graph = 1 if graph else 0
        self._omega_buf = None
        if level_omega is not None:
            self._omega_buf = np.ascontiguousarray(level_omega, dtype=np.float64)
            p.n_level_omega = self._omega_buf.shape[0]
            p.level_omega = C._ptr(self._omega_buf, ctypes.c_double)
        self.params = p
        self.system = system
        keep = []
        s = _marshal(system, keep, device=device_system)
        if device_system:
            import torch
            (torch.cuda.current_stream() if stream is None else stream).synchronize()
        self._stream = stream
        h = ctypes.c_void_p()
        C.check(L.amg_setup(ctypes.byref(s), ctypes.byref(p), _stream_handle(stream), ctypes.byref(h)),
                "amg_setup")
        self.h = h
        self.n = system.dofs

    # ---------------------------------------------------------------- calls
    def solve(self, b, x, tol: float = 1e-8, maxit: int = 500) -> SolveResult:
        r = C.AmgResult()
        code = C.lib().amg_solve(self.h, _dev_ptr(b, self.n, "b"), _dev_ptr(x, self.n, "x"), float(tol),
                                 int(maxit), _stream_handle(self._stream), ctypes.byref(r))
        C.check(code, "amg_solve")
        return SolveResult(r.iters, r.status, r.relres, r.solve_ms)

    def solve_multi(self, B, X, tol: float = 1e-8, maxit: int = 500) -> list:
        """amg_solve_multi: B, X are (k, n) contiguous float64 CUDA tensors
        (k <= 8 right-hand sides); returns one SolveResult per row."""
        k = B.shape[0] if B.dim() == 2 else 0
        if B.dim() != 2 or X.shape != B.shape or B.shape[1] != self.n:
            raise ValueError(f"expected (k, {self.n}) tensors")
        res = (C.AmgResult * k)()
        code = C.lib().amg_solve_multi(self.h, k, _dev_ptr(B, k * self.n, "B"), _dev_ptr(X, k * self.n, "X"),
                                       float(tol), int(maxit), _stream_handle(self._stream), res)
        C.check(code, "amg_solve_multi")
        return [SolveResult(r.iters, r.status, r.relres, r.solve_ms) for r in res]

    def precondition(self, r, z) -> None:
        C.check(C.lib().amg_precondition(self.h, _dev_ptr(r, self.n, "r"), _dev_ptr(z, self.n, "z"),
                                         _stream_handle(self._stream)), "amg_precondition")

    def level_dofs(self, level: int) -> int:
        i = self.level_info(level)
        return 3 * (i.n_lin + i.n_quad) + i.n_pres

    def apply(self, level: int, x, y) -> None:
        n = self.level_dofs(level)
        C.check(C.lib().amg_apply(self.h, level, _dev_ptr(x, n, "x"), _dev_ptr(y, n, "y"),
                                  _stream_handle(self._stream)), "amg_apply")

    def smooth(self, level: int, b, x, forward: bool = True) -> None:
        n = self.level_dofs(level)
        C.check(C.lib().amg_smooth(self.h, level, _dev_ptr(b, n, "b"), _dev_ptr(x, n, "x"),
                                   1 if forward else 0, _stream_handle(self._stream)), "amg_smooth")

    @property
    def num_levels(self) -> int:
        return C.check(C.lib().amg_num_levels(self.h), "amg_num_levels")

    def level_info(self, level: int) -> C.AmgLevelInfo:
        info = C.AmgLevelInfo()
        C.check(C.lib().amg_get_level_info(self.h, level, ctypes.byref(info)), "amg_get_level_info")
        return info

    def level_matrix(self, level: int, which: str = "A"):
        """(rowptr, col, val) of a level operator; val has shape (nnz, np)."""
        info = self.level_info(level)
        code = {"A": 0, "B": 1, "C": 2, "P": 3, "S": 4}[which]
        n = info.n_lin + info.n_quad
        if which == "A":
            nnz, width, nrows = info.nnz_A, info.bs * info.bs, n
        elif which == "P":
            nnz, width, nrows = info.nnz_P, 1, n
        elif which == "B":
            nnz, width, nrows = info.nnz_B, 3, info.n_pres
        elif which == "S":
            nnz, width, nrows = info.nnz_S, 1, info.n_pres
        else:
            nnz, width, nrows = info.nnz_C, 1, info.n_pres
        rowptr = np.zeros(nrows + 1, dtype=np.int32)
        col = np.zeros(max(1, nnz), dtype=np.int32)
        val = np.zeros(max(1, nnz * width), dtype=np.float64)
        C.check(C.lib().amg_get_level_matrix(self.h, level, code, C._ptr(rowptr, ctypes.c_int32),
                                             C._ptr(col, ctypes.c_int32), C._ptr(val, ctypes.c_double)),
                "amg_get_level_matrix")
        return rowptr, col[:nnz], val[: nnz * width].reshape(nnz, width)

    def set_launch_shape(self, level: int, kernels: str, lanes: int, trip: int = 1, xcd: bool = False) -> None:
        """Override the tuner's launch shape of one kernel class on a level:
        kernels 'natural', 'sweep', 'natural_rp' or 'sweep_rp'; lanes per
        row; entries per lane and loop trip (1, 2 or 4). 'vanka': the
        level's Vanka sweeps with `lanes` (16, 32, 64) lanes per residual
        row, then the corrections over 2-D tiles of the inverses (trip 1)
        or over 64-row tiles (trip 2); 'vanka_apply': the latter with
        `lanes` = 4, 8 or 16 wavefronts per tile."""
        C.check(C.lib().amg_set_launch_shape(self.h, level, C.SHAPE[kernels], int(lanes), int(trip),
                                             1 if xcd else 0), "amg_set_launch_shape")

    def set_level_omega(self, omega) -> None:
        """New JA damping per level (level l uses omega[min(l, len - 1)])."""
        w = np.ascontiguousarray(omega, dtype=np.float64)
        C.check(C.lib().amg_set_level_omega(self.h, w.size, C._ptr(w, ctypes.c_double)), "amg_set_level_omega")

    def level_features(self, level: int) -> np.ndarray:
        """The damping network's eight input features of level `level`."""
        out = np.zeros(8, dtype=np.float64)
        C.check(C.lib().amg_level_features(self.h, level, C._ptr(out, ctypes.c_double)), "amg_level_features")
        return out

    def level_features_noalloc(self, level: int, out) -> None:
        """The eight features into a device tensor of 8 float64 (stream-ordered,
        no allocation inside the library)."""
        C.check(C.lib().amg_level_features_noalloc(self.h, level, _dev_ptr(out, 8, "out"),
                                                   _stream_handle(self._stream)), "amg_level_features_noalloc")

    def level_colors(self, level: int) -> np.ndarray:
        info = self.level_info(level)
        out = np.zeros(info.n_lin + info.n_quad, dtype=np.int32)
        C.check(C.lib().amg_get_level_colors(self.h, level, C._ptr(out, ctypes.c_int32)), "amg_get_level_colors")
        return out

    def profile(self, mode: int = 1) -> None:
        """1: time every launch, 2: only the finest level's launches, 0: off."""
        C.check(C.lib().amg_profile_enable(self.h, int(mode)), "amg_profile_enable")

    def profile_read(self, cls: str) -> dict:
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        C.check(C.lib().amg_profile_read(self.h, cls.encode(), ctypes.byref(n), ctypes.byref(ms),
                                         ctypes.byref(by)), "amg_profile_read")
        return dict(launches=n.value, ms=ms.value, bytes=by.value)

    def close(self) -> None:
        if getattr(self, "h", None):
            C.lib().amg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedSolver:
    """amg_setup_batched over several saddle point systems (FGMRES) or
    several SPD systems (PCG with the FP64 cycle, FCG with a reduced-precision
    one, unless `krylov` says otherwise); vectors are the systems' [u; p]
    (SPD: u) one after another, in the order given."""

    def __init__(self, systems, smoother: str | None = None, cycles: int = 1, nu: int = 1,
                 coarse_max: int = 300, max_levels: int = 10, sgs_omega: float = 0.125,
                 sgs_damping: float = 0.5, restart: int = 100, graph: bool = True, precision: str = "FP64",
                 fuse_coarse: bool = True, autotune: bool = True, stream=None, device_system: bool = False,
                 krylov: str | None = None, omega: float | None = None):
        L = C.lib()
        p = C.default_params()
        systems = list(systems)
        spd = bool(systems) and systems[0].n_pres == 0
        sm = parse_smoother(smoother or ("GS-1-1" if spd else "BS-1-1"))
        p.smoother = C.SMOOTH[sm["smoother"]]
        p.pre, p.post = sm["pre"], sm["post"]
        p.omega = omega if omega is not None else sm.get("omega", 0.5)
        p.sgs_omega, p.sgs_damping = sgs_omega, sgs_damping
        p.cycles, p.nu = cycles, nu
        p.coarse_max, p.max_levels = coarse_max, max_levels
        p.krylov = C.KRYLOV[krylov or (("PCG" if precision == "FP64" else "FCG") if spd else "FGMRES")]
        p.restart = restart
        p.graph = 1 if graph else 0
        p.precision = C.PREC[precision]
        p.fuse_coarse = 1 if fuse_coarse else 0
        p.autotune = 1 if autotune else 0
        self.params = p
        self.systems = list(systems)
        keep = []
        arr = (C.AmgSystem * len(self.systems))()
        for i, sysm in enumerate(self.systems):
            arr[i] = _marshal(sysm, keep, device=device_system)
        if device_system:
            import torch
            torch.cuda.synchronize()
        self._stream = stream
        h = ctypes.c_void_p()
        C.check(L.amg_setup_batched(len(self.systems), arr, ctypes.byref(p), _stream_handle(stream),
                                    ctypes.byref(h)), "amg_setup_batched")
        self.h = h
        self.sizes = [s.dofs for s in self.systems]
        self.n = int(sum(self.sizes))

    def solve(self, b, x, tol: float = 1e-8, maxit: int = 500) -> list:
        res = (C.AmgResult * len(self.systems))()
        code = C.lib().amg_solve_batched(self.h, _dev_ptr(b, self.n, "b"), _dev_ptr(x, self.n, "x"), float(tol),
                                         int(maxit), _stream_handle(self._stream), res)
        C.check(code, "amg_solve_batched")
        return [SolveResult(r.iters, r.status, r.relres, r.solve_ms) for r in res]

    def offsets(self):
        """(velocity offsets, pressure offsets) of every system in the merged level-0 vector."""
        u = np.zeros(len(self.systems), dtype=np.int64)
        q = np.zeros(len(self.systems), dtype=np.int64)
        C.check(C.lib().amg_batch_offsets(self.h, u.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                          q.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), "amg_batch_offsets")
        return u, q

    def set_launch_shape(self, level: int, kernels: str, lanes: int, trip: int = 1, xcd: bool = False) -> None:
        """As AMGSolver.set_launch_shape, on a merged level of the batch."""
        C.check(C.lib().amg_set_launch_shape(self.h, level, C.SHAPE[kernels], int(lanes), int(trip),
                                             1 if xcd else 0), "amg_set_launch_shape")

    def precondition(self, r, z) -> None:
        """One preconditioner application in the merged layout."""
        C.check(C.lib().amg_precondition(self.h, _dev_ptr(r, self.n, "r"), _dev_ptr(z, self.n, "z"),
                                         _stream_handle(self._stream)), "amg_precondition")

    @property
    def num_levels(self) -> int:
        return C.check(C.lib().amg_num_levels(self.h), "amg_num_levels")

    def level_info(self, level: int):
        info = C.AmgLevelInfo()
        C.check(C.lib().amg_get_level_info(self.h, level, ctypes.byref(info)), "amg_get_level_info")
        return info

    def profile(self, mode: int = 1) -> None:
        C.check(C.lib().amg_profile_enable(self.h, int(mode)), "amg_profile_enable")

    def profile_read(self, cls: str) -> dict:
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        C.check(C.lib().amg_profile_read(self.h, cls.encode(), ctypes.byref(n), ctypes.byref(ms),
                                         ctypes.byref(by)), "amg_profile_read")
        return dict(launches=n.value, ms=ms.value, bytes=by.value)

    def close(self) -> None:
        if getattr(self, "h", None):
            C.lib().amg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

