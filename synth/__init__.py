"""Seeded synthetic inputs shared by the oracle and the GPU harness.

This module draws random numbers and defines the synthetic boundary data of
the workloads. It holds none of the multigrid method's arithmetic and none of
the finite element assembly: each side (the oracle under ``oracle/`` and the
harness in the package) turns these draws into a linear system on its own.

Every stream is seeded with ``numpy.random.SeedSequence([workload_id, i])``
so that both sides see identical numbers.

Workloads (unit cube, n^3 cubes each split into 6 Kuhn tetrahedra, hierarchical
quadratic elements as in the paper's Section 2.3):

* ``LAPLACE_SMALL``  vector Laplacian, n=4, Dirichlet data on x=0.
* ``ELASTICITY``     pure-displacement elasticity, n=32, E=1, nu=0.3, clamped
                     x=0, piecewise-constant random traction on x=1.
* ``MIXED_ELAST``    mixed displacement-pressure elasticity, n=24, nu=0.49999,
                     same boundary data recipe as ``ELASTICITY``.
* ``STOKES_BATCH``   64 lid-driven Stokes cavities, n ~ U{8..20}, lid speed
                     ~ U[0.5, 2], mu = 0.5.
* ``LAPLACE_LARGE``  vector Laplacian, n=48, 256 Dirichlet data sets.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

LAPLACE_SMALL = 0
ELASTICITY = 1
MIXED_ELAST = 2
STOKES_BATCH = 3
LAPLACE_LARGE = 4
LAPLACE_TRAIN = 5   # training solves for the damping model (disjoint seeds)


def rng(workload: int, i: int) -> np.random.Generator:
    """Generator for draw ``i`` of ``workload``."""
    return np.random.default_rng(np.random.SeedSequence([int(workload), int(i)]))


# --------------------------------------------------------------------------
# Dirichlet data for the vector Laplacian: a trigonometric polynomial in (y, z)
#   g_c(y, z) = sum_{k,l=0..2} a_ckl cos(pi k y + phi_ckl) cos(pi l z + psi_ckl)
# with a ~ N(0,1) normalised per component so that sum |a_c..| = 1 (|g| <= 1).
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class TrigData:
    a: np.ndarray     # (3, 3, 3) amplitudes, [component, k, l]
    phi: np.ndarray   # (3, 3, 3) phases in y
    psi: np.ndarray   # (3, 3, 3) phases in z

    def __call__(self, y: np.ndarray, z: np.ndarray) -> np.ndarray:
        """Evaluate g at points (y, z); returns shape (len(y), 3)."""
        y = np.asarray(y, dtype=np.float64)[:, None, None, None]
        z = np.asarray(z, dtype=np.float64)[:, None, None, None]
        k = np.arange(3, dtype=np.float64)[None, None, :, None]
        l = np.arange(3, dtype=np.float64)[None, None, None, :]
        terms = (self.a[None] * np.cos(math.pi * k * y + self.phi[None])
                 * np.cos(math.pi * l * z + self.psi[None]))
        return terms.sum(axis=(2, 3))


def trig_dirichlet(workload: int, i: int) -> TrigData:
    g = rng(workload, i)
    a = g.standard_normal((3, 3, 3))
    a /= np.abs(a).sum(axis=(1, 2), keepdims=True)
    phi = g.uniform(0.0, 2.0 * math.pi, (3, 3, 3))
    psi = g.uniform(0.0, 2.0 * math.pi, (3, 3, 3))
    return TrigData(a, phi, psi)


# --------------------------------------------------------------------------
# Random traction on the face x=1. The face is split into n*n squares
# (j, k) (y index j, z index k); each square into two triangles:
#   t=0: (y_j,z_k), (y_j+1,z_k), (y_j+1,z_k+1)
#   t=1: (y_j,z_k), (y_j,z_k+1), (y_j+1,z_k+1)
# Each triangle carries a constant traction vector with i.i.d. N(0, sigma).
# --------------------------------------------------------------------------
def face_traction(workload: int, i: int, n: int, sigma: float = 0.1) -> np.ndarray:
    """Traction per boundary triangle of x=1, shape (n, n, 2, 3) = [j, k, t, comp]."""
    return rng(workload, i).normal(0.0, sigma, (n, n, 2, 3))


def lame(E: float, nu: float) -> tuple[float, float]:
    """Lame constants (lambda, mu) for Young's modulus E and Poisson ratio nu."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


# --------------------------------------------------------------------------
# Lid-driven Stokes batch: instance sizes and lid speeds.
# --------------------------------------------------------------------------
def stokes_batch(count: int = 64, nmin: int = 8, nmax: int = 20) -> list[tuple[int, float]]:
    g = rng(STOKES_BATCH, 0)
    ns = g.integers(nmin, nmax + 1, count)
    speeds = g.uniform(0.5, 2.0, count)
    return [(int(n), float(s)) for n, s in zip(ns, speeds)]


def training_sizes(count: int, nmin: int = 16, nmax: int = 32) -> list[int]:
    g = rng(LAPLACE_TRAIN, 10**6)
    return [int(v) for v in g.integers(nmin, nmax + 1, count)]


# --------------------------------------------------------------------------
# Damping-weight network: initial parameters and random test batches.
# Layer shapes 8 -> 32 -> 32 -> 1 in the flat order W1 (32x8), b1, W2 (32x32),
# b2, W3 (32), b3; weights uniform in +-sqrt(6 / (fan_in + fan_out)), biases 0.
# --------------------------------------------------------------------------
MLP_LAYERS = ((8, 32), (32, 32), (32, 1))


def mlp_init(seed: int = 0) -> np.ndarray:
    g = rng(LAPLACE_TRAIN, 2 * 10**6 + seed)
    parts = []
    for fan_in, fan_out in MLP_LAYERS:
        a = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(g.uniform(-a, a, fan_in * fan_out))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)


def mlp_batch(n: int, seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """n random feature rows (uniform in [0, 1.5)) and targets in [0.3, 1.1)."""
    g = rng(LAPLACE_TRAIN, 3 * 10**6 + seed)
    return g.uniform(0.0, 1.5, (n, 8)), g.uniform(0.3, 1.1, n)


WORKLOADS = {
    LAPLACE_SMALL: dict(name="vector-laplacian-4x4x4", n=4),
    ELASTICITY: dict(name="elasticity-32x32x32", n=32, E=1.0, nu=0.3, sigma=0.1),
    MIXED_ELAST: dict(name="mixed-elasticity-24x24x24", n=24, E=1.0, nu=0.49999, sigma=0.1),
    STOKES_BATCH: dict(name="stokes-lid-batch-64", count=64, nmin=8, nmax=20, mu=0.5),
    LAPLACE_LARGE: dict(name="vector-laplacian-48x48x48", n=48, nrhs=256),
}
