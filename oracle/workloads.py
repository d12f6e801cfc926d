"""The oracle's own systems for the synthetic workloads (test infrastructure only).

Random data comes from ``synth`` (seeded draws only); everything else (mesh,
assembly, boundary conditions) is the oracle's.
"""
from __future__ import annotations

import synth

from . import fem


def laplace(n: int, workload: int = synth.LAPLACE_SMALL, i: int = 0) -> fem.SPDSystem:
    return fem.laplace_trig(n, synth.trig_dirichlet(workload, i))


def elasticity(n: int, i: int = 0, E: float = 1.0, nu: float = 0.3,
               workload: int = synth.ELASTICITY) -> fem.SPDSystem:
    lam, mu = fem.lame_from(E, nu)
    return fem.elasticity_traction(n, lam, mu, synth.face_traction(workload, i, n))


def mixed_elasticity(n: int, i: int = 0, E: float = 1.0, nu: float = 0.49999,
                     workload: int = synth.MIXED_ELAST) -> fem.SaddleSystem:
    lam, mu = fem.lame_from(E, nu)
    return fem.mixed_elasticity_traction(n, lam, mu, synth.face_traction(workload, i, n))


def stokes(n: int, speed: float, mu: float = 0.5) -> fem.SaddleSystem:
    return fem.stokes_lid(n, speed, mu)
