"""Velocity-Verlet NVE molecular dynamics (oracle).

§1 of the paper lists batched MD among the library's workloads, and the
Appendix H timing table measures ms per MD step. The integrator (reading):

  v <- v + dt/2 * kappa F(x)/m
  x <- x + dt v
  v <- v + dt/2 * kappa F(x)/m

with kappa = 0.009648533 (angstrom/fs^2 per (eV/angstrom)/amu), dt in fs,
masses in amu, FP64 state. The neighbour list is recomputed by brute force
at every force evaluation, so no skin is involved.

Pinned by tests: against the exact solution of a harmonic oscillator,
time reversibility and momentum conservation.
"""
from typing import Callable, List, Tuple

import numpy as np

ACCEL_UNIT = 0.009648533


def velocity_verlet(force_fn: Callable[[np.ndarray], Tuple[np.ndarray, np.ndarray]],
                    x: np.ndarray, v: np.ndarray, masses: np.ndarray, dt: float,
                    n_steps: int) -> Tuple[np.ndarray, np.ndarray, List[np.ndarray]]:
    """force_fn(x) -> (E_s, F). Returns final x, v and E_s after every step."""
    x = np.array(x, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    inv_m = (ACCEL_UNIT / np.asarray(masses, dtype=np.float64))[:, None]
    _, F = force_fn(x)
    energies = []
    for _ in range(n_steps):
        v = v + 0.5 * dt * F * inv_m
        x = x + dt * v
        E, F = force_fn(x)
        v = v + 0.5 * dt * F * inv_m
        energies.append(np.asarray(E))
    return x, v, energies


def kinetic_energy(v: np.ndarray, masses: np.ndarray) -> float:
    """sum 1/2 m v^2 in eV."""
    return float(0.5 * np.sum(np.asarray(masses)[:, None] * v * v) / ACCEL_UNIT)
