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

Langevin dynamics (§5.5: the NVT integrator of the library, batched systems
with independent random seeds), BAOAB splitting (reading; Leimkuhler and
Matthews), per step of length dt with friction gamma (1/fs) and temperature T:

  B  v <- v + dt/2 * kappa F/m
  A  x <- x + dt/2 v
  O  v <- c1 v + sqrt(1 - c1^2) sqrt(kB T kappa / m) z,   c1 = exp(-gamma dt)
  A  x <- x + dt/2 v
     F <- F(x)
  B  v <- v + dt/2 * kappa F/m

with z three standard normals per atom drawn from `rng.normals3(seed of the
atom's structure, step0 + step index, index of the atom in its structure)`.
Pinned by tests: gamma = 0 reduces it to velocity Verlet; in a harmonic
well it samples the Boltzmann temperature.
"""
from typing import Callable, List, Sequence, Tuple

import numpy as np

from . import rng

ACCEL_UNIT = 0.009648533
KB_EV = 8.617333262e-5


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


def langevin_baoab(force_fn: Callable[[np.ndarray], Tuple[np.ndarray, np.ndarray]],
                   x: np.ndarray, v: np.ndarray, masses: np.ndarray, dt: float, n_steps: int,
                   temperature: float, gamma: float, offsets: Sequence[int], seeds: Sequence[int],
                   step0: Sequence[int]) -> Tuple[np.ndarray, np.ndarray, List[np.ndarray]]:
    """BAOAB Langevin steps for structures packed by `offsets` (one seed and
    step counter per structure). Returns final x, v and E_s after every step."""
    x = np.array(x, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    m = np.asarray(masses, dtype=np.float64)
    inv_m = (ACCEL_UNIT / m)[:, None]
    sigma = np.sqrt(KB_EV * temperature * ACCEL_UNIT / m)[:, None]
    c1 = np.exp(-gamma * dt)
    c2 = np.sqrt(1.0 - c1 * c1)
    offsets = np.asarray(offsets)
    _, F = force_fn(x)
    energies = []
    for k in range(n_steps):
        v = v + 0.5 * dt * F * inv_m
        x = x + 0.5 * dt * v
        z = np.zeros_like(v)
        for s in range(len(offsets) - 1):
            for a in range(offsets[s], offsets[s + 1]):
                z[a] = rng.normals3(int(seeds[s]), int(step0[s]) + k, a - int(offsets[s]))
        v = c1 * v + c2 * sigma * z
        x = x + 0.5 * dt * v
        E, F = force_fn(x)
        v = v + 0.5 * dt * F * inv_m
        energies.append(np.asarray(E))
    return x, v, energies
