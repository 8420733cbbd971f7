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

NPT (§5.5: a Monte Carlo barostat combined with the Langevin integrator,
batched systems with independent cells and seeds; reading of the standard
MC barostat): after a step that brings a structure's own step count
(step0_s + steps taken) to a multiple of `interval`, the structure s with
periodic box lengths L_s (volume V = L_x L_y L_z) proposes a volume move,
  u_0, u_1 = rng.barostat_uniforms(seed_s, move_s)
  dV = (2 u_0 - 1) dV_max,  V' = V + dV,  lambda = (V'/V)^(1/3)
  (dV_max = f V_0, fixed from the volume V_0 when the barostat starts, so that
  the proposal is symmetric; V' <= 0 is rejected)
  trial: L' = lambda L, x' = lambda x for the structure's atoms (velocities kept)
  w = E(x', L') - E(x, L) + P dV - N_s kB T ln(V'/V)
  accept when w <= 0 or u_1 < exp(-w / kB T), else restore; move_s += 1
with P in bar converted by 1 bar = 6.241509074e-7 eV/A^3. Pinned by
tests: an ideal gas (E = 0) samples <V> = (N + 1) kB T / P.
"""
from typing import Callable, List, Sequence, Tuple

import numpy as np

from . import rng

ACCEL_UNIT = 0.009648533
KB_EV = 8.617333262e-5
BAR_EV_A3 = 6.241509074e-7


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


def barostat_move(energy_fn: Callable[[np.ndarray, np.ndarray], np.ndarray], x: np.ndarray, boxes: np.ndarray,
                  E_old: np.ndarray, offsets: Sequence[int], temperature: float, pressure_bar: float,
                  dv_max: Sequence[float], seeds: Sequence[int], moves: Sequence[int], active=None):
    """One volume proposal per active structure (all at once, each decided
    alone; inactive ones are left as they are). energy_fn(x, boxes) -> E_s.
    Returns x, boxes, E_s and the accepted flags."""
    kT = KB_EV * temperature
    P = pressure_bar * BAR_EV_A3
    S = len(offsets) - 1
    lam = np.ones(S)
    dV = np.zeros(S)
    ratio = np.ones(S)
    u1 = np.zeros(S)
    active = np.ones(S, dtype=bool) if active is None else np.asarray(active, dtype=bool)
    for s in range(S):
        if not active[s]:
            continue
        a, b = rng.barostat_uniforms(int(seeds[s]), int(moves[s]))
        V = float(np.prod(boxes[s]))
        dV[s] = (2.0 * a - 1.0) * float(dv_max[s])
        ratio[s] = max((V + dV[s]) / V, 1e-300)
        lam[s] = ratio[s] ** (1.0 / 3.0)
        u1[s] = b
    owner = np.repeat(np.arange(S), np.diff(np.asarray(offsets)))
    x_t = x * lam[owner][:, None]
    boxes_t = boxes * lam[:, None]
    E_t = np.asarray(energy_fn(x_t, boxes_t))
    acc = np.zeros(S, dtype=bool)
    for s in range(S):
        n_s = int(offsets[s + 1] - offsets[s])
        if active[s] and float(np.prod(boxes[s])) + dV[s] > 0.0:
            w = float(E_t[s] - E_old[s]) + P * dV[s] - n_s * kT * np.log(ratio[s])
            acc[s] = w <= 0.0 or u1[s] < np.exp(-w / kT)
    keep = acc[owner]
    x_new = np.where(keep[:, None], x_t, x)
    boxes_new = np.where(acc[:, None], boxes_t, boxes)
    E_new = np.where(acc, E_t, E_old)
    return x_new, boxes_new, E_new, acc


def langevin_npt(force_fn: Callable[[np.ndarray, np.ndarray], Tuple[np.ndarray, np.ndarray]],
                 x: np.ndarray, v: np.ndarray, boxes: np.ndarray, masses: np.ndarray, dt: float, n_steps: int,
                 temperature: float, gamma: float, offsets: Sequence[int], seeds: Sequence[int],
                 step0: Sequence[int], pressure_bar: float, interval: int, fraction: float,
                 baro_seeds: Sequence[int], move0: Sequence[int]):
    """BAOAB steps with volume proposals on each structure's own schedule.
    force_fn(x, boxes) -> (E_s, F). Returns x, v, boxes, E_s after every step and
    the (structure, accepted) pairs of every proposal, in order."""
    x = np.array(x, dtype=np.float64)
    boxes = np.array(boxes, dtype=np.float64)
    moves = np.array(move0, dtype=np.int64)
    dv_max = fraction * np.prod(boxes, axis=1)
    decisions = []
    energies = []
    E, _ = force_fn(x, boxes)
    for k in range(n_steps):
        x, v, Es = langevin_baoab(lambda xx: force_fn(xx, boxes), x, v, masses, dt, 1, temperature, gamma, offsets,
                                  seeds, [int(s0) + k for s0 in step0])
        E = Es[-1]
        active = np.array([(int(s0) + k + 1) % interval == 0 for s0 in step0])
        if active.any():
            x, boxes, E, acc = barostat_move(lambda xx, bb: force_fn(xx, bb)[0], x, boxes, E, offsets, temperature,
                                             pressure_bar, dv_max, baro_seeds, moves, active)
            for s in np.nonzero(active)[0]:
                decisions.append((int(s), bool(acc[s])))
            moves += active
        energies.append(np.asarray(E))
    return x, v, boxes, energies, decisions
