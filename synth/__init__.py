"""Seeded synthetic inputs: structures, model weights, initial velocities.

This module is shared by the CPU oracle, the tests and the benchmark. It holds
no arithmetic of the interaction itself: it only draws random numbers and lays
them out as structures (positions, species, cells), model weights and
Maxwell-Boltzmann velocities. Everything is derived from one master seed so
that every run of every consumer sees the same inputs.

Units: angstrom, eV, fs, amu.
"""
from __future__ import annotations

import dataclasses
import json
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

MASTER_SEED = 20260522

# Boltzmann constant (eV/K) and the conversion factor that turns
# (eV/angstrom)/amu into angstrom/fs^2.
KB_EV = 8.617333262e-5
ACCEL_UNIT = 0.009648533

# Masses (amu) of the synthetic species 0..4 (H, C, N, O, S).
SPECIES_MASS = np.array([1.008, 12.011, 14.007, 15.999, 32.06])


def seed_for(*keys: int) -> np.random.Generator:
    """A generator for one named stream below the master seed."""
    return np.random.default_rng(np.random.SeedSequence([MASTER_SEED, *keys]))


# ---------------------------------------------------------------------------
# Model configuration
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class ModelConfig:
    """Shape of the equivariant interaction model.

    lmax          highest rotation order of features and harmonics
    channels      feature channels C per (l, m)
    layers        interaction layers T
    n_basis       radial Bessel functions
    cutoff        radial cutoff r_c (angstrom)
    envelope_p    exponent p of the polynomial cutoff envelope
    radial_hidden width of the two hidden layers of the radial MLP
    n_species     number of chemical species
    readout_hidden width of the hidden layer of the energy readout
    avg_neighbors normalisation constant nu of the neighbour sum
    coulomb       add the charge head and the soft-core Coulomb energy (open
                  structures only)
    soft_core_r0  radius below which the Coulomb distance is regularised (angstrom)
    correlation   1: the channel mix feeds the gate directly; 2: a MACE-style
                  product block (symmetric contraction of body order 2) sits
                  between the channel mix and the gate in every layer
    """
    lmax: int
    channels: int
    layers: int
    n_species: int
    cutoff: float
    avg_neighbors: float
    n_basis: int = 8
    envelope_p: int = 6
    radial_hidden: int = 64
    readout_hidden: int = 16
    coulomb: bool = False
    soft_core_r0: float = 2.0
    correlation: int = 1

    def to_json(self) -> str:
        return json.dumps(dataclasses.asdict(self), sort_keys=True)

    @staticmethod
    def from_json(text: str) -> "ModelConfig":
        return ModelConfig(**json.loads(text))


def nominal_neighbors(density: float, cutoff: float) -> float:
    """Expected neighbour count of an ideal gas at this density."""
    return density * 4.0 / 3.0 * math.pi * cutoff ** 3


def layer_input_orders(cfg: ModelConfig, t: int) -> List[int]:
    """Rotation orders present in the input features of layer t (1-based):
    the embedding is scalar only, later layers carry every l <= lmax."""
    return [0] if t == 1 else list(range(cfg.lmax + 1))


def path_counts(cfg: ModelConfig, t: int) -> List[int]:
    """Number of (l1, l2, l3) couplings of layer t for each output order l3.

    This only fixes the *shapes* of the weight tensors: l1 runs over the
    layer's input orders, l2 and l3 over 0..lmax, with the triangle rule and
    an even l1+l2+l3 (natural parity).
    """
    counts = [0] * (cfg.lmax + 1)
    for l3 in range(cfg.lmax + 1):
        for l1 in layer_input_orders(cfg, t):
            for l2 in range(cfg.lmax + 1):
                if abs(l1 - l2) <= l3 <= l1 + l2 and (l1 + l2 + l3) % 2 == 0:
                    counts[l3] += 1
    return counts


def product_out_order(cfg: ModelConfig, t: int) -> int:
    """Highest output order of layer t's product block (the last layer only
    needs scalars)."""
    return 0 if t == cfg.layers else cfg.lmax


def product_pairs(cfg: ModelConfig, lout: int) -> List[Tuple[int, int, int]]:
    """(l1, l2, L) couplings of two features of orders l1 <= l2 <= lmax into
    order L <= lout (triangle rule, even l1 + l2 + L), ordered by (L, l1, l2).
    Only fixes weight shapes and their order."""
    out = []
    for L in range(lout + 1):
        for l1 in range(cfg.lmax + 1):
            for l2 in range(l1, cfg.lmax + 1):
                if abs(l1 - l2) <= L <= l1 + l2 and (l1 + l2 + L) % 2 == 0:
                    out.append((l1, l2, L))
    return out


def weight_shapes(cfg: ModelConfig) -> List[Tuple[str, Tuple[int, ...], int]]:
    """(name, shape, fan_in) of every weight tensor, in file order.

    Layout (row-major, FP64):
      emb                 [S, C]
      per layer t = 1..T:
        rad1_t            [n_basis, H]
        rad2_t            [H, H]
        rad3_t            [H, P_t*C]      column = p*C + k, paths ordered by (l3, l1, l2)
        mix_t_l3          [P_{t,l3}*C, C] row = q*C + k, q = rank of the path among those with this l3
        self_t_l3         [C, C]          only for l3 present in the layer's input
        with correlation 2 (Lo = product_out_order, pairs = product_pairs(Lo)):
        sym1_t            [S, Lo+1, C]    per-species, per-channel weight of the linear term
        sym2_t            [S, len(pairs), C]  ... of each product coupling
        lin_t_L           [C, C]          L = 0..Lo, linear after the product block
      read1               [C, readout_hidden]
      read2               [readout_hidden, 1]
      e0                  [S]             per-species reference energy (zeros)
      qhead               [C]             charge head (only with coulomb)
      qbias               [S]             per-species charge offset (only with coulomb)
    """
    C, H = cfg.channels, cfg.radial_hidden
    out: List[Tuple[str, Tuple[int, ...], int]] = [("emb", (cfg.n_species, C), cfg.n_species)]
    for t in range(1, cfg.layers + 1):
        pc = path_counts(cfg, t)
        out.append((f"rad1_{t}", (cfg.n_basis, H), cfg.n_basis))
        out.append((f"rad2_{t}", (H, H), H))
        out.append((f"rad3_{t}", (H, sum(pc) * C), H))
        for l3 in range(cfg.lmax + 1):
            out.append((f"mix_{t}_{l3}", (pc[l3] * C, C), pc[l3] * C))
        for l3 in layer_input_orders(cfg, t):
            out.append((f"self_{t}_{l3}", (C, C), C))
        if cfg.correlation == 2:
            lo = product_out_order(cfg, t)
            npair = len(product_pairs(cfg, lo))
            out.append((f"sym1_{t}", (cfg.n_species, lo + 1, C), 2))
            out.append((f"sym2_{t}", (cfg.n_species, npair, C), npair))
            for L in range(lo + 1):
                out.append((f"lin_{t}_{L}", (C, C), C))
    out.append(("read1", (C, cfg.readout_hidden), C))
    out.append(("read2", (cfg.readout_hidden, 1), cfg.readout_hidden))
    out.append(("e0", (cfg.n_species,), 0))
    if cfg.coulomb:
        # fan-in scaled by 10: partial charges of a few tenths of e
        out.append(("qhead", (C,), 10 * C))
        out.append(("qbias", (cfg.n_species,), 10 * cfg.n_species))
    return out


def model_weights(cfg: ModelConfig, seed_key: int) -> Dict[str, np.ndarray]:
    """Gaussian weights with std 1/sqrt(fan_in), FP64, seeded; e0 = 0."""
    rng = seed_for(seed_key, 1)
    out: Dict[str, np.ndarray] = {}
    for name, shape, fan_in in weight_shapes(cfg):
        if fan_in == 0:
            out[name] = np.zeros(shape)
        else:
            out[name] = rng.standard_normal(shape) / math.sqrt(fan_in)
    return out


def flatten_weights(cfg: ModelConfig, w: Dict[str, np.ndarray]) -> np.ndarray:
    """Concatenate the weights in file order into one contiguous FP64 vector."""
    parts = []
    for name, shape, _ in weight_shapes(cfg):
        a = np.asarray(w[name], dtype=np.float64)
        assert a.shape == shape, (name, a.shape, shape)
        parts.append(a.reshape(-1))
    return np.ascontiguousarray(np.concatenate(parts))


# ---------------------------------------------------------------------------
# Structures
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Batch:
    """S structures packed along the atom axis.

    pos      [N, 3] FP64     positions
    species  [N]    int32    species index 0..n_species-1
    cell     [S, 3, 3] FP64  rows are the lattice vectors (orthorhombic here)
    pbc      [S, 3] uint8    periodic flags per axis
    offsets  [S+1]  int64    structure s owns atoms offsets[s]:offsets[s+1]
    charge   [S]    FP64     total charge of each structure (None: 0)
    """
    pos: np.ndarray
    species: np.ndarray
    cell: np.ndarray
    pbc: np.ndarray
    offsets: np.ndarray
    charge: Optional[np.ndarray] = None

    def total_charge(self) -> np.ndarray:
        return np.zeros(self.n_structures) if self.charge is None else np.asarray(self.charge, dtype=np.float64)

    @property
    def n_atoms(self) -> int:
        return int(self.offsets[-1])

    @property
    def n_structures(self) -> int:
        return len(self.offsets) - 1

    def structure(self, s: int) -> "Batch":
        a, b = int(self.offsets[s]), int(self.offsets[s + 1])
        return Batch(self.pos[a:b].copy(), self.species[a:b].copy(), self.cell[s:s + 1].copy(),
                     self.pbc[s:s + 1].copy(), np.array([0, b - a], dtype=np.int64),
                     None if self.charge is None else np.asarray(self.charge)[s:s + 1].copy())


def concat(batches: Sequence[Batch]) -> Batch:
    sizes = [b.n_atoms for b in batches]
    return Batch(np.concatenate([b.pos for b in batches]).astype(np.float64),
                 np.concatenate([b.species for b in batches]).astype(np.int32),
                 np.concatenate([b.cell for b in batches]).astype(np.float64),
                 np.concatenate([b.pbc for b in batches]).astype(np.uint8),
                 np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64),
                 None if all(b.charge is None for b in batches)
                 else np.concatenate([b.total_charge() for b in batches]))


def uniform_cluster(n: int, box: float, d_min: float, n_species: int,
                    rng: np.random.Generator) -> Batch:
    """n atoms uniform in a non-periodic cube of side `box`, no pair closer
    than d_min (rejection sampling, one atom at a time)."""
    pos = np.zeros((n, 3))
    k = 0
    tries = 0
    while k < n:
        tries += 1
        if tries > 1000000:
            raise RuntimeError("rejection sampling did not converge")
        p = rng.uniform(0.0, box, size=3)
        if k and np.min(np.linalg.norm(pos[:k] - p, axis=1)) < d_min:
            continue
        pos[k] = p
        k += 1
    species = rng.integers(0, n_species, size=n).astype(np.int32)
    return Batch(pos, species, (np.eye(3) * box)[None], np.zeros((1, 3), np.uint8),
                 np.array([0, n], dtype=np.int64))


def jittered_lattice(n: int, density: float, sigma: float, n_species: int,
                     rng: np.random.Generator, periodic: bool = True) -> Batch:
    """Liquid-like periodic cube: n of the m^3 simple-cubic sites
    (m = ceil(n^(1/3))) chosen without replacement, Gaussian jitter of
    std sigma per coordinate, wrapped into [0, L).

    Atoms are emitted in lattice (raster) order of their sites.
    With periodic=False the same recipe gives an open cluster (no wrap).
    """
    L = (n / density) ** (1.0 / 3.0)
    m = int(math.ceil(round(n ** (1.0 / 3.0), 9)))
    a = L / m
    sites = np.sort(rng.choice(m ** 3, size=n, replace=False))
    ijk = np.stack([sites // (m * m), (sites // m) % m, sites % m], axis=1).astype(np.float64)
    pos = (ijk + 0.5) * a + rng.normal(0.0, sigma, size=(n, 3))
    if periodic:
        pos = pos - np.floor(pos / L) * L
    species = rng.integers(0, n_species, size=n).astype(np.int32)
    pbc = np.ones((1, 3), np.uint8) if periodic else np.zeros((1, 3), np.uint8)
    return Batch(pos, species, (np.eye(3) * L)[None], pbc, np.array([0, n], dtype=np.int64))


def maxwell_boltzmann(batch: Batch, temperature: float, rng: np.random.Generator) -> np.ndarray:
    """Velocities (angstrom/fs) with each component ~ N(0, kB*T*kappa/m),
    centre-of-mass velocity removed per structure."""
    m = SPECIES_MASS[batch.species]
    v = rng.standard_normal((batch.n_atoms, 3)) * np.sqrt(KB_EV * temperature * ACCEL_UNIT / m)[:, None]
    for s in range(batch.n_structures):
        a, b = int(batch.offsets[s]), int(batch.offsets[s + 1])
        ms = m[a:b, None]
        v[a:b] -= (ms * v[a:b]).sum(0) / ms.sum()
    return v


# ---------------------------------------------------------------------------
# The workloads
# ---------------------------------------------------------------------------

DENSITY = 0.1  # atoms / angstrom^3


def tiny_config() -> Tuple[ModelConfig, Batch]:
    """24 atoms uniform in a 10 A open cube (d_min 0.9 A), 3 species,
    r_c 5 A, l_max 2, 32 channels, 2 layers."""
    rng = seed_for(1)
    b = uniform_cluster(24, 10.0, 0.9, 3, rng)
    cfg = ModelConfig(lmax=2, channels=32, layers=2, n_species=3, cutoff=5.0,
                      avg_neighbors=nominal_neighbors(24 / 1000.0, 5.0))
    return cfg, b


def single_config(n: int = 3000, channels: int = 128, layers: int = 2,
                  cutoff: float = 5.0, seed_key: int = 2) -> Tuple[ModelConfig, Batch]:
    """Liquid-like periodic box at 0.1 atoms/A^3 (jittered lattice, 0.3 A
    noise), 4 species, l_max 3, 128 channels, 2 layers, r_c 5 A."""
    rng = seed_for(seed_key)
    b = jittered_lattice(n, DENSITY, 0.3, 4, rng)
    cfg = ModelConfig(lmax=3, channels=channels, layers=layers, n_species=4, cutoff=cutoff,
                      avg_neighbors=nominal_neighbors(DENSITY, cutoff))
    return cfg, b


def differentiation_config(n_structures: int = 64, lo: int = 20, hi: int = 200
                           ) -> Tuple[ModelConfig, Batch, np.ndarray, np.ndarray]:
    """Batch of periodic boxes, atom counts uniform in [lo, hi], 5 species,
    l_max 3, 64 channels, 2 layers; seeded N(0,1) energy and force targets."""
    rng = seed_for(3)
    sizes = rng.integers(lo, hi + 1, size=n_structures)
    batch = concat([jittered_lattice(int(n), DENSITY, 0.3, 5, rng) for n in sizes])
    cfg = ModelConfig(lmax=3, channels=64, layers=2, n_species=5, cutoff=5.0,
                      avg_neighbors=nominal_neighbors(DENSITY, 5.0))
    e_ref = rng.standard_normal(n_structures)
    f_ref = rng.standard_normal((batch.n_atoms, 3))
    return cfg, batch, e_ref, f_ref


def serving_model() -> ModelConfig:
    return ModelConfig(lmax=3, channels=128, layers=2, n_species=4, cutoff=5.0,
                       avg_neighbors=nominal_neighbors(DENSITY, 5.0))


def serving_requests(n_requests: int, rate_per_s: float, lo: int = 50, hi: int = 5000,
                     seed_key: int = 4) -> List[Tuple[float, Batch, np.ndarray]]:
    """Poisson stream of MD requests: (arrival time s, structure, velocities at 300 K).
    Atom counts are log-uniform in [lo, hi]."""
    rng = seed_for(seed_key)
    t = 0.0
    out = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        rr = seed_for(seed_key, 100 + r)
        b = jittered_lattice(n, DENSITY, 0.3, 4, rr)
        v = maxwell_boltzmann(b, 300.0, rr)
        out.append((t, b, v))
    return out


def open_box(n: int, n_species: int, rng: np.random.Generator) -> Batch:
    """A liquid-density (0.1 atoms/A^3) jittered lattice with every axis open:
    a compact cluster cut from the liquid."""
    b = jittered_lattice(n, DENSITY, 0.3, n_species, rng)
    b.pbc[:] = 0
    return b


def electrostatics_config(n_structures: int = 64, lo: int = 20, hi: int = 200, seed_key: int = 6
                          ) -> Tuple[ModelConfig, Batch]:
    """Batch of open clusters at 0.1 atoms/A^3, atom counts uniform in
    [lo, hi], 4 species, total charges uniform in {-1, 0, +1}; l_max 3, 128
    channels, 2 layers, r_c 5 A, Coulomb term with a 2 A soft core."""
    rng = seed_for(seed_key)
    sizes = rng.integers(lo, hi + 1, size=n_structures)
    batch = concat([open_box(int(n), 4, rng) for n in sizes])
    batch.charge = rng.integers(-1, 2, size=n_structures).astype(np.float64)
    cfg = ModelConfig(lmax=3, channels=128, layers=2, n_species=4, cutoff=5.0,
                      avg_neighbors=nominal_neighbors(DENSITY, 5.0), coulomb=True, soft_core_r0=2.0)
    return cfg, batch


def scale_config(n: int = 100000) -> Tuple[ModelConfig, Batch]:
    """Large periodic box at 0.1 atoms/A^3, r_c 6 A, l_max 3, 128 channels, 3 layers."""
    rng = seed_for(5)
    b = jittered_lattice(n, DENSITY, 0.3, 4, rng)
    cfg = ModelConfig(lmax=3, channels=128, layers=3, n_species=4, cutoff=6.0,
                      avg_neighbors=nominal_neighbors(DENSITY, 6.0))
    return cfg, b


def scale_subbox() -> Tuple[ModelConfig, Batch]:
    """Independent 2,000-atom periodic box with the large-box model."""
    rng = seed_for(5, 7)
    b = jittered_lattice(2000, DENSITY, 0.3, 4, rng)
    cfg = ModelConfig(lmax=3, channels=128, layers=3, n_species=4, cutoff=6.0,
                      avg_neighbors=nominal_neighbors(DENSITY, 6.0))
    return cfg, b


def paper_shape_cluster(n: int, seed_key: int) -> Tuple[ModelConfig, Batch]:
    """Open cluster at 0.1 atoms/A^3 with a MACE-like model shape
    (l_max 3, 128 channels, 2 layers, r_c 5 A)."""
    rng = seed_for(seed_key)
    b = jittered_lattice(n, DENSITY, 0.3, 4, rng, periodic=False)
    cfg = ModelConfig(lmax=3, channels=128, layers=2, n_species=4, cutoff=5.0,
                      avg_neighbors=nominal_neighbors(DENSITY, 5.0))
    return cfg, b
