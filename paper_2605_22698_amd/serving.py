"""Continuous-batching MD serving on one GPU.

The paper's library runs batched MD and batched inference of independent
systems on one device (§1, §5.5: batched simulations with independent cells).
This module turns that into a serving loop: requests (a structure, initial
velocities and a number of MD steps) arrive over time; while others are
running, new ones are admitted as soon as a slot and enough device memory are
free, and every engine step advances all admitted requests together in one
packed launch (structures packed along the atom axis, edges never crossing
structures). Positions, velocities, forces and neighbour lists stay on the
device; a request leaves the pack when its steps are done.

Admission is by device-memory footprint (the library's own estimate for the
packed atom and edge counts) against a budget, first come first served;
a request that could never fit alone is rejected. Every packing change
rebuilds the packed state from the device copies of the running requests,
which continue bit for bit (each structure's arithmetic does not depend on
what else is packed with it).

The executor interface (`launch`, `step`, `states`, `footprint`) is what the
scheduler needs; `GpuExecutor` implements it on the HIP library.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    """One MD job. pos/vel: host FP64 [n,3]; species int [n]; cell [3,3]; pbc [3]."""
    rid: int
    arrival: float
    pos: np.ndarray
    vel: np.ndarray
    species: np.ndarray
    cell: np.ndarray
    pbc: np.ndarray
    n_steps: int
    seed: int = 0                 # Langevin noise seed of this request (NVT only)
    # filled in by the server
    steps_done: int = 0
    admitted_at: Optional[float] = None
    finished_at: Optional[float] = None
    final_pos: Optional[np.ndarray] = None
    final_vel: Optional[np.ndarray] = None
    final_cell: Optional[np.ndarray] = None
    rejected: bool = False

    @property
    def n_atoms(self) -> int:
        return len(self.species)


class GpuExecutor:
    """Packed MD state on the GPU through the library's MD entry points."""

    def __init__(self, model, masses, cutoff: float, skin: float = 1.0, rebuild_every: int = 20,
                 dt_fs: float = 0.5, edges_per_atom: Optional[float] = None, temperature_K: float = 0.0,
                 friction_per_fs: float = 0.0, pressure_bar: Optional[float] = None, barostat_interval: int = 25,
                 volume_fraction: float = 0.01):
        import torch
        if pressure_bar is not None and not friction_per_fs > 0:
            raise ValueError("NPT (a pressure) needs the Langevin thermostat: give friction_per_fs > 0")
        self.torch = torch
        self.model = model
        self.masses = np.asarray(masses, dtype=np.float64)
        self.cutoff, self.skin, self.rebuild_every, self.dt = cutoff, skin, rebuild_every, dt_fs
        rc = cutoff + skin
        self.edges_per_atom = edges_per_atom if edges_per_atom is not None else 0.1 * 4.0 / 3.0 * math.pi * rc ** 3 * 1.3
        self.md = None
        self.slices: List[slice] = []
        # Langevin NVT when friction > 0 (each request keeps its own seed and
        # step counter across repacks, so its noise does not depend on the pack)
        self.temperature, self.friction = temperature_K, friction_per_fs
        # NPT (Monte Carlo barostat) when a pressure is given: each request
        # proposes on its own step schedule with a volume step fixed from its
        # initial volume
        self.pressure, self.baro_interval, self.volume_fraction = pressure_bar, barostat_interval, volume_fraction
        self._dev = model.device

    def footprint(self, n_atoms: int) -> int:
        return self.model.footprint_bytes(n_atoms, int(n_atoms * self.edges_per_atom))

    def launch(self, parts: Sequence[dict]) -> None:
        """New packed state from per-request dicts with device pos/vel/species and host cell/pbc."""
        import paper_2605_22698_amd as e3
        torch = self.torch
        if self.md is not None:
            self.md.close()
            self.md = None
        if not parts:
            return
        sizes = [p["pos"].shape[0] for p in parts]
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        pos = torch.cat([p["pos"] for p in parts]).contiguous()
        vel = torch.cat([p["vel"] for p in parts]).contiguous()
        sp = torch.cat([p["species"] for p in parts]).contiguous()
        cell = np.stack([p["cell"] for p in parts])
        pbc = np.stack([p["pbc"] for p in parts])
        self.md = e3.MD(self.model, off, pos, vel, sp, self.masses, cell, pbc, self.cutoff, self.skin,
                        self.rebuild_every)
        self.slices = [slice(int(off[k]), int(off[k + 1])) for k in range(len(parts))]
        if self.friction > 0:
            self.md.set_langevin(self.temperature, self.friction, [p.get("seed", 0) for p in parts],
                                 [p.get("steps_done", 0) for p in parts])
            if self.pressure is not None:
                self.md.set_barostat(self.pressure, self.baro_interval, seeds=[p.get("seed", 0) for p in parts],
                                     move0=[p.get("steps_done", 0) // self.baro_interval for p in parts],
                                     dv_max=[self.volume_fraction * p["volume0"] for p in parts])
        self._species = [p["species"] for p in parts]

    def step(self) -> float:
        """One MD step of the whole pack; returns its device time in ms."""
        torch = self.torch
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        self.md.step(1, self.dt)
        b.record()
        b.synchronize()
        return a.elapsed_time(b)

    def states(self) -> List[dict]:
        x, v, _ = self.md.state()
        cells, _, _ = self.md.cells()
        return [{"pos": x[s].clone(), "vel": v[s].clone(), "cell": cells[k].copy()} for k, s in enumerate(self.slices)]

    def upload(self, req: Request) -> dict:
        torch = self.torch
        return {"pos": torch.tensor(req.pos, dtype=torch.float64, device=self._dev),
                "vel": torch.tensor(req.vel, dtype=torch.float64, device=self._dev),
                "species": torch.tensor(req.species, dtype=torch.int32, device=self._dev),
                "cell": np.asarray(req.cell, dtype=np.float64), "pbc": np.asarray(req.pbc, dtype=np.uint8),
                "seed": int(req.seed), "steps_done": int(req.steps_done),
                "volume0": float(abs(np.linalg.det(np.asarray(req.cell, dtype=np.float64))))}

    def close(self):
        if self.md is not None:
            self.md.close()
            self.md = None


@dataclasses.dataclass
class ServingStats:
    step_ms: List[float] = dataclasses.field(default_factory=list)   # device time of each packed step
    iter_ms: List[float] = dataclasses.field(default_factory=list)   # wall time of each engine iteration,
    atoms_per_step: List[int] = dataclasses.field(default_factory=list)  # repack (if any) included
    repacks: int = 0
    rejected: int = 0
    wall_s: float = 0.0

    def summary(self) -> dict:
        ms = np.asarray(self.step_ms) if self.step_ms else np.zeros(1)
        it = np.asarray(self.iter_ms) if self.iter_ms else np.zeros(1)
        atom_steps = float(np.sum(self.atoms_per_step))
        busy = float(np.sum(ms)) / 1e3
        return {"steps": len(self.step_ms), "p50_ms": float(np.percentile(ms, 50)),
                "p99_ms": float(np.percentile(ms, 99)), "p50_iter_ms": float(np.percentile(it, 50)),
                "p99_iter_ms": float(np.percentile(it, 99)), "atom_steps": atom_steps,
                "atom_steps_per_s": atom_steps / self.wall_s if self.wall_s > 0 else 0.0,
                "atom_steps_per_busy_s": atom_steps / busy if busy > 0 else 0.0,
                "repacks": self.repacks, "rejected": self.rejected, "wall_s": self.wall_s}


class Server:
    """First-come-first-served admission by memory footprint and slot count;
    all admitted requests advance together, one packed launch per step."""

    def __init__(self, executor, budget_bytes: int, max_active: int = 64,
                 clock: Optional[Callable[[], float]] = None):
        self.ex = executor
        self.budget = budget_bytes
        self.max_active = max_active
        self.clock = clock or time.perf_counter
        self.pending: List[Request] = []
        self.active: List[Request] = []
        self.done: List[Request] = []
        self.state: List[dict] = []
        self.stats = ServingStats()

    def submit(self, req: Request) -> None:
        if self.ex.footprint(req.n_atoms) > self.budget:
            req.rejected = True
            self.stats.rejected += 1
            self.done.append(req)
            return
        self.pending.append(req)
        self.pending.sort(key=lambda r: (r.arrival, r.rid))

    def _footprint(self, reqs: Sequence[Request]) -> int:
        return self.ex.footprint(sum(r.n_atoms for r in reqs)) if reqs else 0

    def _head_fits(self, now: float, running: Sequence[Request]) -> bool:
        if not self.pending or self.pending[0].arrival > now or len(running) >= self.max_active:
            return False
        return self._footprint(list(running) + [self.pending[0]]) <= self.budget

    def run(self, idle_wait: Optional[Callable[[float], None]] = None) -> ServingStats:
        """Serve until every submitted request is finished or rejected."""
        t0 = self.clock()
        while self.pending or self.active:
            t_iter = self.clock()
            now = t_iter - t0
            running = [r for r in self.active if r.steps_done < r.n_steps]
            finished = len(running) < len(self.active)
            if finished or self._head_fits(now, running):
                # bring the device state of the pack back into the per-request records
                if self.ex.md is not None:
                    for st, cur in zip(self.state, self.ex.states()):
                        st.update(cur)
                keep_r, keep_s = [], []
                for r, st in zip(self.active, self.state):
                    if r.steps_done >= r.n_steps:
                        r.final_pos = st["pos"].cpu().numpy()
                        r.final_vel = st["vel"].cpu().numpy()
                        r.final_cell = np.asarray(st.get("cell", r.cell))
                        r.finished_at = now
                        self.done.append(r)
                    else:
                        keep_r.append(r)
                        keep_s.append(st)
                self.active, self.state = keep_r, keep_s
                while self._head_fits(now, self.active):
                    r = self.pending.pop(0)
                    r.admitted_at = now
                    self.active.append(r)
                    self.state.append(self.ex.upload(r))
                for r, st in zip(self.active, self.state):
                    st["steps_done"] = r.steps_done
                self.ex.launch(self.state)
                self.stats.repacks += 1
            if not self.active:
                if self.pending and idle_wait:
                    idle_wait(max(0.0, self.pending[0].arrival - (self.clock() - t0)))
                continue
            self.stats.step_ms.append(self.ex.step())
            self.stats.iter_ms.append(1e3 * (self.clock() - t_iter))
            self.stats.atoms_per_step.append(sum(r.n_atoms for r in self.active))
            for r in self.active:
                r.steps_done += 1
        self.stats.wall_s = self.clock() - t0
        self.ex.close()
        return self.stats
