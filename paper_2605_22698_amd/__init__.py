"""e3mi: equivariant message-passing interaction on MI355X (gfx950 HIP kernels).

Python face of libe3mi.so. Each class owns one opaque handle of the C ABI
(include/e3mi.h) and only marshals arguments: the neighbour lists, the
interaction, its adjoint and the MD integrator all run in the HIP library.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

import numpy as np

from . import _lib
from ._lib import BF16_MIX, FP32, E3miError, check, lib, ptr

__all__ = ["Model", "Graph", "MD", "E3miError", "FP32", "BF16_MIX", "weight_count", "energy_forces"]


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def weight_count(config_json: str) -> int:
    n = ctypes.c_size_t()
    check(lib().e3mi_weight_count(config_json.encode(), ctypes.byref(n)))
    return n.value


class Model:
    """Weights on the device plus the evaluation workspace.

    config_json: the model configuration (see include/e3mi.h); weights: FP64
    vector in the documented order; precision: FP32 or BF16_MIX.
    """

    def __init__(self, config_json: str, weights: np.ndarray, precision: int = FP32, device="cuda",
                 torch_allocator: bool = True):
        import torch
        self.device = torch.device(device)
        self.config_json = config_json
        w = np.ascontiguousarray(weights, dtype=np.float64)
        self._alloc = _lib.TorchAllocator(self.device) if torch_allocator else None
        h = ctypes.c_void_p()
        a = self._alloc.alloc_cb if self._alloc else _lib.ALLOC_FN()
        f = self._alloc.free_cb if self._alloc else _lib.FREE_FN()
        with torch.cuda.device(self.device):
            check(lib().e3mi_model_create(config_json.encode(), w.ctypes.data, w.size, precision, a, f, None,
                                          ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().e3mi_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable: bool = True, only: str = None):
        """Start (resetting counters) or stop per-stage HIP-event timing;
        only: time just this stage ("name" or "name@t"), else every stage."""
        if enable:
            check(lib().e3mi_profile_select(self.handle, (only or "").encode()))
        check(lib().e3mi_profile_enable(self.handle, 1 if enable else 0))

    def stage_time(self, stage: str):
        """(total ms, launches) of a timed stage, e.g. "radial_fwd" or "tp_fwd@2"."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        check(lib().e3mi_profile_query(self.handle, stage.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def set_flags(self, unfactorised_first_layer: bool = False, unfused_last_layer: bool = False,
                  fused_last_layer: bool = False, radial_per_edge: bool = False) -> None:
        """Evaluation options; see e3mi_model_set_flags."""
        flags = (1 if unfactorised_first_layer else 0) | (2 if unfused_last_layer else 0) | \
            (4 if fused_last_layer else 0) | (8 if radial_per_edge else 0)
        check(lib().e3mi_model_set_flags(self.handle, flags))

    def set_r_chunk_bytes(self, n_bytes: int) -> None:
        """Most bytes of per-edge radial weights held at once; see e3mi_model_set_r_chunk_bytes."""
        check(lib().e3mi_model_set_r_chunk_bytes(self.handle, int(n_bytes)))

    def set_r_keep_bytes(self, n_bytes: int) -> None:
        """Most bytes of per-edge radial weights kept whole across a chunked
        layer's forward pass and adjoint; see e3mi_model_set_r_keep_bytes."""
        check(lib().e3mi_model_set_r_keep_bytes(self.handle, int(n_bytes)))

    def set_weights(self, weights) -> None:
        """Replace the weights (FP64 vector in the documented layout; any device)."""
        w = weights.detach().to("cpu", dtype=__import__("torch").float64).contiguous().numpy() \
            if hasattr(weights, "detach") else np.ascontiguousarray(weights, dtype=np.float64)
        check(lib().e3mi_model_set_weights(self.handle, w.ctypes.data, w.size))
        self._uploaded = None

    def _use_weights(self, weights):
        """Make `weights` (a tensor) the device weights unless they already are,
        judged by value (an in-place update through .data leaves the version
        counter alone); returns the snapshot of what is now on the device."""
        import torch
        w = weights.detach()
        last = getattr(self, "_uploaded", None)
        if last is None or last.shape != w.shape or last.device != w.device or not torch.equal(last, w):
            self.set_weights(w)
            self._uploaded = w.clone()
        return self._uploaded

    def param_grad(self, graph: "Graph", pos, grad_energy, grad_forces, stream=None):
        """dL/dweights (FP64 device vector) for upstream dL/dE [S] and dL/dF [N,3]."""
        import torch
        n = weight_count(self.config_json)
        out = torch.empty(n, dtype=torch.float64, device=self.device)
        gE = grad_energy.to(self.device, torch.float64).contiguous()
        gF = grad_forces.to(self.device, torch.float32).contiguous()
        pos = pos.contiguous()
        check(lib().e3mi_param_grad(self.handle, graph.handle, ptr(pos), ptr(gE), ptr(gF), ptr(out),
                                    _stream(stream)))
        return out

    def hessian_vector(self, graph: "Graph", pos, v, stream=None):
        """H v (FP32 device [N, 3]) for a direction v [N, 3]; see e3mi_hessian_vector."""
        import torch
        v = v.to(self.device, torch.float32).contiguous()
        hv = torch.empty_like(v)
        check(lib().e3mi_hessian_vector(self.handle, graph.handle, ptr(pos.contiguous()), ptr(v), ptr(hv),
                                        _stream(stream)))
        return hv

    def hessian_vectors(self, graph: "Graph", pos, V, stream=None):
        """H V[k] for every direction (V: [K, N, 3]; FP32 device result of the
        same shape); see e3mi_hessian_vectors."""
        import torch
        V = V.to(self.device, torch.float32).contiguous()
        HV = torch.empty_like(V)
        check(lib().e3mi_hessian_vectors(self.handle, graph.handle, ptr(pos.contiguous()), V.shape[0], ptr(V),
                                         ptr(HV), _stream(stream)))
        return HV

    def _unit_directions(self, graph: "Graph", atoms):
        """[K, N, 3] directions: direction k has, for every structure s with
        atoms[k, s] >= 0, a unit entry at (that atom of s, axis k % 3)."""
        import torch
        K, S = atoms.shape
        kk, ss = np.nonzero(atoms >= 0)
        V = torch.zeros((K, graph.n_atoms, 3), dtype=torch.float32, device=self.device)
        if len(kk):
            idx = torch.as_tensor(np.stack([kk, graph.offsets[ss] + atoms[kk, ss], kk % 3]), device=self.device)
            V[idx[0], idx[1], idx[2]] = 1.0
        return V

    def hessian_rows(self, graph: "Graph", pos, rows, stream=None):
        """Sampled Hessian rows (Section 5.2): rows[r, s] is an atom index
        within structure s; returns [R, 3, N, 3] with out[r, a] = H v for v
        the sum over structures of the unit vectors (atom rows[r, s], axis a),
        i.e. every structure's Hessian row of that atom and axis."""
        rows = np.asarray(rows, dtype=np.int64).reshape(-1, graph.n_structures)
        if np.any(rows < 0) or np.any(rows >= np.diff(graph.offsets)[None, :]):
            raise ValueError("row atom index outside its structure")
        V = self._unit_directions(graph, np.repeat(rows, 3, axis=0))
        return self.hessian_vectors(graph, pos, V, stream).view(rows.shape[0], 3, graph.n_atoms, 3)

    def hessian(self, graph: "Graph", pos, stream=None):
        """Full Hessian of every structure (list of FP32 [3 N_s, 3 N_s]) from
        3 max_s N_s Hessian-vector products, each probing one coordinate of
        every structure at once."""
        off = graph.offsets
        sizes = np.diff(off)
        K = 3 * int(sizes.max(initial=0))
        atom = np.arange(K)[:, None] // 3
        V = self._unit_directions(graph, np.where(atom < sizes[None, :], atom, -1))
        HV = self.hessian_vectors(graph, pos, V, stream)  # [K, N, 3]; column k of every Hessian
        return [HV[:3 * n, off[s]:off[s + 1]].reshape(3 * n, 3 * n).t().contiguous() for s, n in enumerate(sizes)]

    def footprint_bytes(self, n_atoms: int, n_edges: int) -> int:
        return int(lib().e3mi_footprint_bytes(self.handle, n_atoms, n_edges))

    def build_graph(self, offsets, pos, species, cell, pbc, cutoff: float, skin: float = 0.0,
                    stream=None) -> "Graph":
        return Graph(self, offsets, pos, species, cell, pbc, cutoff, skin, stream)

    def energy_forces(self, graph: "Graph", pos, atom_energy: bool = False, stream=None):
        """(E [S] FP64, F [N,3] FP32, E_i [N] FP64 or None) as device tensors."""
        import torch
        S, N = graph.n_structures, graph.n_atoms
        E = torch.empty(S, dtype=torch.float64, device=self.device)
        F = torch.empty((N, 3), dtype=torch.float32, device=self.device)
        Ei = torch.empty(N, dtype=torch.float64, device=self.device) if atom_energy else None
        pos = pos.contiguous()
        assert pos.dtype == torch.float64 and pos.shape == (N, 3)
        check(lib().e3mi_energy_forces(self.handle, graph.handle, ptr(pos), ptr(E), ptr(F), ptr(Ei),
                                       _stream(stream)))
        return E, F, Ei


class Graph:
    """Neighbour lists (skin list + per-call cutoff selection) of a packed batch."""

    def __init__(self, model: Model, offsets, pos, species, cell, pbc, cutoff, skin, stream=None):
        import torch
        self.model = model
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        cell = np.ascontiguousarray(cell, dtype=np.float64).reshape(-1, 3, 3)
        pbc = np.ascontiguousarray(pbc, dtype=np.uint8).reshape(-1, 3)
        self.n_structures = len(off) - 1
        self.n_atoms = int(off[-1])
        self.offsets = off
        assert cell.shape[0] == self.n_structures and pbc.shape[0] == self.n_structures
        pos = pos.contiguous()
        self._species = species.to(torch.int32).contiguous()
        assert pos.dtype == torch.float64 and pos.shape == (self.n_atoms, 3)
        h = ctypes.c_void_p()
        check(lib().e3mi_build_graph(model.handle, self.n_structures, off.ctypes.data, ptr(pos),
                                     ptr(self._species), cell.ctypes.data, pbc.ctypes.data, cutoff, skin,
                                     _stream(stream), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().e3mi_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_skin_edges(self) -> int:
        e = ctypes.c_int64()
        check(lib().e3mi_graph_info(self.handle, None, ctypes.byref(e)))
        return e.value

    def last_edge_count(self, stream=None) -> int:
        e = ctypes.c_int64()
        check(lib().e3mi_graph_last_edge_count(self.handle, ctypes.byref(e), _stream(stream)))
        return e.value

    def set_total_charge(self, total_charge):
        """Total charge of each structure (elementary charges) for the
        charge correction of the Coulomb term; see e3mi_graph_set_total_charge."""
        q = np.ascontiguousarray(total_charge, dtype=np.float64)
        if q.shape != (self.n_structures,):
            raise ValueError("one total charge per structure")
        check(lib().e3mi_graph_set_total_charge(self.handle, q.ctypes.data))

    def edges(self, stream=None):
        """Skin list as device tensors (row_ptr [N+1], src [E], shift [E,3], rev [E])."""
        import torch
        E = self.n_skin_edges
        dev = self.model.device
        row_ptr = torch.empty(self.n_atoms + 1, dtype=torch.int32, device=dev)
        src = torch.empty(max(E, 1), dtype=torch.int32, device=dev)
        shift = torch.empty((max(E, 1), 3), dtype=torch.int32, device=dev)
        rev = torch.empty(max(E, 1), dtype=torch.int32, device=dev)
        check(lib().e3mi_graph_copy_edges(self.handle, ptr(row_ptr), ptr(src), ptr(shift), ptr(rev),
                                          _stream(stream)))
        return row_ptr, src[:E], shift[:E], rev[:E]


class MD:
    """Velocity-Verlet NVE trajectories of a packed batch, state kept on the device."""

    def __init__(self, model: Model, offsets, pos, vel, species, masses, cell, pbc, cutoff: float,
                 skin: float = 1.0, rebuild_every: int = 20, stream=None):
        import torch
        self.model = model
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        self.n_structures = len(off) - 1
        self.n_atoms = int(off[-1])
        cell = np.ascontiguousarray(cell, dtype=np.float64).reshape(-1, 3, 3)
        pbc = np.ascontiguousarray(pbc, dtype=np.uint8).reshape(-1, 3)
        masses = np.ascontiguousarray(masses, dtype=np.float64)
        n_species = int(__import__("json").loads(model.config_json)["n_species"])
        for name, t in (("pos", pos), ("vel", vel)):
            if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or tuple(t.shape) != (self.n_atoms, 3):
                raise ValueError(f"{name} must be a float64 tensor of shape [{self.n_atoms}, 3]")
        if not isinstance(species, torch.Tensor) or tuple(species.shape) != (self.n_atoms,) or \
                species.dtype not in (torch.int32, torch.int64):
            raise ValueError(f"species must be an integer tensor of shape [{self.n_atoms}]")
        if masses.shape != (n_species,):
            raise ValueError(f"masses must hold one value per species ({n_species})")
        pos, vel = pos.contiguous(), vel.contiguous()
        species = species.to(torch.int32).contiguous()
        h = ctypes.c_void_p()
        check(lib().e3mi_md_create(model.handle, self.n_structures, off.ctypes.data, ptr(pos), ptr(vel), ptr(species),
                                   masses.ctypes.data, cell.ctypes.data, pbc.ctypes.data, cutoff, skin, rebuild_every,
                                   _stream(stream), ctypes.byref(h)))
        self.handle = h

    def step(self, n_steps: int, dt_fs: float, energy_out=None, stream=None):
        check(lib().e3mi_md_step(self.handle, n_steps, dt_fs, ptr(energy_out), _stream(stream)))

    def state(self, stream=None):
        import torch
        dev = self.model.device
        x = torch.empty((self.n_atoms, 3), dtype=torch.float64, device=dev)
        v = torch.empty((self.n_atoms, 3), dtype=torch.float64, device=dev)
        F = torch.empty((self.n_atoms, 3), dtype=torch.float32, device=dev)
        check(lib().e3mi_md_state(self.handle, ptr(x), ptr(v), ptr(F), _stream(stream)))
        return x, v, F

    def set_langevin(self, temperature_K: float, friction_per_fs: float, seeds=None, step0=None, stream=None):
        """Langevin (BAOAB) steps from now on; see e3mi_md_set_langevin.
        seeds, step0: one per structure (host integers) or None."""
        sd = None if seeds is None else np.ascontiguousarray(seeds, dtype=np.uint64)
        s0 = None if step0 is None else np.ascontiguousarray(step0, dtype=np.int64)
        for a in (sd, s0):
            if a is not None and a.shape != (self.n_structures,):
                raise ValueError("one seed and one step offset per structure")
        check(lib().e3mi_md_set_langevin(self.handle, float(temperature_K), float(friction_per_fs), ptr(sd), ptr(s0),
                                         _stream(stream)))

    def set_barostat(self, pressure_bar: float, interval: int, volume_fraction: float = 0.01, seeds=None,
                     move0=None, dv_max=None):
        """Monte Carlo volume moves on each structure's own schedule; see
        e3mi_md_set_barostat. dv_max: per-structure volume step (A^3) or None."""
        sd = None if seeds is None else np.ascontiguousarray(seeds, dtype=np.uint64)
        m0 = None if move0 is None else np.ascontiguousarray(move0, dtype=np.int64)
        dv = None if dv_max is None else np.ascontiguousarray(dv_max, dtype=np.float64)
        for a in (sd, m0, dv):
            if a is not None and a.shape != (self.n_structures,):
                raise ValueError("one value per structure")
        check(lib().e3mi_md_set_barostat(self.handle, float(pressure_bar), int(interval), float(volume_fraction),
                                         ptr(dv), ptr(sd), ptr(m0)))

    def set_total_charge(self, total_charge, stream=None):
        """Total charge of each structure; recomputes the current forces."""
        q = np.ascontiguousarray(total_charge, dtype=np.float64)
        if q.shape != (self.n_structures,):
            raise ValueError("one total charge per structure")
        check(lib().e3mi_md_set_total_charge(self.handle, q.ctypes.data, _stream(stream)))

    def cells(self):
        """(cells [S, 3, 3] host FP64, proposals, accepted) after the last step."""
        c = np.zeros((self.n_structures, 3, 3), dtype=np.float64)
        p, a = ctypes.c_int64(), ctypes.c_int64()
        check(lib().e3mi_md_cells(self.handle, c.ctypes.data, ctypes.byref(p), ctypes.byref(a)))
        return c, p.value, a.value

    def stats(self) -> Tuple[int, int, int]:
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(lib().e3mi_md_stats(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def close(self):
        if getattr(self, "handle", None):
            lib().e3mi_md_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _energy_forces_function():
    import torch

    class EnergyForces(torch.autograd.Function):
        """(E, F) of a packed batch as a differentiable function of the weights.

        forward: the library's energy + forces; backward: its parameter-gradient
        pass (second order through F). Positions are inputs, not differentiated.
        """

        @staticmethod
        def forward(ctx, weights, pos, model, graph):
            # the weights this forward used, kept for its backward (the model's
            # device weights may have changed by then)
            ctx.weights = model._use_weights(weights)
            E, F, _ = model.energy_forces(graph, pos)
            ctx.model, ctx.graph = model, graph
            ctx.save_for_backward(pos)
            return E, F

        @staticmethod
        def backward(ctx, gE, gF):
            (pos,) = ctx.saved_tensors
            m = ctx.model
            m._use_weights(ctx.weights)
            if gE is None:
                gE = torch.zeros(ctx.graph.n_structures, dtype=torch.float64, device=m.device)
            if gF is None:
                gF = torch.zeros((ctx.graph.n_atoms, 3), dtype=torch.float32, device=m.device)
            g = m.param_grad(ctx.graph, pos, gE, gF)
            return g, None, None, None

    return EnergyForces


_EF = None


def energy_forces(weights, pos, model: Model, graph: Graph):
    """Differentiable (E [S] FP64, F [N,3] FP32) with respect to `weights`."""
    global _EF
    if _EF is None:
        _EF = _energy_forces_function()
    return _EF.apply(weights, pos, model, graph)
