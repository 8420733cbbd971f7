"""The equivariant interaction model, energy, forces and loss gradients (oracle).

§4 of the paper: its backend speeds up the Clebsch-Gordan tensor product
that MACE and NequIP use inside message passing. The paper gives no model
equations; the model below is the reading, each step anchored to the
Appendix F hyperparameter tables:

  geometry     d_e = r_j - r_i + n.cell for edge e = (i <- j, n); r_e = |d_e|
  harmonics    Y_e = real_sh(d_e), l <= l_max                       (sh.py)
  basis        B_e = radial_basis(r_e)                               (basis.py)
  embedding    h0_i = W_emb[z_i] (scalars only)
  layer t      R_e = W3^T silu(W2^T silu(W1^T B_e)), no biases, one weight
                   per (path, channel)   (NequIP table: 2 hidden layers of 64, swish)
               A_i[p,k,m3] = 1/nu sum_{e in in(i)} R_e[p,k]
                                sum_{m1,m2} C^p[m1,m2,m3] h_j[k,l1,m1] Y_e[l2,m2]
               h~_i[l3] = sum_{p: l3(p)=l3} A_i[p] W_{l3}[p] + h_i[l3] S_{l3}
               gate (MACE table: gate_nodes): h[0] = silu(h~[0]),
                    h[l>0] = h~[l] * sigmoid(h~[0])
  readout      E_i = w2^T silu(W_r^T h_i[0]) + E0[z_i]   (MACE table:
                   readout irreps 16x0e -> 0e; §5.3 readout with one head)
  energy       E_s = sum_{i in s} E_i
  forces       F = -dE/dr (§5.2: the Hessian is minus the position
                   derivative of the forces, i.e. forces are -dE/dr)
  Hessian      (H v)_j = sum_i v_i . d^2 E / dr_i dr_j = d(grad E . v)/dr_j,
                   the Hessian-vector product of §5.2's full-Hessian equation
                   (sampled Hessian rows are H v for v = one unit vector per
                   structure; the full Hessian is 3n such products)

Product block (MACE's symmetric contraction of body order 2; the paper's
MACE models use correlation 2, Appendix F; the block follows Batatia et al.,
NeurIPS 2022, written per channel k with species-dependent weights; reading):
  A~^L      the channel mix of the layer's neighbour sum, without the self
            connection, for every order L <= lmax
  B^L_k     = w1[z_i, L, k] A~^L_k + sum_{(l1 <= l2, L)} w2[z_i, p, k] (A~^{l1}_k (x) A~^{l2}_k)_L
            where (x)_L is the CG coupling of the two orders into L
  h~^L      = B^L W_lin,L + h^{t-1,L} W_self,L,  then the gate; output orders
            L <= lmax, only L = 0 in the last layer

Electrostatics (§5.1, when the config enables `coulomb`; open structures):
  charges      q_i = w_q . h_i[0] + b_q[z_i]  (a linear charge head on the
                   final scalar features; reading)
  correction   q~_i = q_i - (sum_{j in s} q_j - Q_s) / N_s  (the paper's
                   charge-correction equation, Q_s the total charge)
  E_LR         = 1/2 sum_{i != j in s} k_e q~_i q~_j / chi(r_ij),
                   1/chi(r) = phi(r/r0) / sqrt(r^2 + 1) + (1 - phi(r/r0)) / r,
                   phi(x) = 1 - 6x^5 + 15x^4 - 10x^3 for x < 1, else 0
               (the PhysNet soft-core form the paper cites; chi(r) = r beyond
               the soft-core radius r0; each atom carries half of each pair
               term in its E_i), k_e = 14.399645 eV A / e^2.

nu is a fixed constant of the model (the nominal neighbour count). Every
layer outputs all orders l <= l_max. Computation is FP64 throughout.

The neighbour sum may be evaluated over edge chunks, each recomputed in the
backward pass, which only bounds memory; the arithmetic per edge is the
definition above.
"""
from typing import Dict, List, Optional, Tuple

import numpy as np
import torch
from torch.utils.checkpoint import checkpoint

from . import basis, cg
from .sh import real_sh, sl

K_E = 14.399645478425668  # e^2 / (4 pi eps0) in eV angstrom


def soft_core_switch(x: torch.Tensor) -> torch.Tensor:
    """phi(x) = 1 - 6x^5 + 15x^4 - 10x^3 for 0 <= x < 1, 0 beyond."""
    p = 1.0 - 6.0 * x ** 5 + 15.0 * x ** 4 - 10.0 * x ** 3
    return torch.where(x < 1.0, p, torch.zeros_like(x))


def inv_chi(r: torch.Tensor, r0: float) -> torch.Tensor:
    """1 / chi(r): the soft-core Coulomb kernel."""
    phi = soft_core_switch(r / r0)
    return phi / torch.sqrt(r * r + 1.0) + (1.0 - phi) / r


def coulomb_atom_energies(pos: torch.Tensor, q: torch.Tensor, offsets: np.ndarray, r0: float) -> torch.Tensor:
    """1/2 sum_{j != i, same structure} k_e q_i q_j / chi(r_ij) for every atom i
    (all pairs of each structure, no cutoff)."""
    out = []
    for s in range(len(offsets) - 1):
        a, b = int(offsets[s]), int(offsets[s + 1])
        x, qs = pos[a:b], q[a:b]
        n = b - a
        if n == 0:
            continue
        d = x[None, :, :] - x[:, None, :]
        off = ~torch.eye(n, dtype=torch.bool)
        r = torch.sqrt((d * d).sum(-1)[off])
        pair = K_E * (qs[:, None] * qs[None, :])[off] * inv_chi(r, r0)
        e = torch.zeros(n * n, dtype=pos.dtype).masked_scatter(off.reshape(-1), pair).reshape(n, n)
        out.append(0.5 * e.sum(1))
    return torch.cat(out) if out else torch.zeros(0, dtype=pos.dtype)


def charges(model, h0: torch.Tensor, species: torch.Tensor, offsets: np.ndarray,
            total_charge: np.ndarray) -> torch.Tensor:
    """Corrected partial charges q~ from the final scalar features h0 [N, C]."""
    w = model.w
    q = h0 @ w["qhead"] + w["qbias"][species]
    owner = torch.from_numpy(np.repeat(np.arange(len(offsets) - 1), np.diff(offsets)))
    S = len(offsets) - 1
    tot = torch.zeros(S, dtype=q.dtype).index_add(0, owner, q)
    n = torch.from_numpy(np.diff(offsets).astype(np.float64))
    shift = (tot - torch.from_numpy(np.asarray(total_charge, dtype=np.float64))) / torch.clamp(n, min=1.0)
    return q - shift[owner]


def silu(x):
    return x * torch.sigmoid(x)


class Model:
    def __init__(self, cfg, weights: Dict[str, np.ndarray]):
        self.cfg = cfg
        self.w = {k: torch.tensor(np.asarray(v), dtype=torch.float64) for k, v in weights.items()}
        self.layer_paths: List[List[Tuple[int, int, int]]] = []
        for t in range(1, cfg.layers + 1):
            l_in = [0] if t == 1 else list(range(cfg.lmax + 1))
            self.layer_paths.append(cg.paths(l_in, cfg.lmax))
        self.cg = {}
        for ps in self.layer_paths:
            for p in ps:
                if p not in self.cg:
                    self.cg[p] = torch.tensor(cg.real_cg(*p))

    def parameters(self) -> Dict[str, torch.Tensor]:
        return self.w

    # -- one layer's neighbour sum over a set of edges --------------------
    def _messages(self, t: int, h_flat: torch.Tensor, B: torch.Tensor, Y: torch.Tensor,
                  src: torch.Tensor, dst: torch.Tensor, n_atoms: int) -> torch.Tensor:
        """Returns A as [N, C, sum_p (2 l3 + 1)] (paths concatenated)."""
        cfg, w = self.cfg, self.w
        C = cfg.channels
        paths = self.layer_paths[t - 1]
        R = silu(silu(B @ w[f"rad1_{t}"]) @ w[f"rad2_{t}"]) @ w[f"rad3_{t}"]
        R = R.view(-1, len(paths), C)
        hj = h_flat[src]                                   # [E, C, (lmax+1)^2]
        out = []
        for pi, (l1, l2, l3) in enumerate(paths):
            Tp = torch.einsum("abc,eka,eb->ekc", self.cg[(l1, l2, l3)], hj[:, :, sl(l1)], Y[:, sl(l2)])
            msg = R[:, pi, :, None] * Tp
            out.append(torch.zeros(n_atoms, C, 2 * l3 + 1, dtype=msg.dtype).index_add(0, dst, msg))
        return torch.cat(out, dim=2) / cfg.avg_neighbors

    def coupling(self, l1: int, l2: int, L: int) -> torch.Tensor:
        if (l1, l2, L) not in self.cg:
            self.cg[(l1, l2, L)] = torch.tensor(cg.real_cg(l1, l2, L))
        return self.cg[(l1, l2, L)]

    def product_basis(self, t: int, At: List[torch.Tensor], species: torch.Tensor) -> List[torch.Tensor]:
        """B^L for L <= the layer's output order, from A~ (list over l of [N, C, 2l+1])."""
        cfg, w = self.cfg, self.w
        lo = 0 if t == cfg.layers else cfg.lmax
        w1 = w[f"sym1_{t}"][species]                      # [N, lo+1, C]
        w2 = w[f"sym2_{t}"][species]                      # [N, pairs, C]
        out = [w1[:, L, :, None] * At[L] for L in range(lo + 1)]
        p = 0
        for L in range(lo + 1):
            for l1 in range(cfg.lmax + 1):
                for l2 in range(l1, cfg.lmax + 1):
                    if not (abs(l1 - l2) <= L <= l1 + l2 and (l1 + l2 + L) % 2 == 0):
                        continue
                    prod = torch.einsum("abc,nka,nkb->nkc", self.coupling(l1, l2, L), At[l1], At[l2])
                    out[L] = out[L] + w2[:, p, :, None] * prod
                    p += 1
        return out

    def _product_block(self, t, At, h, species, l_in):
        w = self.w
        Bs = self.product_basis(t, At, species)
        ht = []
        for L, B in enumerate(Bs):
            acc = torch.einsum("nkm,kq->nqm", B, w[f"lin_{t}_{L}"])
            if L in l_in:
                acc = acc + torch.einsum("nkm,kq->nqm", h[:, :, sl(L)], w[f"self_{t}_{L}"])
            ht.append(acc)
        return ht

    def node_energies(self, pos: torch.Tensor, species: torch.Tensor, dst: torch.Tensor,
                      src: torch.Tensor, shift_vec: torch.Tensor, edge_chunk: Optional[int] = None,
                      features: Optional[list] = None, offsets: Optional[np.ndarray] = None,
                      total_charge: Optional[np.ndarray] = None) -> torch.Tensor:
        """E_i for every atom. pos [N,3] FP64 (may require grad), shift_vec [E,3]
        the Cartesian image displacement of each edge. With the Coulomb term
        the structure offsets (and total charges, default 0) are needed."""
        cfg, w = self.cfg, self.w
        N, C, L = pos.shape[0], cfg.channels, cfg.lmax
        nc = (L + 1) ** 2
        d = pos[src] - pos[dst] + shift_vec
        r = torch.linalg.norm(d, dim=-1)
        Y = real_sh(d, L)
        B = basis.radial_basis(r, cfg.cutoff, cfg.n_basis, cfg.envelope_p)
        h = torch.cat([w["emb"][species][:, :, None], torch.zeros(N, C, nc - 1, dtype=torch.float64)], 2)
        for t in range(1, cfg.layers + 1):
            paths = self.layer_paths[t - 1]
            if edge_chunk is None or edge_chunk >= len(src):
                A = self._messages(t, h, B, Y, src, dst, N)
            else:
                A = None
                for a in range(0, len(src), edge_chunk):
                    b = min(a + edge_chunk, len(src))
                    part = checkpoint(self._messages, t, h, B[a:b], Y[a:b], src[a:b], dst[a:b], N,
                                      use_reentrant=False)
                    A = part if A is None else A + part
            # split A per path
            Ap, off = [], 0
            for (_, _, l3) in paths:
                Ap.append(A[:, :, off:off + 2 * l3 + 1])
                off += 2 * l3 + 1
            l_in = [0] if t == 1 else list(range(L + 1))
            mace = getattr(cfg, "correlation", 1) == 2
            ht = []
            for l3 in range(L + 1):
                acc = torch.zeros(N, C, 2 * l3 + 1, dtype=torch.float64)
                Wm = w[f"mix_{t}_{l3}"]
                q = 0
                for pi, (_, _, pl3) in enumerate(paths):
                    if pl3 != l3:
                        continue
                    acc = acc + torch.einsum("nkm,kq->nqm", Ap[pi], Wm[q * C:(q + 1) * C])
                    q += 1
                if l3 in l_in and not mace:
                    acc = acc + torch.einsum("nkm,kq->nqm", h[:, :, sl(l3)], w[f"self_{t}_{l3}"])
                ht.append(acc)
            if mace:
                ht = self._product_block(t, ht, h, species, l_in)
            g = torch.sigmoid(ht[0])                       # [N, C, 1]
            h = torch.cat([silu(ht[0])] + [ht[l] * g for l in range(1, len(ht))], dim=2)
            if h.shape[2] < nc:
                h = torch.cat([h, torch.zeros(N, C, nc - h.shape[2], dtype=h.dtype)], dim=2)
            if features is not None:
                features.append(h)
        e = silu(h[:, :, 0] @ w["read1"]) @ w["read2"]
        e = e[:, 0] + w["e0"][species]
        if getattr(cfg, "coulomb", False):
            if offsets is None:
                offsets = np.array([0, N])
            if total_charge is None:
                total_charge = np.zeros(len(offsets) - 1)
            q = charges(self, h[:, :, 0], species, offsets, total_charge)
            e = e + coulomb_atom_energies(pos, q, offsets, cfg.soft_core_r0)
        return e


def structure_energies(e_atom: torch.Tensor, offsets: np.ndarray) -> torch.Tensor:
    """E_s = sum over the atoms of structure s."""
    owner = torch.from_numpy(np.repeat(np.arange(len(offsets) - 1), np.diff(offsets)))
    return torch.zeros(len(offsets) - 1, dtype=e_atom.dtype).index_add(0, owner, e_atom)


def _total_charge(batch) -> np.ndarray:
    c = getattr(batch, "charge", None)
    return np.zeros(len(batch.offsets) - 1) if c is None else np.asarray(c, dtype=np.float64)


def _check_open(model, batch):
    if getattr(model.cfg, "coulomb", False) and np.any(np.asarray(batch.pbc)):
        raise ValueError("the Coulomb term is defined for open structures only")


def _edges(batch, cutoff):
    from .neighbours import neighbour_list, shift_vectors
    dst, src, sh = neighbour_list(batch.pos, batch.cell, batch.pbc, batch.offsets, cutoff)
    return (torch.from_numpy(dst), torch.from_numpy(src),
            torch.from_numpy(shift_vectors(sh, dst, batch.cell, batch.offsets)))


def energy_forces(model: Model, batch, edge_chunk: Optional[int] = None, edges=None,
                  features: Optional[list] = None):
    """(E_s [S], F [N,3], E_i [N]) in FP64. F = -dE/dr by autograd."""
    dst, src, shv = edges if edges is not None else _edges(batch, model.cfg.cutoff)
    pos = torch.tensor(batch.pos, dtype=torch.float64, requires_grad=True)
    species = torch.from_numpy(np.asarray(batch.species, dtype=np.int64))
    _check_open(model, batch)
    e_atom = model.node_energies(pos, species, dst, src, shv, edge_chunk, features, batch.offsets,
                                 _total_charge(batch))
    E = structure_energies(e_atom, batch.offsets)
    (g,) = torch.autograd.grad(E.sum(), pos)
    return E.detach().numpy(), (-g).numpy(), e_atom.detach().numpy()


def hessian_vector(model: Model, batch, v: np.ndarray, edges=None) -> np.ndarray:
    """H v [N, 3] in FP64 by differentiating grad E . v once more."""
    dst, src, shv = edges if edges is not None else _edges(batch, model.cfg.cutoff)
    pos = torch.tensor(batch.pos, dtype=torch.float64, requires_grad=True)
    species = torch.from_numpy(np.asarray(batch.species, dtype=np.int64))
    _check_open(model, batch)
    e_atom = model.node_energies(pos, species, dst, src, shv, None, None, batch.offsets, _total_charge(batch))
    (g,) = torch.autograd.grad(e_atom.sum(), pos, create_graph=True)
    (hv,) = torch.autograd.grad((g * torch.as_tensor(v, dtype=torch.float64)).sum(), pos)
    return hv.numpy()


def energy(model: Model, batch, edges=None, edge_chunk: Optional[int] = None) -> np.ndarray:
    dst, src, shv = edges if edges is not None else _edges(batch, model.cfg.cutoff)
    pos = torch.tensor(batch.pos, dtype=torch.float64)
    species = torch.from_numpy(np.asarray(batch.species, dtype=np.int64))
    _check_open(model, batch)
    with torch.no_grad():
        e_atom = model.node_energies(pos, species, dst, src, shv, edge_chunk, None, batch.offsets,
                                     _total_charge(batch))
    return structure_energies(e_atom, batch.offsets).numpy()


def loss_and_grads(model: Model, batch, e_ref: np.ndarray, f_ref: np.ndarray,
                   w_energy: float = 1.0, w_forces: float = 1.0, edges=None,
                   edge_chunk: Optional[int] = None):
    """loss = w_E mean_s (E_s - E_ref)^2 + w_F sum (F - F_ref)^2 / (3 N),
    and its gradient with respect to every weight tensor (second order
    through the forces)."""
    dst, src, shv = edges if edges is not None else _edges(batch, model.cfg.cutoff)
    params = model.parameters()
    for v in params.values():
        v.requires_grad_(True)
    try:
        pos = torch.tensor(batch.pos, dtype=torch.float64, requires_grad=True)
        species = torch.from_numpy(np.asarray(batch.species, dtype=np.int64))
        _check_open(model, batch)
        e_atom = model.node_energies(pos, species, dst, src, shv, edge_chunk, None, batch.offsets,
                                     _total_charge(batch))
        E = structure_energies(e_atom, batch.offsets)
        (g,) = torch.autograd.grad(E.sum(), pos, create_graph=True)
        F = -g
        loss = (w_energy * torch.mean((E - torch.from_numpy(e_ref)) ** 2)
                + w_forces * torch.sum((F - torch.from_numpy(f_ref)) ** 2) / F.numel())
        names = list(params.keys())
        grads = torch.autograd.grad(loss, [params[k] for k in names], allow_unused=True)
        out = {k: (torch.zeros_like(params[k]) if gk is None else gk).detach().numpy()
               for k, gk in zip(names, grads)}
        return float(loss.detach()), out
    finally:
        for v in params.values():
            v.requires_grad_(False)
