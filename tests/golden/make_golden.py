"""Write the stored oracle results the GPU parity tests compare against.

Calls only the seeded generators and the FP64 oracle; no value comes from the
HIP library. Rerun after any change of the oracle's arithmetic or the inputs:

    python tests/golden/make_golden.py [name ...]

single_3000.npz  3,000-atom periodic box at 0.1 atoms/A^3 (jittered lattice,
                 0.3 A noise), 4 species, r_c 5 A, l_max 3, 128 channels,
                 2 layers: per-structure energy, per-atom energies, forces.
scale_sub_2000.npz  the independent 2,000-atom periodic box of the
                 100,000-atom configuration (r_c 6 A, l_max 3, 128 channels,
                 3 layers): energy, per-atom energies, forces.
grad_batch_64.npz  the differentiation batch (64 periodic boxes of 20-200
                 atoms, 5 species, l_max 3, 64 channels, 2 layers, seeded
                 N(0, 1) targets): loss = mean_s (E_s - E_s*)^2 +
                 sum_i |F_i - F_i*|^2 / (3 sum N) and its gradient with
                 respect to every weight (flat, in the library's order),
                 with the energies, per-atom energies and forces. The loss is a sum of
                 per-structure terms, so the oracle evaluates each structure
                 alone, with that structure's share of the normalisation.
"""
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import model as om  # noqa: E402


def single_3000():
    cfg, b = synth.single_config()
    w = synth.model_weights(cfg, 2)
    m = om.Model(cfg, w)
    E, F, Ei = om.energy_forces(m, b, edge_chunk=8192)
    np.savez_compressed(os.path.join(HERE, "single_3000.npz"), energy=E, forces=F, atom_energy=Ei,
                        n_atoms=b.n_atoms)


def scale_sub_2000():
    cfg, b = synth.scale_subbox()
    m = om.Model(cfg, synth.model_weights(cfg, 5))
    E, F, Ei = om.energy_forces(m, b, edge_chunk=4096)
    np.savez_compressed(os.path.join(HERE, "scale_sub_2000.npz"), energy=E, forces=F, atom_energy=Ei,
                        n_atoms=b.n_atoms)


def grad_batch_64():
    cfg, b, e_ref, f_ref = synth.differentiation_config()
    m = om.Model(cfg, synth.model_weights(cfg, 3))
    S, n3 = b.n_structures, 3 * b.n_atoms
    loss, flat, E, F, Ei = 0.0, None, np.zeros(S), np.zeros((b.n_atoms, 3)), np.zeros(b.n_atoms)
    for s in range(S):
        a, z = int(b.offsets[s]), int(b.offsets[s + 1])
        bs = b.structure(s)
        ls, gs = om.loss_and_grads(m, bs, e_ref[s:s + 1], f_ref[a:z], w_energy=1.0 / S,
                                   w_forces=3.0 * (z - a) / n3)
        loss += ls
        g = synth.flatten_weights(cfg, gs)
        flat = g if flat is None else flat + g
        Es, Fs, Eis = om.energy_forces(m, bs)
        E[s], F[a:z], Ei[a:z] = Es[0], Fs, Eis
    np.savez_compressed(os.path.join(HERE, "grad_batch_64.npz"), loss=loss, grad=flat, energy=E, forces=F,
                        atom_energy=Ei, n_atoms=b.n_atoms)


JOBS = {"single_3000": single_3000, "scale_sub_2000": scale_sub_2000, "grad_batch_64": grad_batch_64}

if __name__ == "__main__":
    torch.set_num_threads(os.cpu_count() or 1)
    for name in sys.argv[1:] or list(JOBS):
        t = time.time()
        JOBS[name]()
        print(f"{name}: {time.time() - t:.1f} s", flush=True)
