"""Helpers shared by the GPU tests (inputs to device, model construction,
tolerance checks). Imports torch lazily so the CPU suite never needs a GPU."""
import sys

import numpy as np

import synth


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def device():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch.device("cuda:0")


def model(cfg, seed_key, precision=0):
    import paper_2605_22698_amd as e3
    w = synth.flatten_weights(cfg, synth.model_weights(cfg, seed_key))
    return e3.Model(cfg.to_json(), w, precision=precision, device=device())


def to_dev(batch):
    import torch
    d = device()
    return (torch.tensor(batch.pos, dtype=torch.float64, device=d),
            torch.tensor(batch.species, dtype=torch.int32, device=d))


def gpu_energy_forces(m, batch, skin=0.0, cutoff=None):
    import torch
    pos, sp = to_dev(batch)
    rc = cutoff if cutoff is not None else synth.ModelConfig.from_json(m.config_json).cutoff
    g = m.build_graph(batch.offsets, pos, sp, batch.cell, batch.pbc, rc, skin)
    E, F, Ei = m.energy_forces(g, pos, atom_energy=True)
    torch.cuda.synchronize()
    return E.cpu().numpy(), F.cpu().numpy().astype(np.float64), Ei.cpu().numpy(), g


def check_energy(E_gpu, E_ref, Ei_ref, rel=1e-5):
    """Energy within `rel` of |E_ref|; when the per-atom energies cancel (|E| <
    0.1 sum|E_i|) also bound the error relative to sum|E_i|."""
    E_gpu, E_ref = np.asarray(E_gpu), np.asarray(E_ref)
    scale = np.maximum(np.abs(E_ref), 1e-300)
    err = np.abs(E_gpu - E_ref)
    ok = err <= rel * scale
    if not np.all(ok):
        # fall back to the per-atom scale only where the total cancels
        tot = np.abs(Ei_ref).sum() if Ei_ref is not None else 0.0
        assert np.all(err <= rel * np.maximum(scale, 0.1 * tot)), (E_gpu, E_ref, err)
    return float(np.max(err / scale))


def check_forces(F_gpu, F_ref, abs_tol=1e-4, rel_tol=1e-3):
    """Max-abs error <= abs_tol (eV/A) and <= rel_tol * max|F_ref|."""
    err = np.abs(np.asarray(F_gpu) - np.asarray(F_ref)).max()
    fmax = np.abs(F_ref).max()
    assert err <= abs_tol, (err, fmax)
    assert err <= rel_tol * fmax, (err, fmax, err / fmax)
    return float(err), float(err / fmax)
