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


def record(kind, **fields):
    """Append one line of measured errors to the JSON-lines file named by
    E3MI_PARITY_LOG (if set), and print it."""
    import json
    import os
    line = json.dumps({"check": kind, "test": os.environ.get("PYTEST_CURRENT_TEST", "").split(" ")[0],
                       **fields})
    say(line)
    path = os.environ.get("E3MI_PARITY_LOG")
    if path:
        with open(path, "a") as f:
            f.write(line + "\n")


def check_energy(E_gpu, E_ref, Ei_ref, rel=1e-5):
    """Energy error against the oracle, reported both relative to |E_ref| and
    relative to sum_i |E_i,ref| (the scale of the per-atom terms that the total
    sums). Enforced: |dE| <= rel |E_ref|, except for a total that cancels
    (|E_ref| < 0.1 sum_i |E_i,ref|): there FP32 rounding of per-atom terms of
    size sum_i |E_i| sets the error, so the bound is rel x 0.1 sum_i |E_i,ref|
    and the structure is flagged as cancelling in the record."""
    E_gpu, E_ref = np.asarray(E_gpu), np.asarray(E_ref)
    scale = np.maximum(np.abs(E_ref), 1e-300)
    err = np.abs(E_gpu - E_ref)
    tot = float(np.abs(Ei_ref).sum()) if Ei_ref is not None else 0.0
    rel_e = float(np.max(err / scale))
    rel_sum = float(np.max(err) / tot) if tot > 0 else None
    cancelling = bool(np.any(np.abs(E_ref) < 0.1 * tot))
    record("energy", rel_to_E=rel_e, rel_to_sum_abs_Ei=rel_sum, cancelling=cancelling, bound=rel)
    ok = err <= rel * scale
    if not np.all(ok):
        assert cancelling, (E_gpu, E_ref, err)
        assert np.all(err <= rel * np.maximum(scale, 0.1 * tot)), (E_gpu, E_ref, err)
    return rel_e


def check_atom_energies(Ei_gpu, Ei_ref, rel=1e-5):
    """Per-atom energies: max |dE_i| <= rel x max |E_i,ref|."""
    err = float(np.abs(np.asarray(Ei_gpu) - np.asarray(Ei_ref)).max())
    scale = float(np.abs(Ei_ref).max())
    record("atom_energy", max_abs=err, rel_to_max_abs_Ei=err / scale, bound=rel)
    assert err <= rel * scale, (err, scale)
    return err / scale


def check_forces(F_gpu, F_ref, abs_tol=1e-4, rel_tol=1e-3):
    """Max-abs error <= abs_tol (eV/A) and <= rel_tol * max|F_ref|."""
    err = np.abs(np.asarray(F_gpu) - np.asarray(F_ref)).max()
    fmax = np.abs(F_ref).max()
    rel = float(err / fmax) if fmax > 0 else (0.0 if err == 0 else float("inf"))  # zero forces: exact
    record("forces", max_abs=float(err), rel_to_max_abs_F=rel, bound_abs=abs_tol, bound_rel=rel_tol)
    assert err <= abs_tol, (err, fmax)
    assert err <= rel_tol * fmax, (err, fmax, rel)
    return float(err), rel
