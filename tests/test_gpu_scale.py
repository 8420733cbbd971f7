"""Layers evaluated in receiver chunks (bounded per-edge memory) and the
100,000-atom, 3-layer precision-at-scale configuration (r_c 6 A, l_max 3,
128 channels): chunked = unchunked bitwise (radial adjoint per edge; per
edge pair, the default for unchunked layers, to rounding); the independent 2,000-atom
sub-box against the FP64 oracle in FP32 (energy <= 1e-5 relative, forces
<= 1e-4 eV/A and <= 1e-3 of the largest force) and in BF16 (errors stated,
bounded loosely); the full box in both precisions."""
import os

import numpy as np
import pytest

import synth
from tests.gpu_util import check_atom_energies, check_energy, check_forces, gpu_energy_forces, model, record, say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("correlation,precision", [(1, 0), (2, 0), (1, 1)])
def test_chunked_layers_equal_unchunked(correlation, precision):
    cfg = synth.ModelConfig(lmax=3, channels=64, layers=3, n_species=4, cutoff=5.0,
                            avg_neighbors=synth.nominal_neighbors(0.1, 5.0), correlation=correlation)
    b = synth.jittered_lattice(400, 0.1, 0.3, 4, np.random.default_rng(121))
    m = model(cfg, 122, precision=precision)
    # unchunked layers run the radial adjoint per edge pair by default (forces
    # equal to rounding); per edge, as chunked layers do, they give the same bits
    Ep, Fp, Eip, _ = gpu_energy_forces(m, b, skin=1.0)
    m.set_flags(radial_per_edge=True)
    E0, F0, Ei0, _ = gpu_energy_forces(m, b, skin=1.0)
    assert np.array_equal(E0, Ep) and np.array_equal(Ei0, Eip)
    assert np.abs(Fp - F0).max() <= (1e-5 if precision == 0 else 1e-2) * np.abs(F0).max()
    m.set_r_chunk_bytes(1 << 20)  # 1 MiB: 1 MiB / (23 paths x 64 ch x 4 B) = 178 edges per chunk
    for flags in ({"radial_per_edge": True}, {}):   # chunked layers ignore the pair mode
        m.set_flags(**flags)
        for keep in (0, 1 << 40):     # R recomputed chunk by chunk in the adjoint / kept whole
            m.set_r_keep_bytes(keep)
            E1, F1, Ei1, _ = gpu_energy_forces(m, b, skin=1.0)
            say(f"chunked (correlation {correlation}, precision {precision}, keep {keep}, flags {flags}): "
                f"max |dF| {np.abs(F1 - F0).max():.1e}")
            assert np.array_equal(E0, E1) and np.array_equal(F0, F1) and np.array_equal(Ei0, Ei1)


@pytest.mark.parametrize("chunk_bytes", [None, 64 << 20])
def test_scale_subbox_against_oracle(chunk_bytes):
    ref = np.load(os.path.join(HERE, "golden", "scale_sub_2000.npz"))
    cfg, b = synth.scale_subbox()
    m32, m16 = model(cfg, 5), model(cfg, 5, precision=1)
    if chunk_bytes:
        m32.set_r_chunk_bytes(chunk_bytes)
        m16.set_r_chunk_bytes(chunk_bytes)
    E32, F32, Ei32, _ = gpu_energy_forces(m32, b, skin=1.0)
    E16, F16, Ei16, _ = gpu_energy_forces(m16, b, skin=1.0)
    e = check_energy(E32, ref["energy"], ref["atom_energy"])
    ea = check_atom_energies(Ei32, ref["atom_energy"])
    f = check_forces(F32, ref["forces"])
    fmax = np.abs(ref["forces"]).max()
    e16 = abs(E16[0] - ref["energy"][0]) / b.n_atoms
    ea16 = np.abs(Ei16 - ref["atom_energy"]).max() / np.abs(ref["atom_energy"]).max()
    f16 = np.abs(F16 - ref["forces"]).max() / fmax
    record("bf16", energy_eV_per_atom=float(e16), atom_energy_rel_to_max=float(ea16), force_rel_to_max=float(f16))
    say(f"sub-box (chunk {chunk_bytes}): FP32 energy rel err {e:.2e}, atom energies {ea:.2e} of max, force err "
        f"{f[0]:.2e} eV/A; BF16 energy err {e16:.2e} eV/atom, force err {f16:.2e} of max |F|")
    assert e16 < 1e-3 and f16 < 5e-2


def test_hundred_thousand_atoms_fp32_and_bf16():
    import torch
    cfg, b = synth.scale_config()
    say(f"100k box: N={b.n_atoms}")
    # one model at a time: each keeps about 120 GB of per-edge R
    m = model(cfg, 5)
    E32, F32, _, g = gpu_energy_forces(m, b, skin=0.0)
    n_edges = g.last_edge_count()
    g.close()
    m.close()
    torch.cuda.empty_cache()
    m = model(cfg, 5, precision=1)
    E16, F16, _, g = gpu_energy_forces(m, b, skin=0.0)
    g.close()
    m.close()
    fmax = np.abs(F32).max()
    say(f"  edges {n_edges}; E32 {E32[0]:.6f}, E16 {E16[0]:.6f} eV; |sum F| {np.abs(F32.sum(0)).max():.2e}; "
        f"BF16 vs FP32: {abs(E16[0] - E32[0]) / b.n_atoms:.2e} eV/atom, "
        f"{np.abs(F16 - F32).max() / fmax:.2e} of max |F|")
    assert 8.5e6 < n_edges < 9.6e6
    assert np.isfinite(E32).all() and np.isfinite(F32).all()
    assert np.abs(F32.sum(0)).max() <= 1e-3 * fmax * np.sqrt(b.n_atoms)
    assert abs(E16[0] - E32[0]) / b.n_atoms < 1e-3 and np.abs(F16 - F32).max() < 5e-2 * fmax
