"""GPU energy + forces vs the FP64 oracle (FP32 path).

Tolerances: energy <= 1e-5 relative and forces <= 1e-4 eV/A max-abs against
the FP64 oracle, plus max-abs force error <= 1e-3 of the largest force (the
random-init model has forces of only ~1e-3 eV/A, so the absolute bound alone
would be weak).
"""
import os

import numpy as np
import pytest

import synth
from oracle import model as om
from tests.gpu_util import check_energy, check_forces, gpu_energy_forces, model, say, to_dev

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _oracle(cfg, seed_key, b, chunk=None):
    return om.energy_forces(om.Model(cfg, synth.model_weights(cfg, seed_key)), b, edge_chunk=chunk)


@pytest.mark.parametrize("skin", [0.0, 1.0])
def test_tiny_cluster(skin):
    cfg, b = synth.tiny_config()
    say(f"tiny cluster skin={skin}")
    E, F, Ei, _ = gpu_energy_forces(model(cfg, 1), b, skin=skin)
    Er, Fr, Eir = _oracle(cfg, 1, b)
    e = check_energy(E, Er, Eir)
    f = check_forces(F, Fr)
    np.testing.assert_allclose(Ei, Eir, atol=1e-6 * np.abs(Eir).max())
    say(f"  energy rel err {e:.2e}; force err {f[0]:.2e} eV/A ({f[1]:.2e} of max)")


def test_packed_periodic_batch():
    # small periodic boxes (shorter than 2 r_c: several images per pair), l_max 3, 64 channels
    cfg, b, _, _ = synth.differentiation_config(6, 20, 120)
    say(f"packed batch N={b.n_atoms}")
    E, F, Ei, _ = gpu_energy_forces(model(cfg, 3), b, skin=0.5)
    Er, Fr, Eir = _oracle(cfg, 3, b)
    for s in range(b.n_structures):
        a, z = b.offsets[s], b.offsets[s + 1]
        check_energy(E[s:s + 1], Er[s:s + 1], Eir[a:z])
    check_forces(F, Fr)


@pytest.mark.parametrize("unfactorised", [False, True])
def test_single_layer_model(unfactorised):
    # one interaction layer: it is both the first layer (embedding input) and
    # the scalar-output last layer, with its own gate before the readout
    cfg = synth.ModelConfig(lmax=3, channels=32, layers=1, n_species=3, cutoff=5.0,
                            avg_neighbors=synth.nominal_neighbors(0.1, 5.0))
    b = synth.jittered_lattice(120, 0.1, 0.3, 3, np.random.default_rng(47))
    m = model(cfg, 48)
    if unfactorised:
        m.set_flags(unfactorised_first_layer=True)
    E, F, Ei, _ = gpu_energy_forces(m, b, skin=1.0)
    Er, Fr, Eir = _oracle(cfg, 48, b)
    e = check_energy(E, Er, Eir)
    f = check_forces(F, Fr)
    say(f"single layer (unfactorised {unfactorised}): energy rel err {e:.2e}, force err {f[0]:.2e} eV/A")


def test_three_layer_full_middle_layer():
    # 3 layers: the middle layer runs all 23 paths of l_max 3.
    cfg = synth.ModelConfig(lmax=3, channels=128, layers=3, n_species=4, cutoff=6.0,
                            avg_neighbors=synth.nominal_neighbors(0.1, 6.0))
    b = synth.jittered_lattice(150, 0.1, 0.3, 4, np.random.default_rng(41))
    say(f"3-layer N={b.n_atoms}")
    E, F, Ei, _ = gpu_energy_forces(model(cfg, 5), b, skin=1.0)
    Er, Fr, Eir = _oracle(cfg, 5, b, chunk=4096)
    check_energy(E, Er, Eir)
    check_forces(F, Fr)


def test_lmax2_open_cluster_batch():
    cfg = synth.ModelConfig(lmax=2, channels=64, layers=3, n_species=3, cutoff=5.0, avg_neighbors=8.0)
    rng = np.random.default_rng(42)
    b = synth.concat([synth.uniform_cluster(n, 9.0, 1.0, 3, rng) for n in (5, 30, 17)])
    E, F, Ei, _ = gpu_energy_forces(model(cfg, 6), b, skin=0.3)
    Er, Fr, Eir = _oracle(cfg, 6, b)
    for s in range(b.n_structures):
        a, z = b.offsets[s], b.offsets[s + 1]
        check_energy(E[s:s + 1], Er[s:s + 1], Eir[a:z])
    check_forces(F, Fr)


def test_single_structure_3000_atoms_golden():
    path = os.path.join(HERE, "golden", "single_3000.npz")
    ref = np.load(path)
    cfg, b = synth.single_config()
    say("single structure 3000 atoms (stored oracle result)")
    E, F, Ei, g = gpu_energy_forces(model(cfg, 2), b, skin=1.0)
    e = check_energy(E, ref["energy"], ref["atom_energy"])
    f = check_forces(F, ref["forces"])
    np.testing.assert_allclose(Ei, ref["atom_energy"], atol=1e-5 * np.abs(ref["atom_energy"]).max())
    say(f"  energy rel err {e:.2e}; force err {f[0]:.2e} eV/A ({f[1]:.2e} of max)")


def test_net_force_vanishes_and_repeatable():
    import torch
    cfg, b = synth.single_config(n=800)
    m = model(cfg, 2)
    pos, sp = to_dev(b)
    g = m.build_graph(b.offsets, pos, sp, b.cell, b.pbc, cfg.cutoff, 1.0)
    E1, F1, _ = m.energy_forces(g, pos)
    E2, F2, _ = m.energy_forces(g, pos)
    torch.cuda.synchronize()
    assert torch.equal(E1, E2) and torch.equal(F1, F2)
    F = F1.double().cpu().numpy()
    assert np.abs(F.sum(0)).max() < 1e-5 * np.abs(F).max() * np.sqrt(b.n_atoms)


def test_packing_invariance_bitwise():
    # a structure evaluated alone and inside a packed batch gives identical bits
    import torch
    cfg, b, _, _ = synth.differentiation_config(5, 30, 90)
    m = model(cfg, 3)
    E, F, Ei, _ = gpu_energy_forces(m, b, skin=0.5)
    for s in (0, 3):
        one = b.structure(s)
        E1, F1, Ei1, _ = gpu_energy_forces(m, one, skin=0.5)
        a, z = b.offsets[s], b.offsets[s + 1]
        assert E1[0] == E[s]
        assert np.array_equal(F1, F[a:z])
        assert np.array_equal(Ei1, Ei[a:z])


def test_translation_and_image_shift_invariance():
    import torch
    cfg, b, _, _ = synth.differentiation_config(2, 40, 60)
    m = model(cfg, 3)
    E0, F0, _, _ = gpu_energy_forces(m, b, skin=0.5)
    L = b.cell[:, 0, 0]
    owner = np.repeat(np.arange(b.n_structures), np.diff(b.offsets))
    k = np.random.default_rng(5).integers(-2, 3, size=(b.n_atoms, 3))
    moved = synth.Batch(b.pos + k * L[owner][:, None], b.species, b.cell, b.pbc, b.offsets)
    E1, F1, _, _ = gpu_energy_forces(m, moved, skin=0.5)
    np.testing.assert_allclose(E1, E0, rtol=1e-6)
    np.testing.assert_allclose(F1, F0, atol=1e-6 * np.abs(F0).max())


def test_bf16_mode_errors_against_oracle():
    # BF16 operands for the radial-MLP and channel-mix GEMMs (FP32 accumulation);
    # the errors are reported and only bounded loosely.
    ref = np.load(os.path.join(HERE, "golden", "single_3000.npz"))
    cfg, b = synth.single_config()
    E32, F32, _, _ = gpu_energy_forces(model(cfg, 2), b, skin=1.0)
    E16, F16, _, _ = gpu_energy_forces(model(cfg, 2, precision=1), b, skin=1.0)
    fmax = np.abs(ref["forces"]).max()
    e16 = abs(E16[0] - ref["energy"][0]) / abs(ref["energy"][0])
    f16 = np.abs(F16 - ref["forces"]).max() / fmax
    e32 = abs(E32[0] - ref["energy"][0]) / abs(ref["energy"][0])
    f32 = np.abs(F32 - ref["forces"]).max() / fmax
    per_atom = abs(E16[0] - ref["energy"][0]) / b.n_atoms
    say(f"BF16: energy rel err {e16:.2e} ({per_atom:.2e} eV/atom), force err {f16:.2e} of max |F|; "
        f"FP32: {e32:.2e}, {f32:.2e}")
    # rounding the weights to BF16 shifts every atom's energy alike, so the
    # total error grows with N: bound it per atom
    assert per_atom < 1e-3 and f16 < 5e-2
    assert not np.array_equal(F16, F32)


def test_first_layer_factorisation_matches_per_edge_path():
    import torch
    cfg, b = synth.single_config(n=700)
    m = model(cfg, 2)
    E1, F1, Ei1, _ = gpu_energy_forces(m, b, skin=1.0)
    m.set_flags(unfactorised_first_layer=True)
    E2, F2, Ei2, _ = gpu_energy_forces(m, b, skin=1.0)
    assert abs(E1[0] - E2[0]) <= 1e-6 * abs(E2[0])
    assert np.abs(F1 - F2).max() <= 1e-4 * np.abs(F2).max()
    assert not np.array_equal(F1, F2)  # two different evaluation orders


@pytest.mark.parametrize("n_species", [1, 5, 8])
def test_first_layer_factorisation_other_species_counts(n_species):
    # one species (every column of the (component, species) axis kept), an odd
    # count and the largest the factorisation holds in LDS
    cfg = synth.ModelConfig(lmax=3, channels=32, layers=2, n_species=n_species, cutoff=5.0,
                            avg_neighbors=synth.nominal_neighbors(0.1, 5.0))
    b = synth.jittered_lattice(300, 0.1, 0.3, n_species, np.random.default_rng(130 + n_species))
    m = model(cfg, 131)
    E1, F1, _, _ = gpu_energy_forces(m, b, skin=1.0)
    m.set_flags(unfactorised_first_layer=True)
    E2, F2, _, _ = gpu_energy_forces(m, b, skin=1.0)
    say(f"species {n_species}: |dE| {abs(E1[0] - E2[0]):.1e}, max |dF| {np.abs(F1 - F2).max():.1e}")
    assert abs(E1[0] - E2[0]) <= 1e-6 * abs(E2[0])
    assert np.abs(F1 - F2).max() <= 1e-4 * np.abs(F2).max()
    assert not np.array_equal(F1, F2)


@pytest.mark.parametrize("lmax,channels", [(3, 128), (3, 64), (2, 32)])
def test_fused_last_layer_matches_unfused_path(lmax, channels):
    cfg = synth.ModelConfig(lmax=lmax, channels=channels, layers=2, n_species=4, cutoff=5.0, avg_neighbors=52.36)
    _, b = synth.single_config(n=500)
    m = model(cfg, 5)
    say(f"fused last layer l_max {lmax} C {channels}")
    m.set_flags(fused_last_layer=True)
    E1, F1, Ei1, _ = gpu_energy_forces(m, b, skin=1.0)
    m.set_flags()
    E2, F2, Ei2, _ = gpu_energy_forces(m, b, skin=1.0)
    assert not np.array_equal(F1, F2)  # the two evaluations really differ in order
    assert np.abs(Ei1 - Ei2).max() <= 1e-5 * np.abs(Ei2).max()
    assert abs(E1[0] - E2[0]) <= 1e-6 * abs(E2[0])
    assert np.abs(F1 - F2).max() <= 1e-4 * np.abs(F2).max()
