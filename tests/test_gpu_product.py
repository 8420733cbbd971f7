"""GPU product block (MACE-style symmetric contraction of body order 2,
correlation 2) vs the FP64 oracle: energies <= 1e-5 relative, forces <= 1e-4
eV/A max-abs and <= 1e-3 of the largest force."""
import numpy as np
import pytest

import synth
from oracle import model as om
from tests.gpu_util import check_energy, check_forces, device, gpu_energy_forces, model, say

pytestmark = pytest.mark.gpu


def _cfg(lmax, C, layers=2, n_species=4, cutoff=5.0):
    return synth.ModelConfig(lmax=lmax, channels=C, layers=layers, n_species=n_species, cutoff=cutoff,
                             avg_neighbors=synth.nominal_neighbors(0.1, cutoff), correlation=2)


def _oracle(cfg, seed_key, b, chunk=None):
    return om.energy_forces(om.Model(cfg, synth.model_weights(cfg, seed_key)), b, edge_chunk=chunk)


def test_tiny_cluster_product_block():
    _, b = synth.tiny_config()
    cfg = _cfg(2, 32, n_species=3)
    say("product block tiny cluster")
    E, F, Ei, _ = gpu_energy_forces(model(cfg, 81), b)
    Er, Fr, Eir = _oracle(cfg, 81, b)
    e = check_energy(E, Er, Eir)
    f = check_forces(F, Fr)
    np.testing.assert_allclose(Ei, Eir, atol=1e-6 * np.abs(Eir).max())
    say(f"  energy rel err {e:.2e}; force err {f[0]:.2e} eV/A ({f[1]:.2e} of max)")


def test_packed_periodic_batch_lmax3():
    _, b, _, _ = synth.differentiation_config(5, 20, 110)
    cfg = _cfg(3, 64, n_species=5)
    say(f"product block packed batch N={b.n_atoms}")
    E, F, Ei, _ = gpu_energy_forces(model(cfg, 82), b, skin=0.5)
    Er, Fr, Eir = _oracle(cfg, 82, b)
    for s in range(b.n_structures):
        a, z = b.offsets[s], b.offsets[s + 1]
        check_energy(E[s:s + 1], Er[s:s + 1], Eir[a:z])
    f = check_forces(F, Fr)
    say(f"  force err {f[0]:.2e} eV/A ({f[1]:.2e} of max)")


def test_three_layers_128_channels():
    # the middle layer's product block has every output order (15 couplings)
    cfg = _cfg(3, 128, layers=3)
    b = synth.jittered_lattice(120, 0.1, 0.3, 4, np.random.default_rng(83))
    say(f"product block 3 layers N={b.n_atoms}")
    E, F, Ei, _ = gpu_energy_forces(model(cfg, 84), b, skin=1.0)
    Er, Fr, Eir = _oracle(cfg, 84, b, chunk=4096)
    check_energy(E, Er, Eir)
    f = check_forces(F, Fr)
    say(f"  force err {f[0]:.2e} eV/A ({f[1]:.2e} of max)")


def test_factorised_first_layer_agrees_with_the_per_edge_path():
    cfg = _cfg(3, 64)
    b = synth.jittered_lattice(90, 0.1, 0.3, 4, np.random.default_rng(85))
    m = model(cfg, 86)
    E0, F0, _, _ = gpu_energy_forces(m, b)
    m.set_flags(unfactorised_first_layer=True)
    E1, F1, _, _ = gpu_energy_forces(m, b)
    assert abs(E0[0] - E1[0]) <= 1e-6 * abs(E0[0])
    assert np.abs(F0 - F1).max() <= 1e-6 + 1e-4 * np.abs(F0).max()


def test_alone_equals_packed_bitwise():
    rng = np.random.default_rng(87)
    parts = [synth.jittered_lattice(n, 0.1, 0.3, 4, rng) for n in (30, 75, 52)]
    b = synth.concat(parts)
    cfg = _cfg(3, 64)
    m = model(cfg, 88)
    E, F, _, _ = gpu_energy_forces(m, b)
    for s, p in enumerate(parts):
        Es, Fs, _, _ = gpu_energy_forces(m, p)
        a, z = b.offsets[s], b.offsets[s + 1]
        assert Es[0] == E[s]
        assert np.array_equal(Fs, F[a:z])


def test_energy_weight_gradient_against_oracle():
    # dE/dtheta of the product-block model through e3mi_param_grad (gF = 0),
    # against the oracle's loss (E - (E_o - 1/2))^2, whose gradient is dE/dtheta
    import torch
    cfg = _cfg(2, 32, n_species=3)
    _, b = synth.tiny_config()
    m = model(cfg, 89)
    pos = torch.tensor(b.pos, dtype=torch.float64, device=device())
    sp = torch.tensor(b.species, dtype=torch.int32, device=device())
    g = m.build_graph(b.offsets, pos, sp, b.cell, b.pbc, cfg.cutoff, 0.0)
    gE = torch.ones(1, dtype=torch.float64, device=device())
    gF = torch.zeros((b.n_atoms, 3), dtype=torch.float32, device=device())
    grad = m.param_grad(g, pos, gE, gF).cpu().numpy()
    om_m = om.Model(cfg, synth.model_weights(cfg, 89))
    E_o = om.energy(om_m, b)
    _, go = om.loss_and_grads(om_m, b, E_o - 0.5, np.zeros((b.n_atoms, 3)), 1.0, 0.0)
    ref = synth.flatten_weights(cfg, go)
    err = np.linalg.norm(grad - ref) / np.linalg.norm(ref)
    say(f"  dE/dtheta rel L2 err {err:.2e}")
    assert err <= 1e-4
