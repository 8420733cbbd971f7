"""Pins of the oracle's charge head, charge correction and soft-core Coulomb
energy (§5.1)."""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.distance import pdist

import synth
from oracle import model as om


def _pair_energy(r, q1, q2, r0):
    pos = torch.tensor([[0.0, 0.0, 0.0], [r, 0.0, 0.0]], dtype=torch.float64)
    q = torch.tensor([q1, q2], dtype=torch.float64)
    return float(om.coulomb_atom_energies(pos, q, np.array([0, 2]), r0).sum())


def test_coulomb_constant_is_e2_over_4pi_eps0():
    # CODATA: e = 1.602176634e-19 C, eps0 = 8.8541878128e-12 F/m; eV * angstrom.
    e, eps0 = 1.602176634e-19, 8.8541878128e-12
    assert abs(om.K_E - e / (4 * math.pi * eps0) / 1e-10) < 1e-6


@pytest.mark.parametrize("r", [2.5, 4.0, 11.0])
def test_two_charges_beyond_soft_core_is_plain_coulomb(r):
    # chi(r) = r for r >= r0: the textbook pair energy k_e q1 q2 / r.
    assert abs(_pair_energy(r, 0.4, -0.7, 2.0) - om.K_E * 0.4 * -0.7 / r) < 1e-12


def test_two_charges_deep_inside_soft_core_tend_to_the_regular_form():
    # For r -> 0 the switch tends to 1 and the kernel to 1/sqrt(r^2+1), finite
    # at contact; what is left of the bare 1/r term is (1 - phi)/r ~ 10 r^2/r0^3.
    r0 = 2.0
    for r in (1e-4, 1e-3, 1e-2):
        expect = om.K_E * 0.5 * 0.5 / math.sqrt(r * r + 1.0)
        assert abs(_pair_energy(r, 0.5, 0.5, r0) - expect) < om.K_E * 0.25 * 11 * r * r / r0 ** 3


def test_soft_core_kernel_is_c1_at_the_radius():
    r0 = 2.0
    x = torch.tensor([r0 - 1e-7, r0, r0 + 1e-7], dtype=torch.float64)
    v = om.inv_chi(x, r0)
    assert abs(float(v[0] - v[2])) < 1e-6
    assert abs(float(v[1]) - 1 / r0) < 1e-15
    # the switch has zero slope at x = 1, so dk/dr matches -1/r^2 from both sides
    xs = torch.tensor([r0 - 1e-6, r0 + 1e-6], dtype=torch.float64, requires_grad=True)
    (g,) = torch.autograd.grad(om.inv_chi(xs, r0).sum(), xs)
    assert np.allclose(g.numpy(), -1.0 / r0 ** 2, atol=1e-5)


def test_switch_polynomial_end_points():
    x = torch.tensor([0.0, 0.5, 1.0, 1.5], dtype=torch.float64)
    assert torch.allclose(om.soft_core_switch(x), torch.tensor([1.0, 0.5, 0.0, 0.0], dtype=torch.float64))


def test_many_charges_equal_sum_over_pairs():
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 8, (9, 3))
    q = rng.normal(size=9)
    r0 = 1.5
    E = float(om.coulomb_atom_energies(torch.from_numpy(x), torch.from_numpy(q), np.array([0, 9]), r0).sum())
    d = pdist(x)                            # i < j order
    qq = np.array([q[i] * q[j] for i in range(9) for j in range(i + 1, 9)])
    xs = d / r0
    phi = np.where(xs < 1, 1 - 6 * xs ** 5 + 15 * xs ** 4 - 10 * xs ** 3, 0.0)
    expect = om.K_E * np.sum(qq * (phi / np.sqrt(d * d + 1) + (1 - phi) / d))
    assert abs(E - expect) < 1e-10 * abs(expect)


def test_structures_do_not_interact():
    rng = np.random.default_rng(6)
    x = torch.from_numpy(rng.uniform(0, 5, (7, 3)))
    q = torch.from_numpy(rng.normal(size=7))
    both = om.coulomb_atom_energies(x, q, np.array([0, 3, 7]), 2.0)
    a = om.coulomb_atom_energies(x[:3], q[:3], np.array([0, 3]), 2.0)
    b = om.coulomb_atom_energies(x[3:], q[3:], np.array([0, 4]), 2.0)
    assert torch.allclose(both, torch.cat([a, b]), rtol=0, atol=1e-14)


def _coulomb_model(seed=31, lmax=2, C=16):
    cfg = synth.ModelConfig(lmax=lmax, channels=C, layers=2, n_species=3, cutoff=5.0,
                            avg_neighbors=12.0, coulomb=True, soft_core_r0=2.0)
    return cfg, om.Model(cfg, synth.model_weights(cfg, seed))


def _cluster_batch(charges=(0.0, 1.0)):
    rng = np.random.default_rng(32)
    bs = [synth.uniform_cluster(n, 8.0, 0.9, 3, rng) for n in (13, 9)]
    b = synth.concat(bs)
    b.charge = np.array(charges, dtype=np.float64)
    return b


def test_corrected_charges_sum_to_total_charge():
    cfg, m = _coulomb_model()
    b = _cluster_batch((0.0, -2.0))
    h0 = torch.from_numpy(np.random.default_rng(2).normal(size=(b.n_atoms, cfg.channels)))
    sp = torch.from_numpy(b.species.astype(np.int64))
    q = om.charges(m, h0, sp, b.offsets, b.charge)
    assert abs(float(q[:13].sum())) < 1e-12
    assert abs(float(q[13:].sum()) + 2.0) < 1e-12
    # the correction is a uniform shift: differences between atoms are those of the raw head
    raw = h0 @ m.w["qhead"] + m.w["qbias"][sp]
    assert torch.allclose((q - raw)[:13], (q - raw)[0].expand(13), atol=1e-14)


def test_coulomb_energy_adds_to_the_short_range_model():
    # With a zero feature head the charges are the species offsets shifted so
    # that each structure carries its total charge: the energy difference to
    # the short-range model is then a plain pair sum over known charges.
    cfg = synth.ModelConfig(lmax=2, channels=16, layers=2, n_species=3, cutoff=5.0,
                            avg_neighbors=12.0, coulomb=True, soft_core_r0=2.0)
    w = synth.model_weights(cfg, 31)
    w["qhead"] = np.zeros_like(w["qhead"])
    w["qbias"] = np.array([0.3, -0.45, 0.1])
    b = _cluster_batch((0.0, 1.0))
    E, _, Ei = om.energy_forces(om.Model(cfg, w), b)
    cfg0 = synth.ModelConfig(lmax=2, channels=16, layers=2, n_species=3, cutoff=5.0, avg_neighbors=12.0)
    w0 = {k: v for k, v in w.items() if k not in ("qhead", "qbias")}
    E0, _, _ = om.energy_forces(om.Model(cfg0, w0), b)
    for s, Q in enumerate((0.0, 1.0)):
        a0, a1 = b.offsets[s], b.offsets[s + 1]
        q = w["qbias"][b.species[a0:a1]]
        q = q - (q.sum() - Q) / (a1 - a0)
        d = pdist(b.pos[a0:a1])
        n = a1 - a0
        qq = np.array([q[i] * q[j] for i in range(n) for j in range(i + 1, n)])
        x = np.minimum(d / 2.0, 1.0)
        phi = 1 - 6 * x ** 5 + 15 * x ** 4 - 10 * x ** 3
        expect = om.K_E * np.sum(qq * (phi / np.sqrt(d * d + 1) + (1 - phi) / d))
        assert abs((E[s] - E0[s]) - expect) < 1e-10 * max(1.0, abs(expect))
    assert np.isclose(Ei.sum(), E.sum(), rtol=1e-13)


def test_missing_total_charge_means_neutral():
    cfg, m = _coulomb_model()
    b = _cluster_batch((0.0, 0.0))
    bn = synth.Batch(b.pos, b.species, b.cell, b.pbc, b.offsets, None)
    assert np.array_equal(om.energy(m, b), om.energy(m, bn))


def test_forces_are_minus_gradient_by_finite_differences():
    cfg, m = _coulomb_model()
    b = _cluster_batch((0.0, 1.0))
    E, F, _ = om.energy_forces(m, b)
    h = 1e-5
    for (i, k) in [(0, 0), (5, 2), (14, 1), (21, 0)]:
        bp = synth.Batch(b.pos.copy(), b.species, b.cell, b.pbc, b.offsets, b.charge)
        bm = synth.Batch(b.pos.copy(), b.species, b.cell, b.pbc, b.offsets, b.charge)
        bp.pos[i, k] += h
        bm.pos[i, k] -= h
        fd = -(om.energy(m, bp).sum() - om.energy(m, bm).sum()) / (2 * h)
        assert abs(fd - F[i, k]) < 1e-6 * max(1.0, abs(F[i, k]))


def test_rotation_and_translation_invariant():
    cfg, m = _coulomb_model(lmax=3)
    b = _cluster_batch()
    E, F, _ = om.energy_forces(m, b)
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    br = synth.Batch(b.pos @ Q.T + 1.7, b.species, b.cell, b.pbc, b.offsets, b.charge)
    E2, F2, _ = om.energy_forces(m, br)
    assert np.allclose(E, E2, rtol=1e-12, atol=1e-12)
    assert np.allclose(F @ Q.T, F2, atol=1e-10)


def test_periodic_structures_are_rejected():
    cfg, m = _coulomb_model()
    b = synth.jittered_lattice(16, 0.1, 0.3, 3, np.random.default_rng(3))
    with pytest.raises(ValueError):
        om.energy_forces(m, b)
