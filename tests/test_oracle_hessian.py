"""Pins of the oracle's Hessian-vector product (§5.2): central differences of
the forces, symmetry, the translation and rotation identities, locality per
structure and rotation covariance."""
import numpy as np
import pytest

import synth
from oracle import cg
from oracle import model as om


@pytest.fixture(scope="module")
def system():
    cfg = synth.ModelConfig(lmax=3, channels=8, layers=2, n_species=3, cutoff=5.0, avg_neighbors=10.0)
    m = om.Model(cfg, synth.model_weights(cfg, 91))
    b = synth.uniform_cluster(14, 6.5, 0.9, 3, np.random.default_rng(92))
    return m, b


def _batch(b, pos):
    return synth.Batch(np.asarray(pos, dtype=np.float64), b.species, b.cell, b.pbc, b.offsets, b.charge)


def test_matches_central_differences_of_forces(system):
    m, b = system
    v = np.random.default_rng(93).normal(size=b.pos.shape)
    hv = om.hessian_vector(m, b, v)
    h = 1e-4
    Fp = om.energy_forces(m, _batch(b, b.pos + h * v))[1]
    Fm = om.energy_forces(m, _batch(b, b.pos - h * v))[1]
    fd = -(Fp - Fm) / (2 * h)
    assert np.abs(hv - fd).max() < 1e-6 * max(1.0, np.abs(hv).max())


def test_is_symmetric(system):
    m, b = system
    rng = np.random.default_rng(94)
    u, v = rng.normal(size=b.pos.shape), rng.normal(size=b.pos.shape)
    assert abs(np.sum(u * om.hessian_vector(m, b, v)) - np.sum(v * om.hessian_vector(m, b, u))) < 1e-12


def test_uniform_translation_is_a_null_vector(system):
    m, b = system
    v = np.tile(np.array([0.3, -1.2, 0.7]), (b.n_atoms, 1))
    assert np.abs(om.hessian_vector(m, b, v)).max() < 1e-12


def test_rotation_generator_gives_the_rotated_gradient(system):
    # E(R r) = E(r) for all rotations  =>  H (w x r) = w x grad E = -(w x F)
    m, b = system
    w = np.array([0.4, -0.9, 0.25])
    _, F, _ = om.energy_forces(m, b)
    hv = om.hessian_vector(m, b, np.cross(w, b.pos))
    assert np.abs(hv + np.cross(w, F)).max() < 1e-12


def test_structures_are_independent():
    cfg = synth.ModelConfig(lmax=2, channels=8, layers=2, n_species=3, cutoff=5.0, avg_neighbors=10.0)
    m = om.Model(cfg, synth.model_weights(cfg, 95))
    rng = np.random.default_rng(96)
    parts = [synth.uniform_cluster(n, 6.0, 0.9, 3, rng) for n in (8, 11)]
    b = synth.concat(parts)
    v = rng.normal(size=b.pos.shape)
    hv = om.hessian_vector(m, b, v)
    np.testing.assert_allclose(hv[:8], om.hessian_vector(m, parts[0], v[:8]), atol=1e-13)
    np.testing.assert_allclose(hv[8:], om.hessian_vector(m, parts[1], v[8:]), atol=1e-13)


def test_full_hessian_is_symmetric_and_translation_invariant():
    # A Hessian assembled from 3n products is symmetric and its rows sum to
    # zero over atoms for each Cartesian column (translation invariance).
    cfg = synth.ModelConfig(lmax=2, channels=8, layers=2, n_species=3, cutoff=5.0, avg_neighbors=10.0)
    m = om.Model(cfg, synth.model_weights(cfg, 97))
    b = synth.uniform_cluster(6, 4.5, 1.0, 3, np.random.default_rng(98))
    n = b.n_atoms
    H = np.zeros((3 * n, 3 * n))
    for k in range(3 * n):
        e = np.zeros(3 * n)
        e[k] = 1.0
        H[:, k] = om.hessian_vector(m, b, e.reshape(n, 3)).reshape(-1)
    assert np.abs(H - H.T).max() < 1e-12
    for a in range(3):
        assert np.abs(H[:, a::3].sum(axis=1)).max() < 1e-12


def test_rotating_the_structure_rotates_the_product():
    cfg = synth.ModelConfig(lmax=3, channels=8, layers=2, n_species=3, cutoff=5.0, avg_neighbors=10.0)
    m = om.Model(cfg, synth.model_weights(cfg, 99))
    b = synth.uniform_cluster(10, 6.0, 0.9, 3, np.random.default_rng(100))
    v = np.random.default_rng(101).normal(size=b.pos.shape)
    R = cg.rotation(0.3, 1.1, 2.0)
    hv = om.hessian_vector(m, b, v)
    hvr = om.hessian_vector(m, _batch(b, b.pos @ R.T), v @ R.T)
    assert np.abs(hvr - hv @ R.T).max() < 1e-11
