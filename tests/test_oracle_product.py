"""Pins of the oracle's product block (MACE's symmetric contraction of body
order 2, correlation 2 in Appendix F): closed forms of single couplings,
CG unitarity, rotation equivariance, reduction to the plain layer, and
finite differences of the whole model."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import cg
from oracle import model as om


def _cfg(lmax=3, C=4, layers=2, correlation=2):
    return synth.ModelConfig(lmax=lmax, channels=C, layers=layers, n_species=2, cutoff=5.0,
                             avg_neighbors=10.0, correlation=correlation)


def _model_with(cfg, w1=None, w2=None, seed=3):
    w = synth.model_weights(cfg, seed)
    if w1 is not None:
        w["sym1_1"] = w1
    if w2 is not None:
        w["sym2_1"] = w2
    return om.Model(cfg, w)


def _features(rng, N, C, lmax):
    return [torch.from_numpy(rng.normal(size=(N, C, 2 * l + 1))) for l in range(lmax + 1)]


def _one_pair(cfg, pair):
    """Weights selecting one product coupling (w2 one-hot, w1 = 0) in layer 1."""
    pairs = synth.product_pairs(cfg, cfg.lmax)
    w2 = np.zeros((cfg.n_species, len(pairs), cfg.channels))
    w2[:, pairs.index(pair), :] = 1.0
    w1 = np.zeros((cfg.n_species, cfg.lmax + 1, cfg.channels))
    return w1, w2


def test_pair_list_is_the_natural_parity_couplings():
    cfg = _cfg()
    assert synth.product_pairs(cfg, 0) == [(0, 0, 0), (1, 1, 0), (2, 2, 0), (3, 3, 0)]
    assert len(synth.product_pairs(cfg, 3)) == 15
    assert (1, 1, 1) not in synth.product_pairs(cfg, 3)  # antisymmetric: vanishes for A (x) A


def test_linear_term_alone_is_the_input():
    cfg = _cfg()
    w1 = np.ones((2, 4, 4))
    w2 = np.zeros((2, 15, 4))
    m = _model_with(cfg, w1, w2)
    At = _features(np.random.default_rng(1), 5, 4, 3)
    B = m.product_basis(1, At, torch.zeros(5, dtype=torch.long))
    for L in range(4):
        assert torch.equal(B[L], At[L])


def test_scalar_times_order_l_is_the_plain_product():
    # CG(0, l, l) is the identity: (a0 (x) a_l)_l = a0 a_l
    cfg = _cfg()
    rng = np.random.default_rng(2)
    At = _features(rng, 6, 4, 3)
    sp = torch.zeros(6, dtype=torch.long)
    for l in (0, 1, 2, 3):
        m = _model_with(cfg, *_one_pair(cfg, (0, l, l)))
        B = m.product_basis(1, At, sp)
        assert torch.allclose(B[l], At[0] * At[l], atol=1e-14)


def test_self_coupling_to_scalar_is_the_norm():
    # (a (x) a)_0 = +-|a|^2 / sqrt(2l+1), one sign per order
    cfg = _cfg()
    At = _features(np.random.default_rng(3), 7, 4, 3)
    sp = torch.zeros(7, dtype=torch.long)
    for l in (1, 2, 3):
        m = _model_with(cfg, *_one_pair(cfg, (l, l, 0)))
        B0 = m.product_basis(1, At, sp)[0][..., 0]
        ratio = B0 / ((At[l] ** 2).sum(-1) / math.sqrt(2 * l + 1))
        assert torch.allclose(ratio.abs(), torch.ones_like(ratio), atol=1e-12)
        assert float(ratio.max() - ratio.min()) < 1e-12


def test_vector_couplings_split_the_square_norm():
    # CG unitarity for two vectors: |(a(x)a)_0|^2 + |(a(x)a)_2|^2 = |a|^4
    # (the L = 1 part is a x a = 0), and |(a(x)a)_2|^2 = 2/3 |a|^4
    cfg = _cfg()
    At = _features(np.random.default_rng(4), 8, 4, 3)
    sp = torch.zeros(8, dtype=torch.long)
    B0 = _model_with(cfg, *_one_pair(cfg, (1, 1, 0))).product_basis(1, At, sp)[0]
    B2 = _model_with(cfg, *_one_pair(cfg, (1, 1, 2))).product_basis(1, At, sp)[2]
    a4 = (At[1] ** 2).sum(-1) ** 2
    assert torch.allclose((B0 ** 2).sum(-1) + (B2 ** 2).sum(-1), a4, atol=1e-12)
    assert torch.allclose((B2 ** 2).sum(-1), a4 * 2 / 3, atol=1e-12)


@pytest.mark.parametrize("seed", [6, 7])
def test_product_basis_is_equivariant(seed):
    cfg = _cfg()
    m = om.Model(cfg, synth.model_weights(cfg, seed))
    rng = np.random.default_rng(seed)
    At = _features(rng, 5, 4, 3)
    sp = torch.from_numpy(rng.integers(0, 2, size=5))
    R = cg.rotation(0.7, 1.9, -0.4)
    D = [torch.from_numpy(cg.wigner_d(l, R)) for l in range(4)]
    B = m.product_basis(1, At, sp)
    Br = m.product_basis(1, [At[l] @ D[l].T for l in range(4)], sp)
    for L in range(4):
        assert torch.allclose(Br[L], B[L] @ D[L].T, atol=1e-12)


def test_identity_block_reduces_to_the_plain_layer():
    # w1 = 1, w2 = 0 and identity linears: the product block passes A~ through,
    # so energies equal the correlation-1 model with the same other weights
    cfg2 = _cfg(lmax=2, C=8, layers=2)
    cfg1 = _cfg(lmax=2, C=8, layers=2, correlation=1)
    w = synth.model_weights(cfg2, 9)
    for t in (1, 2):
        w[f"sym1_{t}"] = np.ones_like(w[f"sym1_{t}"])
        w[f"sym2_{t}"] = np.zeros_like(w[f"sym2_{t}"])
        for L in range(synth.product_out_order(cfg2, t) + 1):
            w[f"lin_{t}_{L}"] = np.eye(8)
    w1 = {k: v for k, v in w.items() if not k.startswith(("sym", "lin"))}
    b = synth.uniform_cluster(14, 7.0, 0.9, 2, np.random.default_rng(10))
    E2, F2, _ = om.energy_forces(om.Model(cfg2, w), b)
    E1, F1, _ = om.energy_forces(om.Model(cfg1, w1), b)
    assert np.allclose(E2, E1, rtol=1e-13, atol=1e-14)
    assert np.allclose(F2, F1, atol=1e-14)


def test_product_model_forces_match_finite_differences():
    cfg = _cfg(lmax=3, C=6, layers=2)
    m = om.Model(cfg, synth.model_weights(cfg, 11))
    b = synth.uniform_cluster(12, 6.5, 0.9, 2, np.random.default_rng(12))
    E, F, _ = om.energy_forces(m, b)
    h = 1e-5
    for (i, k) in [(0, 0), (4, 1), (11, 2)]:
        bp = synth.Batch(b.pos.copy(), b.species, b.cell, b.pbc, b.offsets)
        bm = synth.Batch(b.pos.copy(), b.species, b.cell, b.pbc, b.offsets)
        bp.pos[i, k] += h
        bm.pos[i, k] -= h
        fd = -(om.energy(m, bp).sum() - om.energy(m, bm).sum()) / (2 * h)
        assert abs(fd - F[i, k]) < 1e-7 * max(1.0, abs(F[i, k]))


def test_product_model_features_are_equivariant_and_energy_invariant():
    cfg = _cfg(lmax=3, C=4, layers=3)
    m = om.Model(cfg, synth.model_weights(cfg, 13))
    b = synth.uniform_cluster(10, 6.0, 1.0, 2, np.random.default_rng(14))
    f0, f1 = [], []
    E0, _, _ = om.energy_forces(m, b, features=f0)
    R = cg.rotation(2.1, 0.3, 1.2)
    br = synth.Batch(b.pos @ R.T, b.species, b.cell, b.pbc, b.offsets)
    E1, _, _ = om.energy_forces(m, br, features=f1)
    assert np.allclose(E0, E1, rtol=1e-12)
    for h0, h1 in zip(f0[:-1], f1[:-1]):   # the last layer keeps scalars only
        h0, h1 = h0.detach().numpy(), h1.detach().numpy()
        for l in range(cfg.lmax + 1):
            D = cg.wigner_d(l, R)
            np.testing.assert_allclose(h1[:, :, l * l:(l + 1) ** 2], h0[:, :, l * l:(l + 1) ** 2] @ D.T,
                                       atol=1e-12)


def test_product_model_hessian_vector_matches_differences_of_forces():
    # the second-order quantities of the correlation-2 model: H v against
    # central differences of the forces along v
    cfg = _cfg(lmax=2, C=4, layers=2)
    m = _model_with(cfg, seed=7)
    b = synth.uniform_cluster(10, 6.0, 0.9, 2, np.random.default_rng(71))
    v = np.random.default_rng(72).normal(size=b.pos.shape)
    hv = om.hessian_vector(m, b, v)
    h = 1e-4

    def forces(pos):
        bb = synth.Batch(np.asarray(pos), b.species, b.cell, b.pbc, b.offsets, b.charge)
        return om.energy_forces(m, bb)[1]

    fd = -(forces(b.pos + h * v) - forces(b.pos - h * v)) / (2 * h)
    assert np.abs(hv - fd).max() < 1e-6 * max(1.0, np.abs(hv).max())


def test_product_model_loss_gradients_match_central_differences():
    # the weights of the block (w1, w2, the linear after it) and one upstream
    # of it, through the force term of the loss
    cfg = _cfg(lmax=2, C=4, layers=2)
    w = synth.model_weights(cfg, 8)
    rng = np.random.default_rng(73)
    b = synth.concat([synth.jittered_lattice(n, 0.1, 0.3, 2, rng) for n in (10, 14)])
    e_ref = rng.standard_normal(2)
    f_ref = rng.standard_normal((b.n_atoms, 3))
    loss, grads = om.loss_and_grads(om.Model(cfg, w), b, e_ref, f_ref)
    h = 1e-5
    for name in ["sym1_1", "sym2_1", "lin_1_1", "sym2_2", "lin_2_0", "mix_1_2"]:
        for _ in range(2):
            idx = tuple(int(rng.integers(0, s)) for s in w[name].shape)
            vals = []
            for sgn in (1, -1):
                w2 = {k: v.copy() for k, v in w.items()}
                w2[name][idx] += sgn * h
                vals.append(om.loss_and_grads(om.Model(cfg, w2), b, e_ref, f_ref)[0])
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - grads[name][idx]) < 1e-7 + 1e-5 * abs(fd), (name, idx, fd, grads[name][idx])
