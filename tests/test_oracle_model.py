"""Pins of the oracle model: finite differences, symmetries, locality and
special cases that reduce to simpler computations."""
import itertools
import math

import numpy as np
import pytest
import torch

import synth
from oracle import cg
from oracle import model as om
from oracle.sh import real_sh


def small_cfg(lmax=2, channels=8, layers=2, n_species=3, cutoff=5.0):
    return synth.ModelConfig(lmax=lmax, channels=channels, layers=layers, n_species=n_species,
                             cutoff=cutoff, avg_neighbors=10.0)


@pytest.fixture(scope="module")
def tiny():
    cfg, b = synth.tiny_config()
    return om.Model(cfg, synth.model_weights(cfg, 1)), b


def _with_pos(b, pos):
    return synth.Batch(np.asarray(pos, dtype=np.float64), b.species, b.cell, b.pbc, b.offsets)


def test_forces_match_central_differences(tiny):
    m, b = tiny
    E, F, _ = om.energy_forces(m, b)
    rng = np.random.default_rng(0)
    h = 1e-4
    for _ in range(8):
        i, a = int(rng.integers(0, b.n_atoms)), int(rng.integers(0, 3))
        p1, p2 = b.pos.copy(), b.pos.copy()
        p1[i, a] += h
        p2[i, a] -= h
        fd = -(om.energy(m, _with_pos(b, p1))[0] - om.energy(m, _with_pos(b, p2))[0]) / (2 * h)
        assert abs(fd - F[i, a]) < 1e-8 + 1e-6 * abs(F[i, a])


def test_net_force_and_torque_vanish(tiny):
    m, b = tiny
    _, F, _ = om.energy_forces(m, b)
    scale = np.abs(F).max()
    assert np.abs(F.sum(0)).max() < 1e-12 * max(1.0, scale * b.n_atoms)
    torque = np.cross(b.pos, F).sum(0)
    assert np.abs(torque).max() < 1e-11


def test_rotation_translation_permutation_invariance(tiny):
    m, b = tiny
    E0, F0, Ei0 = om.energy_forces(m, b)
    R = cg.rotation(0.7, 1.3, -2.1)
    c = b.pos.mean(0)
    E1, F1, _ = om.energy_forces(m, _with_pos(b, (b.pos - c) @ R.T + c))
    assert abs(E1[0] - E0[0]) < 1e-12 * max(1, abs(E0[0]))
    np.testing.assert_allclose(F1, F0 @ R.T, atol=1e-12)
    E2, F2, _ = om.energy_forces(m, _with_pos(b, b.pos + np.array([3.1, -2.2, 0.7])))
    assert abs(E2[0] - E0[0]) < 1e-12
    np.testing.assert_allclose(F2, F0, atol=1e-12)
    perm = np.random.default_rng(1).permutation(b.n_atoms)
    bp = synth.Batch(b.pos[perm], b.species[perm], b.cell, b.pbc, b.offsets)
    E3, F3, Ei3 = om.energy_forces(m, bp)
    assert abs(E3[0] - E0[0]) < 1e-12
    np.testing.assert_allclose(F3, F0[perm], atol=1e-12)
    np.testing.assert_allclose(Ei3, Ei0[perm], atol=1e-13)


def test_periodic_rotation_with_cell():
    cfg = small_cfg(lmax=3, n_species=4)
    m = om.Model(cfg, synth.model_weights(cfg, 7))
    b = synth.jittered_lattice(30, 0.1, 0.3, 4, np.random.default_rng(2))   # L = 6.7 A < 2 r_c
    E0, F0, _ = om.energy_forces(m, b)
    R = cg.rotation(0.4, 2.0, 1.0)
    br = synth.Batch(b.pos @ R.T, b.species, b.cell @ R.T, b.pbc, b.offsets)
    E1, F1, _ = om.energy_forces(m, br)
    assert abs(E1[0] - E0[0]) < 1e-11 * max(1, abs(E0[0]))
    np.testing.assert_allclose(F1, F0 @ R.T, atol=1e-11)


def test_features_are_equivariant():
    cfg = small_cfg(lmax=3, layers=3)
    m = om.Model(cfg, synth.model_weights(cfg, 3))
    b = synth.uniform_cluster(12, 6.0, 1.0, 3, np.random.default_rng(4))
    f0, f1 = [], []
    om.energy_forces(m, b, features=f0)
    R = cg.rotation(1.1, 0.5, 2.9)
    om.energy_forces(m, _with_pos(b, b.pos @ R.T), features=f1)
    for h0, h1 in zip(f0, f1):
        h0, h1 = h0.detach().numpy(), h1.detach().numpy()
        for l in range(cfg.lmax + 1):
            D = cg.wigner_d(l, R)
            np.testing.assert_allclose(h1[:, :, l * l:(l + 1) ** 2], h0[:, :, l * l:(l + 1) ** 2] @ D.T,
                                       atol=1e-12)


def test_wigner_d_is_an_orthogonal_representation():
    R1, R2 = cg.rotation(0.3, 0.9, 1.7), cg.rotation(-1.2, 2.2, 0.4)
    for l in range(4):
        D1, D2, D12 = cg.wigner_d(l, R1), cg.wigner_d(l, R2), cg.wigner_d(l, R1 @ R2)
        np.testing.assert_allclose(D1 @ D1.T, np.eye(2 * l + 1), atol=1e-12)
        np.testing.assert_allclose(D1 @ D2, D12, atol=1e-12)


def test_supercell_energy_and_forces():
    cfg = small_cfg(lmax=2, n_species=4)
    m = om.Model(cfg, synth.model_weights(cfg, 5))
    b = synth.jittered_lattice(20, 0.1, 0.3, 4, np.random.default_rng(6))   # L = 5.8 A: many images
    L = b.cell[0, 0, 0]
    E0, F0, _ = om.energy_forces(m, b)
    reps = [b.pos + np.array(n) * L for n in itertools.product(range(2), repeat=3)]
    big = synth.Batch(np.concatenate(reps), np.tile(b.species, 8), (np.eye(3) * 2 * L)[None],
                      np.ones((1, 3), np.uint8), np.array([0, 160]))
    E1, F1, _ = om.energy_forces(m, big)
    assert abs(E1[0] - 8 * E0[0]) < 1e-11 * max(1, abs(E1[0]))
    np.testing.assert_allclose(F1.reshape(8, 20, 3), np.broadcast_to(F0, (8, 20, 3)), atol=1e-11)


def test_isolated_atoms_are_additive_and_force_free(tiny):
    m, _ = tiny
    cfg = m.cfg
    pos = np.array([[0, 0, 0], [6, 0, 0], [0, 6.5, 0], [0, 0, 7], [6, 6.5, 7.0]], dtype=float)
    species = np.array([0, 1, 2, 1, 0], np.int32)
    b = synth.Batch(pos, species, (np.eye(3) * 20)[None], np.zeros((1, 3), np.uint8), np.array([0, 5]))
    E, F, _ = om.energy_forces(m, b)
    single = {}
    for z in range(cfg.n_species):
        s = synth.Batch(np.zeros((1, 3)), np.array([z], np.int32), (np.eye(3) * 20)[None],
                        np.zeros((1, 3), np.uint8), np.array([0, 1]))
        single[z] = om.energy(m, s)[0]
    assert abs(E[0] - sum(single[int(z)] for z in species)) < 1e-12
    assert np.all(F == 0)


def test_two_atoms_forces_along_bond(tiny):
    m, _ = tiny
    pos = np.array([[0.1, 0.2, 0.3], [1.9, 1.1, -0.8]])
    b = synth.Batch(pos, np.array([0, 2], np.int32), (np.eye(3) * 20)[None], np.zeros((1, 3), np.uint8),
                    np.array([0, 2]))
    _, F, _ = om.energy_forces(m, b)
    d = pos[1] - pos[0]
    np.testing.assert_allclose(F[0], -F[1], atol=1e-15)
    assert np.linalg.norm(np.cross(F[0], d)) < 1e-14 * max(1e-300, np.linalg.norm(F[0])) + 1e-18
    assert np.linalg.norm(F[0]) > 0


def test_scalar_model_has_no_angular_dependence():
    # Centre atom with two neighbours at 3 A whose mutual distance exceeds the
    # cutoff: at l_max = 0 only distances enter, at l_max = 1 angles do.
    def energy(lmax, angle):
        cfg = synth.ModelConfig(lmax=lmax, channels=6, layers=2, n_species=2, cutoff=3.5, avg_neighbors=3.0)
        m = om.Model(cfg, synth.model_weights(cfg, 9))
        pos = np.array([[0, 0, 0], [3, 0, 0], [3 * math.cos(angle), 3 * math.sin(angle), 0]])
        b = synth.Batch(pos, np.array([0, 1, 1], np.int32), (np.eye(3) * 20)[None],
                        np.zeros((1, 3), np.uint8), np.array([0, 3]))
        return om.energy(m, b)[0]
    assert abs(energy(0, math.pi / 2) - energy(0, math.pi)) < 1e-14
    assert abs(energy(1, math.pi / 2) - energy(1, math.pi)) > 1e-10


def test_message_einsum_against_explicit_loops():
    # One layer-2 neighbour sum over three edges, recomputed with plain loops.
    cfg = small_cfg(lmax=3, channels=3)
    m = om.Model(cfg, synth.model_weights(cfg, 2))
    rng = np.random.default_rng(8)
    N, C, nc = 3, cfg.channels, 16
    h = torch.from_numpy(rng.standard_normal((N, C, nc)))
    d = rng.standard_normal((3, 3))
    src, dst = torch.tensor([1, 2, 0]), torch.tensor([0, 0, 2])
    Y = real_sh(torch.from_numpy(d), 3)
    B = torch.from_numpy(rng.standard_normal((3, cfg.n_basis)))
    A = m._messages(2, h, B, Y, src, dst, N).numpy()
    W1, W2, W3 = (m.w[f"rad{k}_2"].numpy() for k in (1, 2, 3))

    def silu(x):
        return x / (1 + np.exp(-x))
    ref = np.zeros_like(A)
    paths = m.layer_paths[1]
    for e in range(3):
        R = (silu(silu(B[e].numpy() @ W1) @ W2) @ W3).reshape(len(paths), C)
        off = 0
        for pi, (l1, l2, l3) in enumerate(paths):
            Cp = cg.real_cg(l1, l2, l3)
            for k in range(C):
                for m3 in range(2 * l3 + 1):
                    s = 0.0
                    for m1 in range(2 * l1 + 1):
                        for m2 in range(2 * l2 + 1):
                            s += Cp[m1, m2, m3] * h[src[e], k, l1 * l1 + m1].item() * Y[e, l2 * l2 + m2].item()
                    ref[dst[e], k, off + m3] += R[pi, k] * s / cfg.avg_neighbors
            off += 2 * l3 + 1
    np.testing.assert_allclose(A, ref, atol=1e-12)


def test_loss_gradients_match_central_differences():
    cfg = small_cfg(lmax=2, channels=4, n_species=3)
    w = synth.model_weights(cfg, 11)
    rng = np.random.default_rng(12)
    b = synth.concat([synth.jittered_lattice(n, 0.1, 0.3, 3, rng) for n in (12, 18)])
    e_ref = rng.standard_normal(2)
    f_ref = rng.standard_normal((b.n_atoms, 3))
    m = om.Model(cfg, w)
    loss, grads = om.loss_and_grads(m, b, e_ref, f_ref)
    h = 1e-5
    for name in ["emb", "rad1_1", "rad3_2", "mix_2_0", "mix_2_1", "self_2_2", "read1", "read2", "rad2_2"]:
        for _ in range(3):
            idx = tuple(int(rng.integers(0, s)) for s in w[name].shape)
            vals = []
            for sgn in (1, -1):
                w2 = {k: v.copy() for k, v in w.items()}
                w2[name][idx] += sgn * h
                vals.append(om.loss_and_grads(om.Model(cfg, w2), b, e_ref, f_ref)[0])
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - grads[name][idx]) < 1e-7 + 1e-5 * abs(fd), (name, idx, fd, grads[name][idx])


# ---- gate, readout and the neighbour sum pinned by limits and reductions ----

def _np_silu(x):
    return x / (1.0 + np.exp(-x))


def _np_sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _gate_features(lam, cfg, w, b):
    """First-layer output features when the self connection of the scalars
    is lam * identity (embedding entries are positive, so lam drives every
    channel's pre-gate scalar towards +-infinity)."""
    m = om.Model(cfg, w)
    m.w["self_1_0"] = torch.eye(cfg.channels, dtype=torch.float64) * lam
    feats = []
    om.energy_forces(m, b, features=feats)
    return feats[0].detach().numpy()  # [N, C, (lmax+1)^2]


def test_gate_limits_and_form():
    # MACE's gate (Appendix F, gate_nodes): h[0] = silu(h~[0]), h[l>0] =
    # h~[l] sigmoid(h~[0]) per channel. In layer 1 the self connection only
    # touches l = 0, so h~[l>0] does not depend on lam while h~[0] = a + lam e.
    cfg = small_cfg(lmax=2, channels=5, layers=1, n_species=2)
    w = synth.model_weights(cfg, 31)
    w["emb"] = np.random.default_rng(32).uniform(0.5, 1.5, size=w["emb"].shape)
    b = synth.uniform_cluster(7, 6.0, 1.0, 2, np.random.default_rng(33))
    e = w["emb"][b.species]                           # [N, C] = h0 of every atom
    hp, hp2, hm = (_gate_features(lam, cfg, w, b) for lam in (60.0, 120.0, -60.0))
    # l > 0: unchanged in the +infinity limit, gone in the -infinity limit
    vec = slice(1, None)
    assert np.abs(hp[:, :, vec]).max() > 1e-3
    np.testing.assert_allclose(hp[:, :, vec], hp2[:, :, vec], rtol=0, atol=1e-14)
    assert np.abs(hm[:, :, vec]).max() < 1e-10 * np.abs(hp[:, :, vec]).max()
    # l = 0: silu is x at +infinity (slope one, no offset) and 0 at -infinity
    np.testing.assert_allclose(hp2[:, :, 0] - hp[:, :, 0], 60.0 * e, rtol=1e-12)
    assert np.abs(hm[:, :, 0]).max() < 1e-10
    # at a finite lam the exact forms, with a = h~[0] - lam e recovered from +infinity
    a = hp[:, :, 0] - 60.0 * e
    lam = 0.37
    h = _gate_features(lam, cfg, w, b)
    x = a + lam * e
    np.testing.assert_allclose(h[:, :, 0], _np_silu(x), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(h[:, :, vec], hp[:, :, vec] * _np_sigmoid(x)[:, :, None], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("unit", [0, 5, 15])
def test_readout_one_hidden_unit(unit):
    # Readout 16x0e -> 0e (Appendix F): E_i = w2 . silu(W_r^T h_i[0]) + E0[z_i].
    # With w2 one-hot at `unit` the energy of atom i is silu of one column of
    # W_r against its final scalar features, plus E0. Square W_r (C = 16), so
    # a transposed W_r would not fail on shapes.
    cfg = small_cfg(lmax=2, channels=16, layers=2, n_species=3)
    w = synth.model_weights(cfg, 34)
    w["read2"] = np.zeros((16, 1))
    w["read2"][unit, 0] = 1.0
    w["e0"] = np.array([-1.25, 0.5, 3.0])
    m = om.Model(cfg, w)
    b = synth.uniform_cluster(9, 7.0, 1.0, 3, np.random.default_rng(35))
    feats = []
    _, _, Ei = om.energy_forces(m, b, features=feats)
    h0 = feats[-1][:, :, 0].detach().numpy()
    expect = _np_silu(h0 @ w["read1"][:, unit]) + w["e0"][b.species]
    np.testing.assert_allclose(Ei, expect, rtol=1e-13, atol=1e-14)


def _np_radial(r, rc, n_basis, p, W1, W2, W3):
    """R(r) of one edge: Bessel functions through scipy's spherical j0 times
    the polynomial envelope, then the two-hidden-layer MLP without biases."""
    from scipy.special import spherical_jn
    n = np.arange(1, n_basis + 1)
    k = n * math.pi / rc
    bes = math.sqrt(2.0 / rc) * k * spherical_jn(0, k * r)
    x = r / rc
    u = np.polynomial.polynomial.polyval(x, [1.0] + [0.0] * (p - 1) +
                                         [-(p + 1) * (p + 2) / 2.0, p * (p + 2), -p * (p + 1) / 2.0])
    B = bes * (u if x < 1.0 else 0.0)
    return _np_silu(_np_silu(B @ W1) @ W2) @ W3


def test_lmax0_single_layer_is_a_pair_potential():
    # At l_max = 0 with one layer, the only path is (0,0,0) (Y_0 = 1, C = 1),
    # so the neighbour sum is A_i = nu^-1 sum_{j != i, r_ij < r_c} R(r_ij) h0_j.
    # Scale the channel mix by eps: to first order in eps the readout is
    # linear in A, and dE/deps at 0 = sum over ordered pairs of
    # phi_{z_i z_j}(r_ij) with phi_ab(r) = nu^-1 sum_k R_k(r) emb[b,k] (W g_a)_k,
    # g_a the gradient of the atom energy with respect to h~ at h~ = emb[a] S.
    cfg = synth.ModelConfig(lmax=0, channels=4, layers=1, n_species=2, cutoff=4.0, avg_neighbors=3.7)
    w = synth.model_weights(cfg, 36)
    b = synth.uniform_cluster(11, 6.0, 1.0, 2, np.random.default_rng(37))
    m = om.Model(cfg, w)
    eps = torch.zeros((), dtype=torch.float64, requires_grad=True)
    m.w["mix_1_0"] = torch.tensor(w["mix_1_0"]) * eps
    dst, src, shv = om._edges(b, cfg.cutoff)
    pos = torch.tensor(b.pos)
    sp = torch.from_numpy(b.species.astype(np.int64))
    E = m.node_energies(pos, sp, dst, src, shv).sum()
    (dE,) = torch.autograd.grad(E, eps)

    # independent pair sum: all ordered pairs by brute force
    Wr, w2 = w["read1"], w["read2"][:, 0]

    def g_of(a):
        x = w["emb"][a] @ w["self_1_0"]
        dsilu = lambda t: _np_sigmoid(t) * (1.0 + t * (1.0 - _np_sigmoid(t)))
        y = _np_silu(x) @ Wr
        return dsilu(x) * (Wr @ (dsilu(y) * w2))

    g = [g_of(a) for a in range(2)]
    total = 0.0
    for i in range(b.n_atoms):
        for j in range(b.n_atoms):
            r = float(np.linalg.norm(b.pos[j] - b.pos[i]))
            if i == j or r >= cfg.cutoff:
                continue
            R = _np_radial(r, cfg.cutoff, cfg.n_basis, cfg.envelope_p, w["rad1_1"], w["rad2_1"], w["rad3_1"])
            a, c = int(b.species[i]), int(b.species[j])
            total += float(np.sum(R * w["emb"][c] * (w["mix_1_0"] @ g[a]))) / cfg.avg_neighbors
    assert abs(total) > 1e-3
    assert abs(float(dE) - total) <= 1e-12 * max(1.0, abs(total)), (float(dE), total)
