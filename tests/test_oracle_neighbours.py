"""Pins of the oracle's brute-force radius graph."""
import itertools
import math

import numpy as np
from scipy.spatial import cKDTree

import synth
from oracle.neighbours import neighbour_list


def _edge_set(dst, src, sh):
    return set(zip(dst.tolist(), src.tolist(), map(tuple, sh.tolist())))


def test_open_cluster_matches_kdtree():
    cfg, b = synth.tiny_config()
    dst, src, sh = neighbour_list(b.pos, b.cell, b.pbc, b.offsets, cfg.cutoff)
    assert np.all(sh == 0)
    pairs = cKDTree(b.pos).query_pairs(cfg.cutoff, output_type="ndarray")
    ref = set()
    for i, j in pairs:
        ref.add((int(i), int(j), (0, 0, 0)))
        ref.add((int(j), int(i), (0, 0, 0)))
    assert _edge_set(dst, src, sh) == ref


def test_periodic_box_matches_kdtree():
    b = synth.jittered_lattice(400, 0.1, 0.3, 4, np.random.default_rng(11))
    L = b.cell[0, 0, 0]
    rc = 4.0
    assert L > 2 * rc
    dst, src, sh = neighbour_list(b.pos, b.cell, b.pbc, b.offsets, rc)
    pairs = cKDTree(b.pos, boxsize=L).query_pairs(rc, output_type="ndarray")
    ours = set(zip(dst.tolist(), src.tolist()))
    ref = set()
    for i, j in pairs:
        ref.add((int(i), int(j)))
        ref.add((int(j), int(i)))
    assert ours == ref
    # each (i, j) appears once when L > 2 rc, and the image reproduces the distance
    assert len(ours) == len(dst)
    d = b.pos[src] - b.pos[dst] + sh * L
    assert np.all(np.linalg.norm(d, axis=1) < rc)


def test_symmetric():
    cfg, b, _, _ = synth.differentiation_config(4)
    dst, src, sh = neighbour_list(b.pos, b.cell, b.pbc, b.offsets, cfg.cutoff)
    es = _edge_set(dst, src, sh)
    for (i, j, n) in es:
        assert (j, i, tuple(-x for x in n)) in es
    owner = np.searchsorted(b.offsets, dst, side="right")
    assert np.all(owner == np.searchsorted(b.offsets, src, side="right"))


def test_single_atom_lattice_images():
    # One atom in a periodic cube of side a: its neighbours are exactly the
    # lattice points n*a with 0 < |n| a < r_c.
    a, rc = 2.3, 5.0
    b = synth.Batch(np.array([[0.4, 1.1, 2.0]]), np.zeros(1, np.int32), (np.eye(3) * a)[None],
                    np.ones((1, 3), np.uint8), np.array([0, 1]))
    dst, src, sh = neighbour_list(b.pos, b.cell, b.pbc, b.offsets, rc)
    k = int(math.ceil(rc / a))
    ref = {n for n in itertools.product(range(-k, k + 1), repeat=3)
           if 0 < math.sqrt(sum(x * x for x in n)) * a < rc}
    assert set(map(tuple, sh.tolist())) == ref
    assert len(sh) == len(ref)


def test_supercell_neighbour_counts():
    b = synth.jittered_lattice(40, 0.1, 0.3, 3, np.random.default_rng(3))
    L = b.cell[0, 0, 0]
    reps = []
    for n in itertools.product(range(2), repeat=3):
        reps.append(b.pos + np.array(n) * L)
    big = synth.Batch(np.concatenate(reps), np.tile(b.species, 8), (np.eye(3) * 2 * L)[None],
                      np.ones((1, 3), np.uint8), np.array([0, 8 * 40]))
    d1, _, _ = neighbour_list(b.pos, b.cell, b.pbc, b.offsets, 5.0)
    d2, _, _ = neighbour_list(big.pos, big.cell, big.pbc, big.offsets, 5.0)
    c1 = np.bincount(d1, minlength=40)
    c2 = np.bincount(d2, minlength=320).reshape(8, 40)
    assert np.all(c2 == c1[None, :])


def test_mean_count_near_nominal():
    b = synth.jittered_lattice(1500, 0.1, 0.3, 4, np.random.default_rng(9))
    dst, _, _ = neighbour_list(b.pos, b.cell, b.pbc, b.offsets, 5.0)
    mean = len(dst) / 1500
    assert abs(mean / synth.nominal_neighbors(0.1, 5.0) - 1) < 0.03


def test_positions_outside_the_box():
    # Shifting atoms by whole cells changes the image vectors, not the graph.
    b = synth.jittered_lattice(30, 0.1, 0.3, 3, np.random.default_rng(13))
    L = b.cell[0, 0, 0]
    k = np.random.default_rng(14).integers(-3, 4, size=(30, 3))
    moved = b.pos + k * L
    d0, s0, n0 = neighbour_list(b.pos, b.cell, b.pbc, b.offsets, 5.0)
    d1, s1, n1 = neighbour_list(moved, b.cell, b.pbc, b.offsets, 5.0)
    assert np.array_equal(d0, d1) and np.array_equal(s0, s1)
    # r_j - r_i + n L is the same displacement in both
    np.testing.assert_allclose(moved[s1] - moved[d1] + n1 * L, b.pos[s0] - b.pos[d0] + n0 * L, atol=1e-12)
