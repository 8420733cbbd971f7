"""GPU neighbour lists vs the oracle's brute force: bit-exact edge sets."""
import numpy as np
import pytest

import synth
from oracle.neighbours import neighbour_list
from tests.gpu_util import device, model, say, to_dev

pytestmark = pytest.mark.gpu


def _cases():
    rng = np.random.default_rng(31)
    tiny_cfg, tiny = synth.tiny_config()
    small = synth.jittered_lattice(20, 0.1, 0.3, 3, rng)        # 5.85 A box: several images per pair
    box400 = synth.jittered_lattice(400, 0.1, 0.3, 3, rng)
    batch = synth.concat([synth.jittered_lattice(n, 0.1, 0.3, 3, rng) for n in (7, 33, 120, 2)] + [tiny])
    outside = synth.jittered_lattice(60, 0.1, 0.3, 3, rng)
    outside.pos = outside.pos + rng.integers(-3, 4, size=(60, 3)) * outside.cell[0, 0, 0]
    one = synth.Batch(np.array([[0.3, 0.2, 0.1]]), np.zeros(1, np.int32), (np.eye(3) * 2.2)[None],
                      np.ones((1, 3), np.uint8), np.array([0, 1]))
    slab = synth.jittered_lattice(64, 0.1, 0.3, 3, rng)
    slab.pbc = np.array([[1, 1, 0]], np.uint8)
    return {"tiny_open": tiny, "small_periodic": small, "box400": box400, "packed_batch": batch,
            "outside_cell": outside, "single_atom_lattice": one, "slab": slab}


CASES = _cases()


@pytest.fixture(scope="module")
def m():
    cfg, _ = synth.tiny_config()
    return model(cfg, 1)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("skin", [0.0, 1.0])
def test_edges_equal_bruteforce(m, name, skin):
    import torch
    b = CASES[name]
    say(f"graph case {name} skin {skin} N={b.n_atoms}")
    rc = 5.0
    pos, sp = to_dev(b)
    g = m.build_graph(b.offsets, pos, sp, b.cell, b.pbc, rc, skin)
    row_ptr, src, shift, rev = (t.cpu().numpy() for t in g.edges())
    torch.cuda.synchronize()
    dst_r, src_r, sh_r = neighbour_list(b.pos, b.cell, b.pbc, b.offsets, rc + skin)
    assert g.n_skin_edges == len(dst_r)
    np.testing.assert_array_equal(row_ptr, np.concatenate([[0], np.cumsum(np.bincount(dst_r, minlength=b.n_atoms))]))
    np.testing.assert_array_equal(src, src_r)
    np.testing.assert_array_equal(shift, sh_r)
    dst = np.repeat(np.arange(b.n_atoms), np.diff(row_ptr))
    np.testing.assert_array_equal(rev[rev], np.arange(len(rev)))
    np.testing.assert_array_equal(src[rev], dst)
    np.testing.assert_array_equal(shift[rev], -shift)


def test_pruned_edge_count(m):
    b = CASES["box400"]
    pos, sp = to_dev(b)
    g = m.build_graph(b.offsets, pos, sp, b.cell, b.pbc, 5.0, 1.0)
    m.energy_forces(g, pos)
    dst_r, _, _ = neighbour_list(b.pos, b.cell, b.pbc, b.offsets, 5.0)
    assert g.last_edge_count() == len(dst_r)


def test_empty_and_isolated(m):
    import torch
    b = synth.Batch(np.array([[0.0, 0, 0], [9.0, 0, 0]]), np.array([0, 1], np.int32), (np.eye(3) * 30)[None],
                    np.zeros((1, 3), np.uint8), np.array([0, 2]))
    pos, sp = to_dev(b)
    g = m.build_graph(b.offsets, pos, sp, b.cell, b.pbc, 5.0, 0.5)
    assert g.n_skin_edges == 0
    E, F, _ = m.energy_forces(g, pos)
    torch.cuda.synchronize()
    assert torch.all(F == 0)
    # a structure with no atoms next to one with atoms
    b2 = synth.Batch(b.pos, b.species, np.concatenate([b.cell, b.cell]), np.zeros((2, 3), np.uint8),
                     np.array([0, 0, 2]))
    g2 = m.build_graph(b2.offsets, pos, sp, b2.cell, b2.pbc, 5.0, 0.5)
    E2, F2, _ = m.energy_forces(g2, pos)
    torch.cuda.synchronize()
    assert E2[0].item() == 0.0
    assert abs(E2[1].item() - E[0].item()) == 0.0


def test_rejects_triclinic_and_nan(m):
    import paper_2605_22698_amd as e3
    b = synth.jittered_lattice(20, 0.1, 0.3, 3, np.random.default_rng(1))
    pos, sp = to_dev(b)
    cell = b.cell.copy()
    cell[0, 0, 1] = 0.5
    with pytest.raises(e3.E3miError) as ei:
        m.build_graph(b.offsets, pos, sp, cell, b.pbc, 5.0, 0.0)
    assert ei.value.code == -6
    bad = pos.clone()
    bad[3, 1] = float("nan")
    with pytest.raises(e3.E3miError) as ei:
        m.build_graph(b.offsets, bad, sp, b.cell, b.pbc, 5.0, 0.0)
    assert ei.value.code == -5
    with pytest.raises(e3.E3miError):
        m.build_graph(b.offsets, pos, sp, b.cell, b.pbc, 4.0, 0.0)   # below the model cutoff


def test_rejects_species_out_of_range(m):
    # species index the per-species tables: values outside [0, n_species)
    # are rejected by the graph build (and so by MD creation) with EINVAL
    import paper_2605_22698_amd as e3
    b = synth.jittered_lattice(20, 0.1, 0.3, 3, np.random.default_rng(2))
    pos, sp = to_dev(b)
    n_species = synth.ModelConfig.from_json(m.config_json).n_species
    for v in (-1, n_species, 1 << 20):
        bad = sp.clone()
        bad[7] = v
        with pytest.raises(e3.E3miError) as ei:
            m.build_graph(b.offsets, pos, bad, b.cell, b.pbc, 5.0, 0.0)
        assert ei.value.code == -1 and "species" in str(ei.value)
    g = m.build_graph(b.offsets, pos, sp, b.cell, b.pbc, 5.0, 0.0)   # the model is still usable
    assert g.n_skin_edges > 0
