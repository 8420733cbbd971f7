"""The radial MLP and its adjoint once per edge pair (the default for layers
whose edges are all in memory at once) against the same model evaluated edge
by edge (E3MI_FLAG_RADIAL_PER_EDGE): an edge and its reverse have exactly
opposite FP64 vectors, so the forward pass (R written to both rows) gives the
same bits, energies included; the adjoint takes the pair's summed dR through
the MLP once, so forces agree to FP32 rounding (max |dF| <= 1e-5 of the
largest force; BF16 mode: 1e-2, one more rounding of the summed dR to BF16).
Cases with several images of one neighbour, an atom that only sees its own
images, open and slab boundaries and a packed batch; each pair-mode result is
also checked against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import model as om
from tests.gpu_util import check_energy, check_forces, gpu_energy_forces, model, record, say

pytestmark = pytest.mark.gpu


def _cases():
    rng = np.random.default_rng(151)
    _, tiny = synth.tiny_config()
    small = synth.jittered_lattice(20, 0.1, 0.3, 4, rng)        # 5.85 A box: several images per pair
    one = synth.Batch(np.array([[0.3, 0.2, 0.1]]), np.zeros(1, np.int32), (np.eye(3) * 2.2)[None],
                      np.ones((1, 3), np.uint8), np.array([0, 1]))   # only its own images
    slab = synth.jittered_lattice(64, 0.1, 0.3, 4, rng)
    slab.pbc = np.array([[1, 1, 0]], np.uint8)
    batch = synth.concat([synth.jittered_lattice(n, 0.1, 0.3, 4, rng) for n in (7, 33, 2)] + [tiny, one])
    return {"tiny_open": tiny, "small_periodic": small, "single_atom_lattice": one, "slab": slab,
            "packed_batch": batch}


CASES = _cases()


def _cfg(lmax, channels, layers):
    return synth.ModelConfig(lmax=lmax, channels=channels, layers=layers, n_species=4, cutoff=5.0,
                             avg_neighbors=synth.nominal_neighbors(0.1, 5.0))


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("arch", [(3, 64, 2), (2, 64, 3)])
def test_pairs_equal_per_edge_and_oracle(name, arch):
    b = CASES[name]
    cfg = _cfg(*arch)
    m = model(cfg, 152)
    m.set_flags(radial_per_edge=True)
    E0, F0, Ei0, _ = gpu_energy_forces(m, b, skin=1.0)
    m.set_flags()
    E1, F1, Ei1, _ = gpu_energy_forces(m, b, skin=1.0)
    fmax = max(np.abs(F0).max(), 1e-30)
    d = float(np.abs(F1 - F0).max())
    say(f"pairs vs per edge ({name}, lmax {arch[0]}, {arch[2]} layers, N={b.n_atoms}): max |dF| {d:.1e}, "
        f"{d / fmax:.1e} of max |F|")
    assert np.array_equal(E0, E1) and np.array_equal(Ei0, Ei1)
    assert d <= 1e-5 * fmax
    Er, Fr, Eir = om.energy_forces(om.Model(cfg, synth.model_weights(cfg, 152)), b)
    check_energy(E1, Er, Eir)
    check_forces(F1, Fr)


@pytest.mark.parametrize("precision,correlation", [(0, 2), (1, 1)])
def test_pairs_larger_box(precision, correlation):
    """400 atoms, 3 layers (a middle layer with every path), the product
    block or the BF16 mode."""
    cfg = synth.ModelConfig(lmax=3, channels=64, layers=3, n_species=4, cutoff=5.0,
                            avg_neighbors=synth.nominal_neighbors(0.1, 5.0), correlation=correlation)
    b = synth.jittered_lattice(400, 0.1, 0.3, 4, np.random.default_rng(153))
    m = model(cfg, 154, precision=precision)
    m.set_flags(radial_per_edge=True)
    E0, F0, Ei0, _ = gpu_energy_forces(m, b, skin=1.0)
    m.set_flags()
    E1, F1, Ei1, _ = gpu_energy_forces(m, b, skin=1.0)
    fmax = np.abs(F0).max()
    d = float(np.abs(F1 - F0).max())
    record("pairs_vs_per_edge", precision=precision, correlation=correlation, max_abs=d, rel_to_max_abs_F=d / fmax)
    assert np.array_equal(E0, E1) and np.array_equal(Ei0, Ei1)
    assert d <= (1e-5 if precision == 0 else 1e-2) * fmax
