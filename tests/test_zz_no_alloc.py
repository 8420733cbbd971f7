"""The allocation-free evaluation (e3mi_energy_forces_static) against the
ordinary entry point, through the C ABI: two calls in a row, the second on a
smaller input, both bitwise equal to e3mi_energy_forces on the same graph; an
input too large for the static array is refused and leaves the model usable."""
import ctypes

import numpy as np
import pytest

import synth
from tests.gpu_util import check_energy, check_forces, model, say, to_dev

pytestmark = pytest.mark.gpu


def _static(m, g, pos):
    import torch
    from paper_2605_22698_amd import _lib
    S, N = g.n_structures, g.n_atoms
    E = torch.full((S,), float("nan"), dtype=torch.float64, device=m.device)
    F = torch.full((N, 3), float("nan"), dtype=torch.float32, device=m.device)
    Ei = torch.full((N,), float("nan"), dtype=torch.float64, device=m.device)
    code = _lib.lib().e3mi_energy_forces_static(m.handle, g.handle, _lib.ptr(pos), _lib.ptr(E), _lib.ptr(F),
                                                _lib.ptr(Ei), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return code, E, F, Ei


def test_static_scratch_equals_energy_forces_twice_then_refuses_oversize():
    import torch
    from paper_2605_22698_amd import _lib
    cfg = synth.ModelConfig(lmax=3, channels=64, layers=2, n_species=4, cutoff=5.0,
                            avg_neighbors=synth.nominal_neighbors(0.1, 5.0))
    m = model(cfg, 31)
    rng = np.random.default_rng(32)
    for n in (180, 45):  # the second call's input is smaller
        b = synth.jittered_lattice(n, 0.1, 0.3, 4, rng)
        pos, sp = to_dev(b)
        g = m.build_graph(b.offsets, pos, sp, b.cell, b.pbc, cfg.cutoff, 0.5)
        E, F, Ei = m.energy_forces(g, pos, atom_energy=True)
        code, E2, F2, Ei2 = _static(m, g, pos)
        torch.cuda.synchronize()
        assert code == 0, _lib.lib().e3mi_last_error().decode()
        say(f"static scratch, {n} atoms: max |dF| {float((F2 - F).abs().max()):.1e}")
        assert torch.equal(E, E2) and torch.equal(F, F2) and torch.equal(Ei, Ei2)
        check_energy(E2.cpu().numpy(), E.cpu().numpy(), Ei.cpu().numpy())
        check_forces(F2.double().cpu().numpy(), F.double().cpu().numpy())
    # the 3,000-atom box needs far more than 128 MiB: refused, model unchanged
    cfg2, big = synth.single_config(n=3000)
    m2 = model(cfg2, 2)
    pos, sp = to_dev(big)
    g = m2.build_graph(big.offsets, pos, sp, big.cell, big.pbc, cfg2.cutoff, 0.0)
    E, F, _ = m2.energy_forces(g, pos)
    code, _, _, _ = _static(m2, g, pos)
    assert code == -2  # E3MI_ENOMEM
    assert "static scratch" in _lib.lib().e3mi_last_error().decode()
    E3, F3, _ = m2.energy_forces(g, pos)
    torch.cuda.synchronize()
    assert torch.equal(E, E3) and torch.equal(F, F3)
