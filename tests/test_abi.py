"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and rejects bad configurations before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from paper_2605_22698_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "e3mi.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(e3mi_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libe3mi.so is not built: run python -m paper_2605_22698_amd.build")
    return _lib.lib()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "e3mi_energy_forces" in names and len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES), "binding signatures out of sync with the header"


@pytest.mark.parametrize("cfg", [synth.tiny_config()[0], synth.single_config()[0], synth.scale_config(64)[0],
                                 synth.differentiation_config(2)[0]])
def test_weight_count_matches_generator(lib, cfg):
    n = ctypes.c_size_t()
    _lib.check(lib.e3mi_weight_count(cfg.to_json().encode(), ctypes.byref(n)))
    assert n.value == sum(int(np.prod(s)) for _, s, _ in synth.weight_shapes(cfg))
    assert n.value == synth.flatten_weights(cfg, synth.model_weights(cfg, 0)).size


def test_config_errors(lib):
    n = ctypes.c_size_t()
    assert lib.e3mi_weight_count(b"{}", ctypes.byref(n)) == -1
    assert "missing key" in lib.e3mi_last_error().decode()
    cfg = synth.tiny_config()[0]
    bad = cfg.to_json().replace('"lmax": 2', '"lmax": 5').encode()
    assert lib.e3mi_weight_count(bad, ctypes.byref(n)) == -6
    bad = cfg.to_json().replace('"channels": 32', '"channels": 96').encode()
    assert lib.e3mi_weight_count(bad, ctypes.byref(n)) == -6
    assert lib.e3mi_weight_count(cfg.to_json().encode(), None) == -1


def test_model_create_rejects_wrong_weight_count(lib):
    cfg = synth.tiny_config()[0]
    w = np.zeros(10)
    h = ctypes.c_void_p()
    rc = lib.e3mi_model_create(cfg.to_json().encode(), w.ctypes.data, w.size, 0, _lib.ALLOC_FN(), _lib.FREE_FN(),
                               None, ctypes.byref(h))
    assert rc == -1 and "weight count" in lib.e3mi_last_error().decode()
    assert not h.value
    rc = lib.e3mi_model_create(cfg.to_json().encode(), w.ctypes.data, w.size, 7, _lib.ALLOC_FN(), _lib.FREE_FN(),
                               None, ctypes.byref(h))
    assert rc == -1


def test_null_handles(lib):
    assert lib.e3mi_energy_forces(None, None, None, None, None, None, None) == -1
    assert lib.e3mi_md_step(None, 1, 0.5, None, None) == -1
    assert lib.e3mi_graph_info(None, None, None) == -1
    assert lib.e3mi_footprint_bytes(None, 10, 10) == 0
    assert lib.e3mi_model_set_flags(None, 8) == -1 and "null model" in lib.e3mi_last_error().decode()
    assert lib.e3mi_model_destroy(None) == 0


def test_md_binding_rejects_bad_state_before_the_library():
    # the MD binding checks shapes and dtypes of the state and the mass table
    # before any call into the library (no device needed)
    import torch
    import paper_2605_22698_amd as e3

    class _FakeModel:
        config_json = synth.tiny_config()[0].to_json()
        handle = None

    cfg, b = synth.tiny_config()
    n = b.n_atoms
    pos = torch.tensor(b.pos, dtype=torch.float64)
    vel = torch.zeros((n, 3), dtype=torch.float64)
    sp = torch.tensor(b.species, dtype=torch.int32)
    masses = synth.SPECIES_MASS[:cfg.n_species]
    bad = [
        dict(pos=pos.float()), dict(pos=pos[:-1]), dict(vel=vel.float()), dict(vel=vel[:, :2]),
        dict(species=sp[:-1]), dict(species=sp.double()), dict(masses=synth.SPECIES_MASS[:cfg.n_species + 1]),
    ]
    for change in bad:
        args = dict(pos=pos, vel=vel, species=sp, masses=masses)
        args.update(change)
        with pytest.raises(ValueError):
            e3.MD(_FakeModel(), b.offsets, args["pos"], args["vel"], args["species"], args["masses"], b.cell, b.pbc,
                  cfg.cutoff)
