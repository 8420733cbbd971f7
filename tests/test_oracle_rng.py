"""Pins of the oracle's counter-based generator (Philox4x64-10, §5.5 seeds)."""
import numpy as np
import pytest

from oracle import rng

MASK = (1 << 64) - 1


@pytest.mark.parametrize("key,counter", [
    ((0, 0), (0, 0, 0, 0)),
    ((12345, 678), (0, 0, 0, 0)),
    ((MASK, MASK), (7, 3, 2, 1)),
    ((0x243F6A8885A308D3, 0x13198A2E03707344), (0xA4093822299F31D0, 0x082EFA98EC4E6C89, 11, 0)),
    ((1, 2), (123456789, 987654321, 42, 17)),
])
def test_block_function_matches_numpy_philox(key, counter):
    # numpy's Philox bit generator (an independent implementation of the
    # same published function) advances its 256-bit counter by one before
    # each block of four 64-bit outputs
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(counter, dtype=np.uint64))
    raw = [int(x) for x in bg.random_raw(8)]
    c = list(counter)
    for block in range(2):
        c[0] = (c[0] + 1) & MASK
        if c[0] == 0:
            c[1] = (c[1] + 1) & MASK
        assert rng.philox4x64_10(c, key) == raw[4 * block:4 * block + 4]


def test_uniforms_open_interval_and_normals_moments():
    u = np.array([rng.uniforms(9, s, a) for s in range(50) for a in range(100)])
    assert u.min() > 0.0 and u.max() < 1.0
    z = np.array([rng.normals3(9, s, a) for s in range(100) for a in range(100)])  # 30000 draws
    assert np.abs(z.mean(axis=0)).max() < 0.03
    assert np.abs(z.var(axis=0) - 1.0).max() < 0.04
    zz = z.ravel()
    assert abs(np.mean(zz ** 4) - 3.0) < 0.15
    c = np.corrcoef(z.T)
    assert np.abs(c - np.eye(3)).max() < 0.03


def test_draws_depend_on_seed_step_atom():
    a = rng.normals3(1, 0, 0)
    assert a != rng.normals3(2, 0, 0) and a != rng.normals3(1, 1, 0) and a != rng.normals3(1, 0, 1)
    assert a == rng.normals3(1, 0, 0)
