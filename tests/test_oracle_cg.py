"""Pins of the oracle's real Clebsch-Gordan tensors against sympy and invariants."""
import math

import numpy as np
import pytest
import torch
from sympy import S
from sympy.physics.quantum.cg import CG

from oracle import cg
from oracle.sh import real_sh

ALL = cg.paths([0, 1, 2, 3], 3)


def test_path_counts():
    assert len(ALL) == 23
    assert [sum(1 for p in ALL if p[2] == l3) for l3 in range(4)] == [4, 6, 7, 6]
    assert len(cg.paths([0], 3)) == 4
    assert len(cg.paths([0, 1, 2], 2)) == 11
    assert len(cg.paths([0], 2)) == 3
    for (l1, l2, l3) in ALL:
        assert (l1 + l2 + l3) % 2 == 0 and abs(l1 - l2) <= l3 <= l1 + l2


def _sympy_cg(l1, m1, l2, m2, l3, m3):
    return float(CG(S(l1), S(m1), S(l2), S(m2), S(l3), S(m3)).doit())


def _c_coefficient(C, l1, l2, l3, n):
    y = real_sh(torch.from_numpy(n[None]), 3)[0].numpy()
    v = np.einsum("abc,a,b->c", C, y[l1 * l1:(l1 + 1) ** 2], y[l2 * l2:(l2 + 1) ** 2])
    y3 = y[l3 * l3:(l3 + 1) ** 2]
    return v, float(v @ y3 / (y3 @ y3)), y3


@pytest.mark.parametrize("path", ALL)
def test_coupling_constant_closed_form(path):
    l1, l2, l3 = path
    C = cg.real_cg(*path)
    expected = math.sqrt((2 * l1 + 1) * (2 * l2 + 1) / (2 * l3 + 1)) * abs(_sympy_cg(l1, 0, l2, 0, l3, 0))
    for n in np.random.default_rng(0).standard_normal((3, 3)):
        n = n / np.linalg.norm(n)
        v, c, y3 = _c_coefficient(C, l1, l2, l3, n)
        np.testing.assert_allclose(v, c * y3, atol=1e-12)   # proportional to Y_l3
        assert c > 0
        assert abs(c - expected) < 1e-12


def _U(l):
    """Rows: real harmonic index m (-l..l); columns: complex index m' (-l..l)."""
    U = np.zeros((2 * l + 1, 2 * l + 1), dtype=complex)
    r2 = 1.0 / math.sqrt(2.0)
    for m in range(-l, l + 1):
        if m > 0:
            U[m + l, m + l] = (-1) ** m * r2
            U[m + l, -m + l] = r2
        elif m < 0:
            U[m + l, m + l] = 1j * r2
            U[m + l, -m + l] = -1j * (-1) ** m * r2
        else:
            U[l, l] = 1.0
    return U


@pytest.mark.parametrize("path", ALL)
def test_matches_sympy_tensor_in_real_basis(path):
    l1, l2, l3 = path
    cc = np.zeros((2 * l1 + 1, 2 * l2 + 1, 2 * l3 + 1))
    for m1 in range(-l1, l1 + 1):
        for m2 in range(-l2, l2 + 1):
            m3 = m1 + m2
            if abs(m3) <= l3:
                cc[m1 + l1, m2 + l2, m3 + l3] = _sympy_cg(l1, m1, l2, m2, l3, m3)
    U1, U2, U3 = _U(l1), _U(l2), _U(l3)
    creal = np.einsum("ai,bj,ck,ijk->abc", U1.conj(), U2.conj(), U3, cc)
    k = np.unravel_index(np.argmax(np.abs(creal)), creal.shape)
    creal = creal / (creal[k] / abs(creal[k]))          # remove a global phase
    assert np.max(np.abs(creal.imag)) < 1e-12
    creal = creal.real
    n = np.array([0.2, 0.7, -0.4])
    n /= np.linalg.norm(n)
    _, c, _ = _c_coefficient(creal, l1, l2, l3, n)
    if c < 0:
        creal = -creal
    np.testing.assert_allclose(cg.real_cg(*path), creal, atol=1e-12)


@pytest.mark.parametrize("path", ALL)
def test_orthonormal(path):
    C = cg.real_cg(*path)
    np.testing.assert_allclose(np.einsum("abc,abd->cd", C, C), np.eye(C.shape[2]), atol=1e-12)


@pytest.mark.parametrize("path", ALL)
def test_coupled_triple_is_rotation_invariant(path):
    # sum C Y1(a) Y2(b) Y3(c) must not change when a, b, c rotate together.
    l1, l2, l3 = path
    C = cg.real_cg(*path)
    rng = np.random.default_rng(5)
    a, b, c = rng.standard_normal((3, 3))

    def inv(a, b, c):
        ya = real_sh(torch.from_numpy(a[None]), 3)[0].numpy()[l1 * l1:(l1 + 1) ** 2]
        yb = real_sh(torch.from_numpy(b[None]), 3)[0].numpy()[l2 * l2:(l2 + 1) ** 2]
        yc = real_sh(torch.from_numpy(c[None]), 3)[0].numpy()[l3 * l3:(l3 + 1) ** 2]
        return np.einsum("abc,a,b,c->", C, ya, yb, yc)
    base = inv(a, b, c)
    for ang in [(0.1, 0.2, 0.3), (1.9, -0.7, 2.4)]:
        R = cg.rotation(*ang)
        assert abs(inv(R @ a, R @ b, R @ c) - base) < 1e-12


def test_special_cases():
    for l in range(4):
        np.testing.assert_allclose(cg.real_cg(0, l, l)[0], np.eye(2 * l + 1), atol=1e-12)
        np.testing.assert_allclose(cg.real_cg(l, 0, l)[:, 0, :], np.eye(2 * l + 1), atol=1e-12)
        np.testing.assert_allclose(cg.real_cg(l, l, 0)[:, :, 0], np.eye(2 * l + 1) / math.sqrt(2 * l + 1),
                                   atol=1e-12)
    C = cg.real_cg(1, 1, 2)
    for m3 in range(5):
        M = C[:, :, m3]
        np.testing.assert_allclose(M, M.T, atol=1e-12)
        assert abs(np.trace(M)) < 1e-12


def test_forbidden_paths_raise():
    with pytest.raises(ValueError):
        cg.real_cg(1, 1, 1)
    with pytest.raises(ValueError):
        cg.real_cg(1, 1, 3)
