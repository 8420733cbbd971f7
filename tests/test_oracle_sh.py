"""Pins of the oracle's real spherical harmonics against scipy and closed forms."""
import math

import numpy as np
import pytest
import scipy.special as sp
import torch

from oracle.sh import real_sh


def _dirs(k, seed=0):
    v = np.random.default_rng(seed).standard_normal((k, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _scipy_real(l, m, n):
    """Real harmonic from scipy's complex one (Condon-Shortley phase included),
    scaled to component normalisation."""
    theta = np.arccos(np.clip(n[:, 2], -1, 1))
    phi = np.arctan2(n[:, 1], n[:, 0])
    y = sp.sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        val = math.sqrt(2.0) * (-1) ** m * y.real
    elif m < 0:
        val = math.sqrt(2.0) * (-1) ** m * y.imag
    else:
        val = y.real
    return math.sqrt(4.0 * math.pi) * val


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_matches_scipy_complex_harmonics(l):
    n = _dirs(50)
    ours = real_sh(torch.from_numpy(n * 2.7), 3).numpy()
    for m in range(-l, l + 1):
        np.testing.assert_allclose(ours[:, l * l + m + l], _scipy_real(l, m, n), atol=1e-13)


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_addition_theorem(l):
    a, b = _dirs(40, 1), _dirs(40, 2)
    ya = real_sh(torch.from_numpy(a), 3).numpy()[:, l * l:(l + 1) ** 2]
    yb = real_sh(torch.from_numpy(b), 3).numpy()[:, l * l:(l + 1) ** 2]
    lhs = np.sum(ya * yb, axis=1)
    rhs = (2 * l + 1) * sp.eval_legendre(l, np.sum(a * b, axis=1))
    np.testing.assert_allclose(lhs, rhs, atol=1e-13)


def test_parity():
    n = _dirs(30, 3)
    y = real_sh(torch.from_numpy(n), 3).numpy()
    ym = real_sh(torch.from_numpy(-n), 3).numpy()
    for l in range(4):
        s = slice(l * l, (l + 1) ** 2)
        np.testing.assert_allclose(ym[:, s], (-1) ** l * y[:, s], atol=1e-15)


def test_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi: exact for degree <= 6 products.
    xg, wg = np.polynomial.legendre.leggauss(8)
    nphi = 16
    phi = 2 * np.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    n = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    y = real_sh(torch.from_numpy(n), 3).numpy()
    gram = (y * w[:, None]).T @ y / (4 * np.pi)
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-13)


def test_scale_invariant():
    n = _dirs(10, 4)
    np.testing.assert_allclose(real_sh(torch.from_numpy(n), 3).numpy(),
                               real_sh(torch.from_numpy(n * 0.37), 3).numpy(), atol=1e-14)
