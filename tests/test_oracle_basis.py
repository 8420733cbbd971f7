"""Pins of the oracle's radial basis against quadrature and closed forms."""
import numpy as np
import pytest
import torch
from scipy.integrate import quad

from oracle import basis


def test_bessel_orthonormal_with_r2_weight():
    rc = 5.0
    n_basis = 8

    def b(n, r):
        return basis.bessel(torch.tensor([r], dtype=torch.float64), rc, n_basis)[0, n].item()
    G = np.zeros((n_basis, n_basis))
    for i in range(n_basis):
        for j in range(i, n_basis):
            G[i, j] = G[j, i] = quad(lambda r: b(i, r) * b(j, r) * r * r, 1e-9, rc, limit=200)[0]
    np.testing.assert_allclose(G, np.eye(n_basis), atol=1e-9)


@pytest.mark.parametrize("p", [5, 6, 8])
def test_envelope_endpoints_and_derivative(p):
    x = torch.linspace(0.01, 0.999, 41, dtype=torch.float64, requires_grad=True)
    u = basis.envelope(x, p)
    (du,) = torch.autograd.grad(u.sum(), x)
    xd = x.detach()
    closed = -p * (p + 1) * (p + 2) / 2.0 * xd ** (p - 1) * (1 - xd) ** 2
    np.testing.assert_allclose(du.numpy(), closed.numpy(), atol=1e-12)
    assert basis.envelope(torch.tensor(0.0, dtype=torch.float64), p).item() == 1.0
    # the polynomial and its first two derivatives vanish at x -> 1 from below
    x1 = torch.tensor(1.0 - 1e-7, dtype=torch.float64, requires_grad=True)
    u1 = basis.envelope(x1, p)
    (g1,) = torch.autograd.grad(u1, x1, create_graph=True)
    (g2,) = torch.autograd.grad(g1, x1)
    assert abs(u1.item()) < 1e-13 and abs(g1.item()) < 1e-10 and abs(g2.item()) < 1e-4


def test_zero_at_and_beyond_cutoff():
    r = torch.tensor([5.0, 5.5, 7.0], dtype=torch.float64)
    assert torch.all(basis.radial_basis(r, 5.0, 8, 6) == 0)


def test_envelope_value_closed_form():
    # For p = 6 the envelope equals 1 - 28 x^6 + 48 x^7 - 21 x^8, which is
    # (1-x)^3 times a cubic: check it against that factorised form.
    x = torch.linspace(0, 0.99, 30, dtype=torch.float64)
    fact = (1 - x) ** 3 * (1 + 3 * x + 6 * x ** 2 + 10 * x ** 3 + 15 * x ** 4 + 21 * x ** 5)
    np.testing.assert_allclose(basis.envelope(x, 6).numpy(), fact.numpy(), atol=1e-13)
