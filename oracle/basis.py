"""Radial basis (oracle).

Reading of the NequIP table of Appendix F (`num_rbf 8`,
`radial_envelope polynomial_envelope`; also in the MACE table): the Bessel
functions b_n(r) = sqrt(2/r_c) sin(n pi r / r_c) / r, n = 1..n_basis, times
the polynomial envelope of exponent p (the paper does not give p; p = 6)

  u(x) = 1 - (p+1)(p+2)/2 x^p + p(p+2) x^(p+1) - p(p+1)/2 x^(p+2),  x = r/r_c < 1
  u(x) = 0                                                             x >= 1.

Pinned by tests: orthonormality of b_n under the r^2 weight on [0, r_c]
(scipy quadrature), u(0) = 1, u(1) = u'(1) = u''(1) = 0, and the closed
form u'(x) = -p(p+1)(p+2)/2 x^(p-1) (1-x)^2.
"""
import math

import torch


def bessel(r: torch.Tensor, cutoff: float, n_basis: int) -> torch.Tensor:
    """[...] distances -> [..., n_basis]."""
    n = torch.arange(1, n_basis + 1, dtype=r.dtype)
    return math.sqrt(2.0 / cutoff) * torch.sin(n * math.pi * r[..., None] / cutoff) / r[..., None]


def envelope(x: torch.Tensor, p: int) -> torch.Tensor:
    poly = (1.0 - (p + 1) * (p + 2) / 2.0 * x ** p + p * (p + 2) * x ** (p + 1)
            - p * (p + 1) / 2.0 * x ** (p + 2))
    return torch.where(x < 1.0, poly, torch.zeros_like(x))


def radial_basis(r: torch.Tensor, cutoff: float, n_basis: int, p: int) -> torch.Tensor:
    """B_n(r) = b_n(r) u(r / r_c), [...] -> [..., n_basis]."""
    return bessel(r, cutoff, n_basis) * envelope(r / cutoff, p)[..., None]
