"""Real spherical harmonics up to l = 3 (oracle).

Reading (the paper uses harmonics up to l_max 2 and 3, Appendix F tables,
without fixing a convention): the standard orthonormal real harmonics scaled
by sqrt(4*pi), so that sum_m Y_lm(n)^2 = 2l+1 ("component" normalisation),
ordered m = -l..l, component index l*l + (m + l). Evaluated on the unit
vector n = v/|v| = (x, y, z):

  l=0  1
  l=1  sqrt3 (y, z, x)
  l=2  sqrt15 xy, sqrt15 yz, sqrt5/2 (3z^2-1), sqrt15 xz, sqrt15/2 (x^2-y^2)
  l=3  sqrt(35/8) y(3x^2-y^2), sqrt105 xyz, sqrt(21/8) y(5z^2-1),
       sqrt7/2 z(5z^2-3), sqrt(21/8) x(5z^2-1), sqrt105/2 z(x^2-y^2),
       sqrt(35/8) x(x^2-3y^2)

Pinned by tests against scipy's complex harmonics (converted to the real
basis), the addition theorem with scipy's Legendre polynomials, parity and
quadrature orthonormality.
"""
import math

import torch


def real_sh(vec: torch.Tensor, lmax: int) -> torch.Tensor:
    """[..., 3] vectors (any length > 0) -> [..., (lmax+1)^2] harmonics of their direction."""
    if not 0 <= lmax <= 3:
        raise ValueError("lmax must be in 0..3")
    n = vec / torch.linalg.norm(vec, dim=-1, keepdim=True)
    x, y, z = n[..., 0], n[..., 1], n[..., 2]
    out = [torch.ones_like(x)]
    if lmax >= 1:
        s3 = math.sqrt(3.0)
        out += [s3 * y, s3 * z, s3 * x]
    if lmax >= 2:
        s15 = math.sqrt(15.0)
        out += [s15 * x * y, s15 * y * z, math.sqrt(5.0) / 2.0 * (3.0 * z * z - 1.0),
                s15 * x * z, s15 / 2.0 * (x * x - y * y)]
    if lmax >= 3:
        out += [math.sqrt(35.0 / 8.0) * y * (3.0 * x * x - y * y),
                math.sqrt(105.0) * x * y * z,
                math.sqrt(21.0 / 8.0) * y * (5.0 * z * z - 1.0),
                math.sqrt(7.0) / 2.0 * z * (5.0 * z * z - 3.0),
                math.sqrt(21.0 / 8.0) * x * (5.0 * z * z - 1.0),
                math.sqrt(105.0) / 2.0 * z * (x * x - y * y),
                math.sqrt(35.0 / 8.0) * x * (x * x - 3.0 * y * y)]
    return torch.stack(out, dim=-1)


def sl(l: int) -> slice:
    """Slice of the components of order l in a [..., (lmax+1)^2] tensor."""
    return slice(l * l, (l + 1) * (l + 1))
