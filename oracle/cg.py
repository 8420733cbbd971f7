"""Real-basis Clebsch-Gordan coefficients (oracle).

The tensor product the paper's backend accelerates (§4) couples features of
order l1 with harmonics of order l2 into order l3 through Clebsch-Gordan
coefficients (§2, steerable convolutions built on CG tensor products).

Reading (natural parity only, `include_pseudotensors False` in the MACE table
of Appendix F): a path (l1, l2, l3) exists when |l1-l2| <= l3 <= l1+l2 and
l1+l2+l3 is even. Its coefficient tensor C in R^{(2l1+1)x(2l2+1)x(2l3+1)} is
defined as the unique rotation-equivariant bilinear map in the real basis of
`sh.real_sh`:
  * equivariance: C(D1 a, D2 b) = D3 C(a, b) for every rotation,
  * normalisation: sum_{m1 m2} C[m1,m2,m3] C[m1,m2,m3'] = delta(m3, m3'),
  * sign: sum_{m1 m2} C[m1,m2,m3] Y1(n) Y2(n) = +c Y3(n) with c > 0.

This is computed literally: the real Wigner matrices D_l(R) are obtained from
the harmonics themselves (Y_l(R n) = D_l(R) Y_l(n), solved by least squares
over sample directions), the invariance constraint is stacked for a few
rotations and its one-dimensional null space is taken by SVD, then scaled and
signed as above.

Pinned by tests against sympy's complex Clebsch-Gordan coefficients (both
the closed form for |c| and the full tensor after the complex -> real change
of basis), orthonormality and rotation invariance of the coupled triple.
"""
import functools
import math
from typing import List, Tuple

import numpy as np
import torch

from .sh import real_sh


def rotation(alpha: float, beta: float, gamma: float) -> np.ndarray:
    """Rotation matrix Rz(alpha) Ry(beta) Rz(gamma)."""
    def rz(a):
        c, s = math.cos(a), math.sin(a)
        return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])

    def ry(a):
        c, s = math.cos(a), math.sin(a)
        return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])
    return rz(alpha) @ ry(beta) @ rz(gamma)


def _sample_dirs(k: int = 64) -> np.ndarray:
    # Fixed, well-spread directions (a Fibonacci sphere); any set spanning
    # the harmonics of order <= 3 would do.
    i = np.arange(k) + 0.5
    z = 1.0 - 2.0 * i / k
    phi = math.pi * (1.0 + math.sqrt(5.0)) * i
    r = np.sqrt(1.0 - z * z)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def wigner_d(l: int, R: np.ndarray) -> np.ndarray:
    """Real Wigner matrix with Y_l(R n) = D Y_l(n) for every direction n."""
    n = _sample_dirs()
    sl = slice(l * l, (l + 1) * (l + 1))
    Y = real_sh(torch.from_numpy(n), l)[:, sl].numpy()            # [k, 2l+1]
    Yr = real_sh(torch.from_numpy(n @ R.T), l)[:, sl].numpy()     # rows Y(R n_k)
    # Yr = Y D^T  ->  D^T = lstsq(Y, Yr)
    Dt, *_ = np.linalg.lstsq(Y, Yr, rcond=None)
    return Dt.T


_CONSTRAINT_ROTATIONS = [(0.3, 1.1, 2.0), (2.5, 0.4, -1.3), (-0.9, 2.2, 0.7)]


@functools.lru_cache(maxsize=None)
def real_cg(l1: int, l2: int, l3: int) -> np.ndarray:
    """C[m1, m2, m3] for a natural-parity path; raises for a forbidden one."""
    if not (abs(l1 - l2) <= l3 <= l1 + l2) or (l1 + l2 + l3) % 2:
        raise ValueError(f"no natural-parity path ({l1},{l2},{l3})")
    d1, d2, d3 = 2 * l1 + 1, 2 * l2 + 1, 2 * l3 + 1
    rows = []
    for ang in _CONSTRAINT_ROTATIONS:
        R = rotation(*ang)
        K = np.kron(np.kron(wigner_d(l1, R).T, wigner_d(l2, R).T), wigner_d(l3, R).T)
        rows.append(K - np.eye(d1 * d2 * d3))
    M = np.concatenate(rows, axis=0)
    _, s, vt = np.linalg.svd(M)
    null = vt[-1]
    if s[-1] > 1e-9 or (len(s) > 1 and s[-2] < 1e-6):
        raise RuntimeError(f"equivariant map for ({l1},{l2},{l3}) is not unique")
    C = null.reshape(d1, d2, d3)
    C *= math.sqrt(d3) / np.linalg.norm(C)
    n = np.array([[0.31, -0.52, 0.79]])
    y = real_sh(torch.from_numpy(n), max(l1, l2, l3))[0].numpy()
    v = np.einsum("abc,a,b->c", C, y[l1 * l1:(l1 + 1) ** 2], y[l2 * l2:(l2 + 1) ** 2])
    if float(v @ y[l3 * l3:(l3 + 1) ** 2]) < 0.0:
        C = -C
    return C


def paths(l_in: List[int], lmax: int) -> List[Tuple[int, int, int]]:
    """Natural-parity paths (l1, l2, l3) with l1 in l_in and l2, l3 <= lmax,
    ordered by (l3, l1, l2)."""
    out = []
    for l3 in range(lmax + 1):
        for l1 in l_in:
            for l2 in range(lmax + 1):
                if abs(l1 - l2) <= l3 <= l1 + l2 and (l1 + l2 + l3) % 2 == 0:
                    out.append((l1, l2, l3))
    return out
