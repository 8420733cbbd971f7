"""Radius graph by brute force (oracle).

§3.2 of the paper builds the graph from a chemical system (positions, atomic
numbers, cell) and a cutoff radius (`graph_cutoff_angstrom`, 5.0 in every
Appendix F table); several structures are handled as one batch (§1).

Definition used here: for every structure, all directed edges i <- j with an
integer image vector n (n_a = 0 along non-periodic axes) such that
  d = r_j - r_i + n . cell,   0 < |d| < r_c,
which includes several images of one neighbour and an atom's own images
when the cell is shorter than r_c, and excludes i = j with n = 0. Edges never
join different structures. Output is sorted by (i, j, n).

Every image vector that can reach the cutoff is tried against every pair:
O(N^2 x images) per structure. Pinned by tests: symmetry of the edge set,
neighbour counts, and replicated-supercell consistency.
"""
import math
from typing import Tuple

import numpy as np


def _image_range(cell: np.ndarray, cutoff: float, periodic: bool, axis: int) -> int:
    """Largest |n_a| that can reach the cutoff between two wrapped atoms
    (fractional coordinates in [0, 1), so they differ by less than one cell)."""
    if not periodic:
        return 0
    vol = abs(np.linalg.det(cell))
    b, c = cell[(axis + 1) % 3], cell[(axis + 2) % 3]
    width = vol / np.linalg.norm(np.cross(b, c))   # perpendicular width of the cell
    return int(math.floor(1.0 + cutoff / width))


def neighbour_list(pos: np.ndarray, cell: np.ndarray, pbc: np.ndarray, offsets: np.ndarray,
                   cutoff: float) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Returns (dst, src, shift): receivers i, senders j (global atom indices)
    and integer image vectors n [E, 3], sorted by (i, j, n).

    The image vector n refers to the positions as given. Candidate images
    are enumerated around the wrapped positions (which only bounds the search);
    every distance is then evaluated as (r_j - r_i) + n . cell."""
    dst_all, src_all, sh_all = [], [], []
    for s in range(len(offsets) - 1):
        a, b = int(offsets[s]), int(offsets[s + 1])
        x = np.asarray(pos[a:b], dtype=np.float64)
        n_s = b - a
        if n_s == 0:
            continue
        cs = np.asarray(cell[s], dtype=np.float64)
        per = np.array([bool(pbc[s][k]) for k in range(3)])
        frac = x @ np.linalg.inv(cs)
        wrap = np.where(per[None, :], np.floor(frac), 0.0).astype(np.int64)   # r = r_wrapped + wrap . cell
        ranges = [_image_range(cs, cutoff, per[k], k) for k in range(3)]
        diff = x[None, :, :] - x[:, None, :]          # [i, j, 3] = r_j - r_i
        dwrap = wrap[:, None, :] - wrap[None, :, :]   # wrap_i - wrap_j
        same = np.eye(n_s, dtype=bool)
        for nx in range(-ranges[0], ranges[0] + 1):
            for ny in range(-ranges[1], ranges[1] + 1):
                for nz in range(-ranges[2], ranges[2] + 1):
                    n = np.array([nx, ny, nz]) + dwrap                   # image vector for the raw positions
                    d = diff + n.astype(np.float64) @ cs
                    r2 = np.einsum("ijk,ijk->ij", d, d)
                    mask = (r2 < cutoff * cutoff) & ~(same & np.all(n == 0, axis=2))
                    ii, jj = np.nonzero(mask)
                    if len(ii):
                        dst_all.append(ii + a)
                        src_all.append(jj + a)
                        sh_all.append(n[ii, jj])
    if not dst_all:
        return (np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros((0, 3), np.int64))
    dst = np.concatenate(dst_all).astype(np.int64)
    src = np.concatenate(src_all).astype(np.int64)
    sh = np.concatenate(sh_all).astype(np.int64)
    order = np.lexsort((sh[:, 2], sh[:, 1], sh[:, 0], src, dst))
    return dst[order], src[order], sh[order]


def shift_vectors(shift: np.ndarray, dst: np.ndarray, cell: np.ndarray, offsets: np.ndarray) -> np.ndarray:
    """Cartesian image displacement n . cell of each edge."""
    owner = np.searchsorted(offsets, dst, side="right") - 1
    return np.einsum("ea,eab->eb", shift.astype(np.float64), cell[owner])
