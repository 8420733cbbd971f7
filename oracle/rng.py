"""Counter-based random numbers for the stochastic integrators (oracle).

§5.5 runs Langevin dynamics on batches of independent systems, each with its
own random seed. Random numbers that the method draws cannot be handed in
from outside for a long trajectory, so the oracle and the device each
implement the same counter-based generator from its published definition:
Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11). A draw is a
pure function of (key, counter), so a structure's noise depends only on its
own seed, step and atom index, not on what else is packed with it.

Reading used by both sides:
  key     = (seed, 0)
  counter = (step, local atom index, 0, 0)
  u_k     = ((x_k >> 11) + 1/2) / 2^53, k = 0..3     (uniform in (0, 1))
  normals = Box-Muller on (u_0, u_1) and (u_2, u_3):
            z_0 = sqrt(-2 ln u_0) cos(2 pi u_1), z_1 = sqrt(-2 ln u_0) sin(2 pi u_1),
            z_2 = sqrt(-2 ln u_2) cos(2 pi u_3)        (three per atom and step)

Pinned by tests: the block function against numpy's Philox bit generator
(an independent implementation of the same published function), and the
moments of the normals.
"""
import math
from typing import List, Sequence, Tuple

_MASK = (1 << 64) - 1
_M0, _M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157   # round multipliers
_W0, _W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B   # key schedule (Weyl) increments


def philox4x64_10(counter: Sequence[int], key: Sequence[int]) -> List[int]:
    """The Philox4x64 block function, 10 rounds, on Python integers."""
    c = [int(x) & _MASK for x in counter]
    k = [int(x) & _MASK for x in key]
    for _ in range(10):
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        c = [(p1 >> 64) ^ c[1] ^ k[0], p1 & _MASK, (p0 >> 64) ^ c[3] ^ k[1], p0 & _MASK]
        k = [(k[0] + _W0) & _MASK, (k[1] + _W1) & _MASK]
    return c


def uniforms(seed: int, step: int, atom: int) -> Tuple[float, float, float, float]:
    x = philox4x64_10((step, atom, 0, 0), (seed, 0))
    return tuple(((v >> 11) + 0.5) * 2.0 ** -53 for v in x)


def barostat_uniforms(seed: int, move: int) -> Tuple[float, float]:
    """Two uniforms for the move-th volume proposal of a structure: key
    (seed, 1), counter (move, 0, 0, 0) (a stream apart from the thermostat's)."""
    x = philox4x64_10((move, 0, 0, 0), (seed, 1))
    return ((x[0] >> 11) + 0.5) * 2.0 ** -53, ((x[1] >> 11) + 0.5) * 2.0 ** -53


def normals3(seed: int, step: int, atom: int) -> Tuple[float, float, float]:
    """Three standard normal draws for one atom at one step."""
    u0, u1, u2, u3 = uniforms(seed, step, atom)
    r0 = math.sqrt(-2.0 * math.log(u0))
    r1 = math.sqrt(-2.0 * math.log(u2))
    return (r0 * math.cos(2.0 * math.pi * u1), r0 * math.sin(2.0 * math.pi * u1), r1 * math.cos(2.0 * math.pi * u3))
