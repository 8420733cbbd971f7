"""FP64 CPU oracle of the equivariant interaction — TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import or run anything in this package. The product path (the HIP library
and its Python binding) never does, and shares no code with it.

What it computes (paper: §4, the e3j backend accelerates the Clebsch-Gordan
tensor product of MACE and NequIP; Appendix F, the MACE and NequIP
hyperparameter tables fix the shapes):

  neighbours.py  radius graph from positions, species, cell and cutoff (§3.2,
                 the Graph built from a chemical system with a cutoff radius)
  sh.py          real spherical harmonics, l <= 3, component normalised
  cg.py          real Clebsch-Gordan coefficients, natural parity
  basis.py       Bessel radial basis times a polynomial cutoff envelope
  model.py       embedding -> T interaction layers (radial MLP, CG tensor
                 product, neighbour sum, per-order channel mix + self
                 connection, gate) -> readout; E = sum_i E_i (§5.3 readout
                 form with one head); forces F = -dE/dr by autograd (§5.2,
                 forces are derivatives of the energy); loss gradients
  md.py          velocity-Verlet NVE integration (§1, batched MD) and
                 BAOAB Langevin NVT (§5.5)
  rng.py         Philox4x64-10 counter-based random numbers (§5.5 seeds)

The paper prints no equation for the interaction itself; every modelling
choice is a reading anchored to the nearest printed hyperparameter. Each
function is pinned by tests against mathematics the paper's setting fixes
(library routines, closed forms, invariances, finite differences). Absolute
energy values of the assembled model are pinned only through those
properties: parity unpinned for the absolute value of `model.energy`.
"""
from . import sh, cg, basis, neighbours, model, md, rng  # noqa: F401
