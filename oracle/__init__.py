"""FP64 CPU oracle for the sparse lattice-Boltzmann step — TEST INFRASTRUCTURE.

A plain, slow, obviously correct NumPy implementation of what the GPU path
computes, used only to check it: only ``tests/``, the smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code, constants or
tables with the GPU library; both sides take their inputs from ``workloads``.

The paper (Section 2) names the ingredients without formulas: a lattice
Boltzmann method on a sparse lattice of fluid sites, the D3Q19 lattice,
propagation and collision steps, Ladd velocity iolets, and (Section 4) simple
bounce-back walls.  The formulas here are the textbook definitions behind
those names (Krueger et al., The Lattice Boltzmann Method, 2017: ch. 3 for the
equilibrium and BGK collision, ch. 5 for bounce-back and moving walls); every
place where the paper is silent follows the reading recorded in the design
notes.

Modules:
  lattice  - D3Q15 / D3Q19 velocity sets and weights (exact rationals)
  links    - upstream classification of every (site, direction) pair
  lbgk     - sparse FP64 step: pull streaming + boundary rules + LBGK collision,
             observables (pressure, velocity, stress, wall shear stress), totals
  dense    - the same step on a dense box with shifted arrays (cross-check)
  adjoint  - reverse-mode (discrete adjoint) of the step and objective
"""
