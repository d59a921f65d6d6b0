"""Oracle: a plain, slow, FP64 CPU implementation of the LEE lattice Boltzmann scheme.

TEST INFRASTRUCTURE.  Only the test suite, the package smoke check and the benchmark's
CPU-baseline leg may import, call, link or run anything in this package.  It shares no
code with the GPU library and imports nothing from it.

Contents (each function cites the part of the paper it follows):
  lattices      velocity sets and coefficients, generated from the paper's formulas
  lbe           moments, equilibrium, update matrices H(tau) / Gamma(k), the C stepper, norms
  closed_forms  d'Alembert, plane waves (continuum and Gamma(k)^n) and the 3D radial pulse
  mlp           FP64 forward/backward of the boundary-closure network (not in the paper)

Parity status of each part is recorded in the test suite; the reduced-precision storage
modes and the learned boundary closure are not in the paper, so their parity is pinned
only against this FP64 oracle ("parity unpinned" beyond it).
"""
from . import lattices  # noqa: F401
