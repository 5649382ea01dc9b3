"""Plain FP64 CPU oracle for the AMG multilevel-correction eigensolver.

TEST INFRASTRUCTURE ONLY.  Nothing in the eigensolver library imports, links
or calls this package; only the tests, the smoke check and the benchmark's CPU
baseline use it.  It shares no code with the GPU path: its AMG setup, V-cycle,
Rayleigh-Ritz and driver are written here from the paper, with numpy/scipy
library primitives (sparse products, dense symmetric-definite eigensolver) and
three plain-C loops (Ruge-Stueben first and second pass, Gauss-Seidel sweep).

Pins (tests/test_oracle_*.py): dense brute-force eigensolves for N <= 2000, the
closed-form spectrum of the lumped-mass unit-square problem, a hand-derived
1D hierarchy, hand-traced Ruge-Stueben passes, level-2 sizes (N+1)/2 on
5-point grids, the Galerkin chain identity, the M-orthonormality and
Ritz-bound invariants, the exact-eigenpair fixed point, the V-cycle
contraction bounds and the relative-residual closed form.
"""
from . import amg, eigensolver, native  # noqa: F401
from .eigensolver import Oracle, guard_count  # noqa: F401
