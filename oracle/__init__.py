"""CPU oracle for the hierarchical multigrid finite cell solver (FP64).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test-suite, the smoke check and the CPU leg of
the benchmark use it.  It shares no code with the GPU library; the only common
input is the seeded problem descriptor from ``fcm_inputs``.

The oracle is deliberately plain and slow:
  * ``basis``      -- integrated Legendre modes (Section 2.1 / p-FEM basis)
  * ``geometry``   -- indicator function alpha and box classification (Sec. 2.1, eq. weakform)
  * ``fcm``        -- DOFs, cut-cell integration by recursive bisection, assembly
  * ``mg``         -- additive Schwarz smoother (eq. AdditiveSchwarz), V-cycle (Alg. 1),
                      hierarchical transfers (eq. restrictionoperation), PCG and MG solver.
  * ``mlhp``       -- multi-level hp overlay discretisation (Section 2.2) and its
                      hp-multigrid levels and node-patch Schwarz blocks (Section 3.2).

Every floating-point computation is IEEE double precision.

Parity pins: see tests/test_oracle_*.py.  Parity unpinned: none of the
functions below is unpinned; the paper's exact iteration counts are not
reproduced because its geometries exist only in figures.
"""
from . import basis, geometry, fcm, mg, mlhp  # noqa: F401
