"""CPU FP64 oracle for the sparse spectral Galerkin method (test infrastructure).

This package is test infrastructure only.  Tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the solver path never does.  It
shares no code with the HIP library: it is a plain, slow, obviously correct
restatement of the paper's definitions, in float64 / complex128 and exact
integers, with numpy as the only library.

* ``stamp``    -- the stamping set S^N[a](F) by brute-force Minkowski sums
                  (Sec. 6, Eq. StampSet), first-appearance levels, lexicographic
                  slot order, and the App. A cardinality count.
* ``galerkin`` -- the truncated Galerkin operator L_N (Sec. 9, Eq.
                  FiniteGalerkinOperator), its neighbour relation, connected
                  classes (Sec. 6, proof of Prop. SolutionSupport), the dense
                  per-class matrix and the direct solve of Alg. 1, steps 3-5.

Parity pins: every function here is checked in ``tests/test_oracle_*.py``
against closed forms, brute force, physical-space evaluation of the PDE
operator and textbook solvers (see the test module docstrings).  Nothing in
this package is "parity unpinned".
"""
from . import stamp, galerkin  # noqa: F401
