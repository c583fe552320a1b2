"""CPU oracle for the mixed-precision tile Cholesky / Gaussian log-likelihood path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, links or executes anything in this package; only the
tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
call it.  It shares no code with the HIP path: every function here is written
from the paper's statement of the operations (section and equation cited in
each docstring) or from the textbook definition, in float64 with plain numpy.

Modules
  fpformat    round-to-format emulation (FP32, FP16, BF16, FP8-E4M3FN), bit codes
  covariance  Matérn covariance for half-integer smoothness, Morton ordering
  dense       plain FP64 Cholesky, triangular solves, log-determinant, log-likelihood, GEMM
  tiled       per-tile precision map and the emulated mixed-precision tile Cholesky
  refine      preconditioned conjugate gradients and classical iterative refinement
  gemm        multi-format GEMM emulation (incl. FP8 with power-of-two block scales)

Every function is pinned by tests against something other than itself (closed
forms, exact rational arithmetic, library routines, invariances); the pins are
listed in tests/test_oracle_*.py.
"""
