"""CPU FP64 oracle for the Difference Potentials Method auxiliary-problem path.

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously-correct NumPy implementations of what the
GPU path computes, written from the paper (Epshteyn & Xia, "Efficient Numerical Algorithms
based on Difference Potentials for Chemotaxis Systems in 3D", Sec. 2).  Only tests/, the
smoke() entry point and bench.py's cpu_baseline leg may import anything here; the product
library never does, and this package never imports the product library.

Modules:
  aux       -- the auxiliary problem (AP) solve by dense DST-I eigen-decomposition, O(N^4)
  geometry  -- point sets M+/M-/N+/N-/gamma (Def. "point sets"), projection onto Gamma
  basis     -- real spherical harmonics for the spectral boundary representation
  dpm       -- particular solution, difference potential, BEP matrix, least squares, Green's formula
  pks       -- the IMEX right-hand sides of the chemotaxis scheme (upwind, minmod) and one DPM step

Parity status: every function is pinned by tests/test_oracle_*.py against brute force,
closed forms, invariants or theorems of the paper; none is "parity unpinned" except the
values of a full PKS time step against the paper's tables (the paper leaves the boundary-slope
and initial-trace details open, and prints no per-step data).
"""
