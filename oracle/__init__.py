"""Plain FP64 CPU oracle for the matrix-free monolithic multigrid method for
Q_k-Q_{k-1} Taylor-Hood Stokes / generalized Stokes systems (Jodlbauer, Langer,
Wick, Zulehner, "Matrix-free Monolithic Multigrid Methods for Stokes and
Generalized Stokes Problems").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or run
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (``paper_2205_15770_amd``); the only module both sides read is the
seeded input generator ``synth_inputs``, which holds none of the method's
arithmetic.

Where the HIP library is matrix-free, the oracle is the plain definition: it
assembles the sparse matrices A, B, M_p (and C) of the Taylor-Hood
discretisation cell by cell with explicit Lagrange basis functions and Gauss
quadrature, applies the Dirichlet conditions by zeroing rows and columns, and
runs the paper's algorithms (Chebyshev-Jacobi, inexact symmetric Uzawa,
multigrid cycle, coarse direct solve) step by step on those matrices.

Modules
  fe        1D nodes, Lagrange basis, Gauss rule              (Section 2)
  mesh      box mesh hierarchy, DoF numbering, geometry      (Sections 2, 3.1)
  assemble  element matrices, CSR assembly, Dirichlet, RHS   (Section 2, Eq. (2.1)-(2.3))
  transfer  canonical-injection prolongation, R = P^T        (Section 3.2)
  smoother  diagonals, Lanczos, Chebyshev-Jacobi, Uzawa      (Section 3.3.1, Algorithm 2)
  mg        multigrid cycle, bordered coarse solve           (Algorithm 1, Section 4.1)
  krylov    FGMRES outer loop, stationary iteration, rate q  (Section 4.1)
  rows      single rows of K x for sampled checks at full size
"""
