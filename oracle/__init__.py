"""Plain FP64 CPU oracle for the FOSB hot path (PEC, EFIE, combination technique).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke entry point and the
benchmark's CPU-baseline leg may import or run anything in this package; the
GPU library never calls it and shares no code with it.  Inputs come from the
seeded generators in ``workloads`` (geometry and parameters only).

Every function restates the paper's definitions in the most direct form that
numpy/scipy allow (FP64, LAPACK LU via scipy), without blocking or fusion
beyond what the definitions state:

  mesh.py        RWG tables on planar triangulations (Galerkin section)
  quadrature.py  6-point triangle rule, Gauss-Legendre, Sauter-Schwab
                 regularising transforms for touching triangle pairs
  efie.py        EFIE Galerkin matrix, incident right-hand side, far-field map
                 (EFIE and far-field definitions, problem setting section)
  uq.py          shape-derivative right-hand-side weights, covariance, RHS
                 correlation, two-sided solve, full tensor solve, combination
                 technique, far-field variance and its gradient
  mie.py         Mie series for the PEC sphere (reference solution used by the
                 sphere experiments)
  static.py      closed-form potential of a uniformly charged triangle (pins
                 the singular quadrature)

Conventions that the paper leaves open are fixed once, here and in the GPU
library alike (see each module's docstring).
"""
