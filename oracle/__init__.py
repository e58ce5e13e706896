"""CPU oracle for the matrix-free Laplace solvers (test infrastructure only).

This package is a plain, slow, FP64 transcription of what the method computes:
dense per-quadrature-point element integrals assembled into CSR matrices, a
textbook geometric-multigrid preconditioned conjugate gradient solver, and the
adjoint gradient with respect to a cellwise diffusion coefficient.  It uses no
sum factorization, no blocking and no fusion.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
it.  The GPU library never does, and this package imports nothing from the GPU
path; the two share only the seeded input generators in ``seeded_inputs``.

Functions without an independent pin say "parity unpinned" in their docstring.
"""
