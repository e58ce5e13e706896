"""Seeded synthetic inputs shared by the oracle-based tests and the benchmark.

This module holds random-number draws only: no discretization, geometry or
solver arithmetic lives here, so both the CPU oracle and the GPU path can take
their inputs from it without sharing any of the method's code.

Every generator is NumPy's PCG64 (``numpy.random.default_rng(seed)``).
"""
import numpy as np

# Seeds of the standard workloads (input vectors and fields).
SEED_CG_Q2_SMALL = 0       # CG Q2, 8^3 cells, apply input
SEED_CG_Q4_CURVED = 1      # CG Q4, 64^3 curved cells, apply input
SEED_SIPG_Q3 = 3           # SIPG Q3, 32^3 cells
SEED_SIPG_Q5 = 4           # SIPG Q5, 32^3 cells
SEED_KAPPA_FIELD = 5       # log-diffusivity field g
SEED_KAPPA_PERTURB = 6     # perturbation that defines the target state
SEED_FD_CELLS = 7          # cells probed by finite differences
SEED_MIXED_BC = 8          # apply inputs with mixed boundary conditions on (-1,1)^3


def uniform_vector(n, seed, dtype=np.float64):
    """n values drawn i.i.d. from U[-1, 1) with PCG64(seed)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, int(n)).astype(dtype)


def gaussian_field(n, seed, sigma):
    """n values drawn i.i.d. from N(0, sigma^2) with PCG64(seed)."""
    return np.random.default_rng(seed).normal(0.0, sigma, int(n))


def choose_cells(n_cells, count, seed):
    """`count` distinct cell indices out of range(n_cells), PCG64(seed)."""
    return np.sort(np.random.default_rng(seed).choice(int(n_cells), int(count), replace=False))
