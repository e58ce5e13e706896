"""Matrix-free high-order Laplace operators and multigrid solvers on AMD MI355X (gfx950).

The compute path is libmfl.so (hand-written HIP kernels behind the C ABI in
include/mfl.h); this package only marshals torch tensors into it.
"""
from ._mfl import (CARTESIAN, CG, CURVED, DIRICHLET, F32, F64, KAPPA_CELLWISE, KAPPA_COSINE,
                   METRIC_AUTO, METRIC_ON_THE_FLY, METRIC_STORED, MIXED, NEUMANN, SIPG, MflError, Problem,
                   apply_noalloc, check_vector, lib, make_params, query)
from .autograd import PoissonSolve

__all__ = ["Problem", "PoissonSolve", "MflError", "lib", "make_params", "query", "CG", "SIPG",
           "CARTESIAN", "CURVED", "DIRICHLET", "NEUMANN", "MIXED", "F64", "F32", "KAPPA_CELLWISE",
           "KAPPA_COSINE", "METRIC_AUTO", "METRIC_STORED", "METRIC_ON_THE_FLY", "check_vector",
           "apply_noalloc"]
