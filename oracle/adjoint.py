"""Adjoint gradient of J(u) = 1/2 ||u - u_target||_2^2 with respect to a cellwise kappa.

Not part of the paper: an addition on top of its CG operator.  For A(kappa) u = b with
b independent of kappa and A linear in the cell coefficients,

    dJ/dkappa_c = -lambda^T (dA/dkappa_c) u,   A lambda = u - u_target,

and dA/dkappa_c is the element matrix of cell c at kappa = 1, restricted to
interior DoFs (Dirichlet rows and columns do not depend on kappa).  A is symmetric,
so the adjoint system uses the same operator.  The adjoint right-hand side has its
Dirichlet entries zeroed.
"""
import numpy as np
import scipy.sparse.linalg as spla

from . import cg
from .mesh import Box


def gradient(box, u, lam, kappa_fn=None):
    """g_c = -lambda_c^T A_c^{(1)} u_c with boundary entries of u, lambda zeroed.  With a
    position-dependent factor kappa_fn of the coefficient (kappa = kappa_c kappa_fn(x)),
    A_c^{(1)} is the element matrix at kappa_c = 1 with that factor kept."""
    Ae = cg.element_matrices(box, None, kappa_fn=kappa_fn)
    dofs = box.cell_dofs()
    bmask = box.boundary_mask()
    uz = np.where(bmask, 0.0, u)[dofs]
    lz = np.where(bmask, 0.0, lam)[dofs]
    return -np.einsum("ei,eij,ej->e", lz, Ae, uz)


def solve_direct(box, kappa, b, kappa_fn=None):
    A = cg.assemble(box, kappa, kappa_fn=kappa_fn)
    return spla.spsolve(A.tocsc(), b), A


def objective_and_gradient(cells_per_dim, degree, kappa, u_target, curve_amp=0.0, kappa_fn=None):
    """J and dJ/dkappa with direct solves (the plain definition)."""
    box = Box(cells_per_dim, degree, curve_amp)
    b = cg.rhs(box)
    u, A = solve_direct(box, kappa, b, kappa_fn)
    res = u - u_target
    J = 0.5 * float(res @ res)
    rhs_adj = res.copy()
    rhs_adj[box.boundary_mask()] = 0.0
    lam = spla.spsolve(A.tocsc(), rhs_adj)
    return J, gradient(box, u, lam, kappa_fn), u, lam
