"""The three-dimensional example with smooth solution (Sec. 4.3, eq. pois_analytic).

The analytic solution is a sum of three Gaussians of width alpha = 1/5,

    u(x) = (1 / (alpha sqrt(2 pi)))^3 sum_j exp(-|x - x_j|^2 / alpha^2),

centred at (-0.5, 0.5, 0.25), (-0.6, -0.5, -0.125) and (0.5, -0.5, 0.5).  The domain is
the cube (-1, 1)^3 with Neumann conditions on the faces x_e = -1 and Dirichlet conditions
on the faces x_e = +1, kappa = 1.  The forcing f = -Laplace(u), the Dirichlet data
g_D = u and the Neumann data g_N = grad(u) . n are chosen so that u solves the problem.

Discrete problem with the Dirichlet convention of the operator (identity rows on
Dirichlet DoFs, their columns eliminated): with x0 the nodal interpolant of g_D on the
Dirichlet DoFs (zero elsewhere) and A0 the operator without boundary conditions,

    b_i = int f phi_i + int_{Gamma_N} g_N phi_i - (A0 x0)_i   (i not on a Dirichlet face),
    b_i = x0_i                                                  (i on a Dirichlet face),

so that the solution of A x = b carries the Dirichlet data on the Dirichlet DoFs.

Test infrastructure only: used by the tests, never by the library.
"""
import numpy as np
import scipy.sparse.linalg as spla

from . import cg, sipg
from .basis import gauss_legendre, lagrange_values
from .mesh import Box

ALPHA = 0.2
CENTERS = np.array([[-0.5, 0.5, 0.25], [-0.6, -0.5, -0.125], [0.5, -0.5, 0.5]])
SCALE = (1.0 / (ALPHA * np.sqrt(2.0 * np.pi))) ** 3


def box(cells_per_dim, degree):
    """The Cartesian mesh of (-1, 1)^3 used by the example."""
    return Box(cells_per_dim, degree, lo=-1.0, length=2.0)


def _gaussians(x):
    d = x[..., None, :] - CENTERS          # (..., 3 centres, 3)
    r2 = np.sum(d * d, axis=-1)            # (..., 3)
    return d, r2, np.exp(-r2 / ALPHA ** 2)


def solution(x):
    _, _, e = _gaussians(np.asarray(x, dtype=np.float64))
    return SCALE * np.sum(e, axis=-1)


def gradient(x):
    """grad u, shape (..., 3): d/dx exp(-r^2/a^2) = -2 (x - x_j) / a^2 exp(...)."""
    d, _, e = _gaussians(np.asarray(x, dtype=np.float64))
    return SCALE * np.sum((-2.0 / ALPHA ** 2) * d * e[..., None], axis=-2)


def forcing(x):
    """f = -Laplace(u); in 3D Laplace exp(-r^2/a^2) = (4 r^2 / a^4 - 6 / a^2) exp(...)."""
    _, r2, e = _gaussians(np.asarray(x, dtype=np.float64))
    return -SCALE * np.sum((4.0 * r2 / ALPHA ** 4 - 6.0 / ALPHA ** 2) * e, axis=-1)


def neumann_load(box, bc="mixed", n_quad=None):
    """int_{Gamma_N} g_N phi_i over the faces without Dirichlet conditions (Cartesian
    cells; k+1 Gauss points per face direction unless n_quad is given)."""
    from .mesh import bc_mask
    if box.a != 0.0:
        raise ValueError("face integrals are implemented for Cartesian cells")
    m = bc_mask(bc)
    nq = box.n if n_quad is None else int(n_quad)
    xq, wq = gauss_legendre(nq)
    V = lagrange_values(box.gll, xq)                    # (nq, n)
    b = np.zeros(box.n_dofs)
    Nc, h = box.Nc, box.h
    for side in (0, 1):
        if m & (1 << side):
            continue                                    # Dirichlet faces carry no load
        Vs = lagrange_values(box.gll, np.array([float(side)]))   # (1, n): the end point
        for e in range(3):
            # tensor factors per direction (x fastest): the face direction takes the end
            # point, the two others the Gauss points
            facs = [Vs if d == e else V for d in range(3)]
            val = np.kron(facs[2], np.kron(facs[1], facs[0]))     # (points, n^3)
            w1 = [np.ones(1) if d == e else wq for d in range(3)]
            w2 = np.kron(w1[2], np.kron(w1[1], w1[0])) * h * h
            c_face = 0 if side == 0 else Nc - 1
            cells = np.arange(box.n_cells)
            cc = box.cell_coords(cells)
            cells = cells[cc[e] == c_face]
            X = box.cell_node_coords(cells)                           # (cells, n^3, 3)
            xphys = np.einsum("qi,cia->cqa", val, X)
            normal = np.zeros(3)
            normal[e] = -1.0 if side == 0 else 1.0
            gN = gradient(xphys) @ normal                             # (cells, points)
            be = np.einsum("cq,qi->ci", w2[None, :] * gN, val)
            np.add.at(b, box.cell_dofs(cells).ravel(), be.ravel())
    return b


def dirichlet_values(box, bc="mixed"):
    """x0: the interpolant of u on the Dirichlet DoFs, zero elsewhere."""
    x0 = np.zeros(box.n_dofs)
    d = box.boundary_mask(bc)
    x0[d] = solution(box.dof_points()[d])
    return x0


def rhs(box, bc="mixed", A0=None):
    """The right-hand side b of the module docstring.  A0: the assembled operator without
    boundary conditions (assembled here when not given)."""
    if A0 is None:
        A0 = cg.assemble(box, bc="neumann")
    x0 = dirichlet_values(box, bc)
    b = cg.rhs(box, forcing, zero_boundary=False) + neumann_load(box, bc) - A0 @ x0
    d = box.boundary_mask(bc)
    b[d] = x0[d]
    return b


def solve_direct(Nc, k, bc="mixed"):
    """Sparse direct solution of the discrete problem; returns (box, u_h)."""
    bx = box(Nc, k)
    A0 = cg.assemble(bx, bc="neumann")
    b = rhs(bx, bc, A0=A0)
    A = cg.assemble(bx, bc=bc)
    return bx, spla.spsolve(A.tocsc(), b)


def relative_l2_error(box, u):
    """|| u_h - u ||_{L2} / || u ||_{L2} with k+3 Gauss points per direction."""
    return cg.l2_error(box, u, exact=solution) / cg.l2_norm(box, solution)


# ---- DG-SIP discretization of the same example ----------------------------------------
# The paper's penalty sigma = (k+1)^2 d / h, i.e. c_pen = 3 in sipg.DGBox.

def dg_box(cells_per_dim, degree, c_pen=3.0):
    return sipg.DGBox(cells_per_dim, degree, c_pen=c_pen, lo=-1.0, length=2.0)


def dg_rhs(dg, bc="mixed"):
    """(f, v) plus the boundary data terms of eq. (bc_dgsip) (sipg.boundary_data_load)."""
    return sipg.rhs(dg, forcing) + sipg.boundary_data_load(
        dg, solution, lambda x, nrm: gradient(x) @ nrm, bc)


def dg_solve_direct(Nc, k, bc="mixed", c_pen=3.0):
    dg = dg_box(Nc, k, c_pen)
    A = sipg.assemble(dg, bc)
    return dg, spla.spsolve(A.tocsc(), dg_rhs(dg, bc))
