"""Geometric multigrid preconditioned CG for the SIPG discretization (Sec. 4.1, used by
the paper for DG-SIP as well as for continuous elements).

* Levels: DG boxes with Nc, Nc/2, ..., each re-discretized with its own matrix (penalty
  sigma = c_pen (k+1)^2 / h of its own mesh size).
* Transfer: the embedding of the coarse DG space in the fine one.  A coarse cell's
  polynomial is evaluated at the Gauss points of each of its 8 children (all within the
  coarse cell: the DG space has no continuity constraints, so the prolongation is block
  diagonal over coarse cells); restriction is its transpose.
* Smoother, eigenvalue estimate, coarse solver and outer CG: the same textbook routines
  as for the continuous discretization (mg.chebyshev, mg.lanczos_max_eig, mg.coarse_steps,
  mg.pcg).  The DG operator has no Dirichlet rows: every DoF is an unknown.
* Jacobi basis: point Jacobi acts on the coefficients of a basis.  jacobi_basis='gauss'
  uses the Lagrange basis in the Gauss points (the basis of the vectors); 'gll' uses the
  Lagrange basis in the Gauss-Lobatto points of each cell, expressed in the Gauss basis as
  C = T D'^{-1} T^T with T = S (x) S (x) S per cell (S[q][j] = GLL basis j at Gauss point
  q: the change of coefficients from the GLL to the Gauss basis) and D' = diag(T^T A T),
  the diagonal of the operator in the GLL basis.

Test infrastructure only: used by the tests, never by the library.
"""
import numpy as np
import scipy.sparse as sp

from . import mg, sipg
from .basis import gauss_lobatto, lagrange_values


def gll_change_of_basis(dg):
    """Block-diagonal T (per cell S (x) S (x) S) mapping GLL-basis coefficients to
    Gauss-basis coefficients of the same polynomials."""
    xl, _ = gauss_lobatto(dg.n)
    S = lagrange_values(xl, dg.nodes)              # (Gauss points, GLL basis)
    T3 = np.kron(S, np.kron(S, S))
    return sp.block_diag([T3] * dg.n_cells).tocsr()


def child_embedding_1d(dg_coarse):
    """E[s][f, c]: coarse 1D basis c (Lagrange in the Gauss points of [0,1]) at the
    f-th Gauss point of child s (the child covers [s/2, (s+1)/2] of the coarse cell)."""
    x = dg_coarse.nodes
    return [lagrange_values(x, (s + x) / 2.0) for s in (0, 1)]


def prolongation(coarse, fine):
    """(fine.n_dofs, coarse.n_dofs) embedding, cell-major layouts on both levels."""
    E = child_embedding_1d(coarse)
    n3 = coarse.n ** 3
    Nc, Nf = coarse.Nc, fine.Nc
    blocks = {}
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                blocks[(cx, cy, cz)] = np.kron(E[cz], np.kron(E[cy], E[cx]))
    rows, cols, vals = [], [], []
    R = np.repeat(np.arange(n3), n3)
    C = np.tile(np.arange(n3), n3)
    for c in range(coarse.n_cells):
        x, y, z = c % Nc, (c // Nc) % Nc, c // (Nc * Nc)
        for (a, b, d), B in blocks.items():
            f = (2 * x + a) + Nf * ((2 * y + b) + Nf * (2 * z + d))
            rows.append(f * n3 + R)
            cols.append(c * n3 + C)
            vals.append(B.ravel())
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(fine.n_dofs, coarse.n_dofs)).tocsr()


class DGMultigrid:
    """Level hierarchy and V(1,1) cycle of the SIPG operator."""

    def __init__(self, fine_cells, degree, c_pen=1.0, bc="dirichlet", lo=0.0, length=1.0,
                 min_cells=2, cheb_degree=5, cheb_lo=0.06, cheb_hi=1.2, eig_iters=15,
                 coarse_eps=1e-3, jacobi_basis="gauss"):
        self.cheb_updates = cheb_degree + 1
        sizes = []
        Nc = fine_cells
        while Nc >= min_cells:
            sizes.append(Nc)
            if Nc % 2 or Nc // 2 < min_cells:
                break
            Nc //= 2
        sizes = sizes[::-1]                              # coarsest first
        self.levels = []
        for l, Nc in enumerate(sizes):
            dg = sipg.DGBox(Nc, degree, c_pen=c_pen, lo=lo, length=length)
            A = sipg.assemble(dg, bc)
            if jacobi_basis == "gll":
                T = gll_change_of_basis(dg)
                dpinv = 1.0 / (T.T @ A @ T).diagonal()
                Dinv = (lambda T, dpinv: lambda r: T @ (dpinv * (T.T @ r)))(T, dpinv)
            elif jacobi_basis == "gauss":
                Dinv = 1.0 / A.diagonal()
            else:
                raise ValueError(jacobi_basis)
            lev = {"box": dg, "A": A, "Dinv": Dinv}
            if l == 0:
                # C (the Jacobi step as a matrix) is symmetric positive definite: the
                # spectrum of C A is that of L^T A L with C = L L^T
                if jacobi_basis == "gll":
                    C = (T @ sp.diags(dpinv) @ T.T).toarray()
                else:
                    C = np.diag(Dinv)
                Lc = np.linalg.cholesky(C)
                ev = np.linalg.eigvalsh(Lc.T @ A.toarray() @ Lc)
                lev["lmin"], lev["lmax"] = float(ev.min()), float(ev.max())
                lev["steps"] = mg.coarse_steps(lev["lmin"], lev["lmax"], coarse_eps)
            else:
                lam = mg.lanczos_max_eig(A, Dinv, key=Nc, iters=eig_iters)
                lev["lambda"] = lam
                lev["lo"], lev["hi"] = cheb_lo * lam, cheb_hi * lam
                lev["P"] = prolongation(self.levels[l - 1]["box"], dg)
            self.levels.append(lev)
        self.fine_products = 0

    vcycle = mg.Multigrid.vcycle

    def jacobi(self, l, r):
        """The Jacobi step of level l applied to r."""
        return mg.precondition(self.levels[l]["Dinv"], r)


def solve(fine_cells, degree, b, c_pen=1.0, tol=1e-10, maxit=200, **mg_kwargs):
    """GMG-PCG solve of the SIPG system with right-hand side b."""
    m = DGMultigrid(fine_cells, degree, c_pen=c_pen, **mg_kwargs)
    fine = m.levels[-1]
    x, its, res, products = mg.pcg(fine["A"], b, m.vcycle, tol=tol, maxit=maxit)
    return {"x": x, "iterations": its, "residual": res, "mg": m,
            "fine_products": products + m.fine_products}
