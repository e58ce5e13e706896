"""Textbook geometric multigrid preconditioned conjugate gradients (Section 4.1).

* Levels: the box with Nc, Nc/2, ..., down to the coarsest cell count, each level
  re-discretized with its own matrix; the coarse diffusion coefficient of a cell is
  the mean of its 8 children.
* Transfer: prolongation is the embedding of the coarse Q_k space in the fine one
  (coarse basis functions evaluated at the fine nodes, in reference coordinates),
  with Dirichlet rows and columns removed; restriction is its transpose.
* Smoother: Chebyshev iteration on D^{-1} A (D = diag A) over the interval
  [0.06, 1.2] * lambda_max, where lambda_max is the largest Ritz value of 15
  Jacobi-preconditioned CG iterations.  The recurrence runs six updates of x; from
  a zero initial guess (pre-smoothing) that costs five matrix-vector products,
  from a nonzero one (post-smoothing) six, including the initial residual.  With
  the outer product and the residual before restriction this gives the 13 fine
  level products per iteration the paper counts (Sec. 4.3).
* Coarse solver: Chebyshev iteration over the exact extreme eigenvalues of
  D^{-1} A of the interior block, with the number of steps from the a-priori bound
  2 ((sqrt(c)-1)/(sqrt(c)+1))^m <= 1e-3 (c = lambda_max / lambda_min).
* Outer solver: CG with one V(1,1) cycle as preconditioner, x_0 = 0, stopped at
  ||r||_2 <= tol ||b||_2.
"""
import math

import numpy as np
import scipy.sparse as sp

from . import cg
from .mesh import Box
from .rng import uniform_pm1


def coarsen_kappa(kappa, Nc):
    """Mean of the 8 children of every coarse cell (lexicographic, x fastest)."""
    K = np.asarray(kappa).reshape(Nc, Nc, Nc)        # [z, y, x]
    Kc = 0.125 * (K[0::2, 0::2, 0::2] + K[0::2, 0::2, 1::2] + K[0::2, 1::2, 0::2] +
                  K[0::2, 1::2, 1::2] + K[1::2, 0::2, 0::2] + K[1::2, 0::2, 1::2] +
                  K[1::2, 1::2, 0::2] + K[1::2, 1::2, 1::2])
    return Kc.ravel()


def prolongation_1d(coarse, fine):
    """P1[f, I]: coarse global 1D basis function I at fine grid line f."""
    k = coarse.k
    P = np.zeros((fine.N1, coarse.N1))
    for f in range(fine.N1):
        cf = min(f // k, fine.Nc - 1)                 # fine cell
        c = cf // 2                                   # its coarse parent
        xi = ((cf - 2 * c) + fine.gll[f - cf * k]) / 2.0
        P[f, c * k:c * k + k + 1] = cg.lagrange_values(coarse.gll, [xi])[0]
    return P


def prolongation(coarse, fine, bc="dirichlet"):
    """3D embedding with Dirichlet rows (fine) and columns (coarse) removed."""
    P1 = sp.csr_matrix(prolongation_1d(coarse, fine))
    P = sp.kron(P1, sp.kron(P1, P1)).tocsr()
    keep_f = sp.diags((~fine.boundary_mask(bc)).astype(np.float64))
    keep_c = sp.diags((~coarse.boundary_mask(bc)).astype(np.float64))
    return (keep_f @ P @ keep_c).tocsr()


def precondition(Dinv, r):
    """Jacobi step: Dinv * r for a vector of inverse diagonal entries, Dinv(r) when Dinv is
    a callable (a smoother preconditioner other than the point Jacobi of the basis)."""
    return Dinv(r) if callable(Dinv) else Dinv * r


def lanczos_max_eig(A, Dinv, key, iters=15, bmask=None):
    """Largest Ritz value of `iters` Jacobi-preconditioned CG steps on A x = b,
    b = SplitMix64 stream `key` in [-1, 1) with Dirichlet entries zeroed."""
    T, _ = cg_lanczos(A, Dinv, key, iters, bmask)
    return float(np.linalg.eigvalsh(T).max())


def cg_lanczos(A, Dinv, key, iters, bmask=None):
    n = A.shape[0]
    b = uniform_pm1(key, n)
    if bmask is not None:
        b[bmask] = 0.0
    x = np.zeros(n)
    r = b.copy()
    z = precondition(Dinv, r)
    p = z.copy()
    rz = r @ z
    alphas, betas = [], []
    for _ in range(iters):
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = precondition(Dinv, r)
        rz_new = r @ z
        beta = rz_new / rz
        alphas.append(alpha)
        betas.append(beta)
        rz = rz_new
        p = z + beta * p
        if rz_new <= 1e-30 * (b @ precondition(Dinv, b)):
            break
    m = len(alphas)
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = math.sqrt(betas[j]) / alphas[j]
    return T, b


def chebyshev(A, Dinv, b, x0, lo, hi, updates):
    """Chebyshev iteration on D^{-1} A with eigenvalue interval [lo, hi] and
    `updates` updates of x.  x0 = None means a zero initial guess (no product for
    the initial residual).  Returns (x, number of products with A)."""
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    products = 0
    if x0 is None:
        x = np.zeros_like(b)
        r = b.copy()
    else:
        x = x0.copy()
        r = b - A @ x
        products += 1
    d = precondition(Dinv, r) / theta
    if updates > 1:
        sigma1 = theta / delta
        rho = 1.0 / sigma1
    for _ in range(updates - 1):
        x += d
        r = b - A @ x
        products += 1
        rho_new = 1.0 / (2.0 * sigma1 - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * precondition(Dinv, r)
        rho = rho_new
    x += d
    return x, products


def coarse_steps(lmin, lmax, eps=1e-3):
    """Smallest m with 2 ((sqrt(c)-1)/(sqrt(c)+1))^m <= eps, c = lmax/lmin."""
    c = lmax / lmin
    rate = (math.sqrt(c) - 1.0) / (math.sqrt(c) + 1.0)
    if rate <= 0.0:
        return 1
    return max(1, math.ceil(math.log(2.0 / eps) / math.log(1.0 / rate)))


class Multigrid:
    """Level hierarchy, smoother data and V(1,1) cycle for the CG operator with Dirichlet
    conditions on the faces of `bc` ('dirichlet': all, 'mixed': the upper faces).  A
    position-dependent coefficient kappa_fn is evaluated at the quadrature points of every
    level (each level is re-discretized), on top of the cellwise kappa."""

    def __init__(self, fine_cells, degree, kappa=None, curve_amp=0.0, min_cells=2,
                 cheb_degree=5, cheb_lo=0.06, cheb_hi=1.2, eig_iters=15, coarse_eps=1e-3,
                 bc="dirichlet", lo=0.0, length=1.0, kappa_fn=None):
        self.cheb_updates = cheb_degree + 1
        sizes = []
        Nc = fine_cells
        while Nc >= min_cells:
            sizes.append(Nc)
            if Nc % 2 or Nc // 2 < min_cells:
                break
            Nc //= 2
        sizes = sizes[::-1]                          # coarsest first
        kap = np.ones(fine_cells ** 3) if kappa is None else np.asarray(kappa, np.float64)
        kappas = [kap]
        for Nc in sizes[::-1][1:]:
            kappas.append(coarsen_kappa(kappas[-1], 2 * Nc))
        kappas = kappas[::-1]
        self.levels = []
        for l, Nc in enumerate(sizes):
            box = Box(Nc, degree, curve_amp, lo=lo, length=length)
            A = cg.assemble(box, kappas[l], bc=bc, kappa_fn=kappa_fn)
            Dinv = 1.0 / A.diagonal()
            lev = {"box": box, "A": A, "Dinv": Dinv, "kappa": kappas[l]}
            if l == 0:
                interior = ~box.boundary_mask(bc)
                Ai = A[interior][:, interior].toarray()
                di = np.sqrt(Dinv[interior])
                ev = np.linalg.eigvalsh(di[:, None] * Ai * di[None, :])
                lev["lmin"], lev["lmax"] = float(ev.min()), float(ev.max())
                lev["steps"] = coarse_steps(lev["lmin"], lev["lmax"], coarse_eps)
            else:
                lam = lanczos_max_eig(A, Dinv, key=Nc, iters=eig_iters, bmask=box.boundary_mask(bc))
                lev["lambda"] = lam
                lev["lo"], lev["hi"] = cheb_lo * lam, cheb_hi * lam
                lev["P"] = prolongation(self.levels[l - 1]["box"], box, bc)
            self.levels.append(lev)
        self.fine_products = 0

    def vcycle(self, b, l=None):
        l = len(self.levels) - 1 if l is None else l
        lev = self.levels[l]
        if l == 0:
            x, _ = chebyshev(lev["A"], lev["Dinv"], b, None, lev["lmin"], lev["lmax"], lev["steps"])
            return x
        fine = l == len(self.levels) - 1
        x, p1 = chebyshev(lev["A"], lev["Dinv"], b, None, lev["lo"], lev["hi"], self.cheb_updates)
        r = b - lev["A"] @ x
        xc = self.vcycle(lev["P"].T @ r, l - 1)
        x = x + lev["P"] @ xc
        x, p2 = chebyshev(lev["A"], lev["Dinv"], b, x, lev["lo"], lev["hi"], self.cheb_updates)
        if fine:
            self.fine_products += p1 + 1 + p2
        return x


def pcg(A, b, precond, tol=1e-10, maxit=200):
    """Preconditioned CG from x_0 = 0, stopping at ||r|| <= tol ||b||.
    Returns (x, iterations, relative residual, number of products with A)."""
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, 0.0, 0
    z = precond(r)
    p = z.copy()
    rz = r @ z
    products = 0
    for it in range(1, maxit + 1):
        q = A @ p
        products += 1
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        res = np.linalg.norm(r) / nb
        if res <= tol:
            return x, it, res, products
        z = precond(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit, res, products


def solve(fine_cells, degree, b=None, kappa=None, curve_amp=0.0, tol=1e-10, maxit=200, **mg_kwargs):
    """GMG-PCG solve (boundary conditions and domain from mg_kwargs, default Dirichlet on
    the unit cube); b defaults to the sine right-hand side."""
    mg = Multigrid(fine_cells, degree, kappa=kappa, curve_amp=curve_amp, **mg_kwargs)
    fine = mg.levels[-1]
    if b is None:
        b = cg.rhs(fine["box"])
    x, its, res, products = pcg(fine["A"], b, mg.vcycle, tol=tol, maxit=maxit)
    return {"x": x, "iterations": its, "residual": res, "mg": mg,
            "fine_products": products + mg.fine_products}
