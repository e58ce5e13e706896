"""Pins of two oracle helpers that the solver tests only exercise indirectly (CPU only).

* ``mg.coarsen_kappa`` (Sec. 4.1: the coarse levels are re-discretized; the coarse
  coefficient of a cell is the mean of its 8 children):
  - a field that is constant on every 2x2x2 block maps to that constant;
  - a field linear in the cell indices with a different slope per axis maps to its value
    at the coarse cell centre (an axis swap or a wrong child stride fails);
  - for a blockwise constant coefficient the Galerkin product P^T A_fine P equals the
    re-discretized coarse operator (nested spaces, exact Gauss quadrature on Cartesian
    cells), which pins where each coarse value lands in the coarse mesh;
  - PCG preconditioned by a three-level V-cycle with a cellwise coefficient reaches the
    sparse direct solution with 13 fine-level products per iteration.
* ``dgmg.gll_change_of_basis`` (Sec. 2.1: any tensor-product basis; the DG smoother's
  Jacobi step acts on the Gauss-Lobatto Lagrange coefficients of each cell):
  - T applied to the values of a random Q_k polynomial at the GLL points of every cell
    gives its values at the Gauss points (k = 1..6), polynomials evaluated directly;
  - each cell block equals S (x) S (x) S with S built here from exact rational Lagrange
    polynomials (sympy) at the GLL nodes, evaluated at the Gauss points.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse.linalg as spla
import sympy

from oracle import cg, dgmg, mg, sipg
from oracle.basis import gauss_legendre, gauss_lobatto
from oracle.mesh import Box
from seeded_inputs import gaussian_field


def test_coarsen_kappa_block_constant_field():
    Nc = 8
    coarse = np.exp(gaussian_field((Nc // 2) ** 3, 51, 0.7)).reshape(Nc // 2, Nc // 2, Nc // 2)
    fine = np.empty((Nc, Nc, Nc))
    for z, y, x in itertools.product(range(Nc), repeat=3):
        fine[z, y, x] = coarse[z // 2, y // 2, x // 2]
    out = mg.coarsen_kappa(fine.ravel(), Nc)
    assert np.allclose(out, coarse.ravel(), rtol=4e-16, atol=0)


def test_coarsen_kappa_axis_slopes():
    """kappa(cx, cy, cz) = 1 + 2 cx + 30 cy + 500 cz on the fine cells: the mean of the 8
    children of coarse cell (X, Y, Z) is the value at the centre 2X + 1/2, 2Y + 1/2, 2Z + 1/2."""
    Nc = 6
    c = np.arange(Nc ** 3)
    cx, cy, cz = c % Nc, (c // Nc) % Nc, c // (Nc * Nc)
    out = mg.coarsen_kappa(1.0 + 2.0 * cx + 30.0 * cy + 500.0 * cz, Nc)
    C = np.arange((Nc // 2) ** 3)
    X, Y, Z = C % (Nc // 2), (C // (Nc // 2)) % (Nc // 2), C // (Nc // 2) ** 2
    expect = 1.0 + 2.0 * (2 * X + 0.5) + 30.0 * (2 * Y + 0.5) + 500.0 * (2 * Z + 0.5)
    assert np.allclose(out, expect, rtol=0, atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_galerkin_coarse_operator_with_blockwise_kappa(k):
    Nf = 4
    kc = np.exp(gaussian_field((Nf // 2) ** 3, 52 + k, 0.8))
    kf = np.empty(Nf ** 3)
    for z, y, x in itertools.product(range(Nf), repeat=3):
        kf[x + Nf * (y + Nf * z)] = kc[x // 2 + (Nf // 2) * (y // 2 + (Nf // 2) * (z // 2))]
    fine, coarse = Box(Nf, k), Box(Nf // 2, k)
    Af = cg.assemble(fine, kf)
    Ac = cg.assemble(coarse, mg.coarsen_kappa(kf, Nf))
    P = mg.prolongation(coarse, fine)
    G = (P.T @ Af @ P).toarray()
    inner = ~coarse.boundary_mask()
    ref = Ac.toarray()[np.ix_(inner, inner)]
    assert np.abs(G[np.ix_(inner, inner)] - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("bc", ["dirichlet", "mixed"])
def test_multilevel_pcg_with_cellwise_kappa(bc):
    Nc, k = 8, 2
    kap = np.exp(gaussian_field(Nc ** 3, 53, 0.5))
    m_kw = dict(bc=bc, lo=-1.0, length=2.0) if bc == "mixed" else {}
    box = Box(Nc, k, lo=m_kw.get("lo", 0.0), length=m_kw.get("length", 1.0))
    b = np.random.default_rng(54).uniform(-1, 1, box.n_dofs)
    b[box.boundary_mask(bc)] = 0.0
    out = mg.solve(Nc, k, b=b, kappa=kap, tol=1e-12, min_cells=2, **m_kw)
    assert len(out["mg"].levels) == 3
    A = cg.assemble(box, kap, bc=bc)
    xs = spla.spsolve(A.tocsc(), b)
    assert np.abs(out["x"] - xs).max() <= 1e-10 * np.abs(xs).max()
    assert out["fine_products"] == 13 * out["iterations"]
    # the coarse levels carry the children means (levels are listed coarsest first)
    levels = out["mg"].levels
    assert np.array_equal(levels[1]["kappa"], mg.coarsen_kappa(kap, Nc))
    assert np.array_equal(levels[0]["kappa"], mg.coarsen_kappa(levels[1]["kappa"], Nc // 2))


def random_qk_poly(k, seed):
    """A random polynomial of degree <= k in each variable, evaluated from its monomial
    coefficients (no Lagrange basis involved)."""
    coef = np.random.default_rng(seed).uniform(-1, 1, (k + 1, k + 1, k + 1))

    def p(x):
        out = np.zeros(x.shape[:-1])
        for a, b, c in itertools.product(range(k + 1), repeat=3):
            out += coef[a, b, c] * x[..., 0] ** a * x[..., 1] ** b * x[..., 2] ** c
        return out
    return p


def cell_tensor_points(dg, pts1d):
    """(n_cells, n^3, 3) physical points: the 1D reference points of every direction mapped
    to each cell, local index i + n j + n^2 l (x fastest)."""
    n = len(pts1d)
    out = np.empty((dg.n_cells, n ** 3, 3))
    for c in range(dg.n_cells):
        cx, cy, cz = c % dg.Nc, (c // dg.Nc) % dg.Nc, c // (dg.Nc * dg.Nc)
        for l, j, i in itertools.product(range(n), repeat=3):
            out[c, i + n * j + n * n * l] = [dg.lo + (cx + pts1d[i]) * dg.h, dg.lo + (cy + pts1d[j]) * dg.h,
                                             dg.lo + (cz + pts1d[l]) * dg.h]
    return out


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_change_of_basis_maps_gll_values_to_gauss_values(k):
    dg = sipg.DGBox(2, k, lo=-1.0, length=2.0)
    T = dgmg.gll_change_of_basis(dg)
    p = random_qk_poly(k, 60 + k)
    xl, _ = gauss_lobatto(k + 1)
    xg, _ = gauss_legendre(k + 1)
    u_gll = p(cell_tensor_points(dg, xl)).ravel()
    u_gauss = p(cell_tensor_points(dg, xg)).ravel()
    assert np.abs(T @ u_gll - u_gauss).max() <= 1e-12 * np.abs(u_gauss).max()
    # the Gauss-point basis is the basis of the vectors: its own points also match
    assert np.allclose(sipg.cell_points(dg).reshape(-1, 3), cell_tensor_points(dg, xg).reshape(-1, 3),
                       rtol=0, atol=1e-14)


@pytest.mark.parametrize("k", [1, 2, 4, 6])
def test_change_of_basis_block_is_exact_gll_basis_at_gauss_points(k):
    n = k + 1
    xl, _ = gauss_lobatto(n)
    xg, _ = gauss_legendre(n)
    X = sympy.Symbol("X")
    r = [sympy.Rational(float(v)) for v in xl]
    S = np.zeros((n, n))
    for j in range(n):
        phi = sympy.Integer(1)
        for m in range(n):
            if m != j:
                phi *= (X - r[m]) / (r[j] - r[m])
        for q in range(n):
            S[q, j] = float(phi.subs(X, sympy.Rational(float(xg[q]))))
    dg = sipg.DGBox(1, k)
    T = dgmg.gll_change_of_basis(dg).toarray()
    assert np.abs(T - np.kron(S, np.kron(S, S))).max() <= 1e-13
