"""Pins of the oracle's position-dependent coefficient (Sec. 4.3, eq. (diffusivity_shell),
read as kappa(x) = 1 + amp prod_e cos^2(2 pi x_e + 0.1 e), evaluated at the physical image of
every Gauss point) -- CPU only.

* On Cartesian cells the integrand factorizes: with tensor Gauss quadrature the element
  matrix of the product part equals the Kronecker sum of 1D matrices weighted by
  cos^2(2 pi x_e + 0.1 e) along each axis, built here from exact rational Lagrange
  polynomials (sympy) and the Gauss rule.  This pins where and along which axis each
  factor is evaluated.
* The pure-Neumann operator annihilates constants for any coefficient (curved cells).
* Symmetric positive definite with Dirichlet conditions (curved cells, dense eigenvalues).
* With the coefficient in the forcing f = -div(kappa grad u) of u = sin sin sin the
  discretization converges at rate k + 1 in L2 on curved meshes (Sec. 4.3 observes the
  optimal rate).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import sympy

from oracle import cg
from oracle.basis import gauss_legendre, gauss_lobatto
from oracle.mesh import Box


def exact_basis_at(nodes, points):
    """V[q, i], D[q, i]: Lagrange basis i in `nodes` and its derivative at `points`, from
    exact rational polynomials."""
    X = sympy.Symbol("X")
    r = [sympy.Rational(float(v)) for v in nodes]
    n = len(nodes)
    V = np.zeros((len(points), n))
    D = np.zeros((len(points), n))
    for i in range(n):
        p = sympy.Integer(1)
        for j in range(n):
            if j != i:
                p *= (X - r[j]) / (r[i] - r[j])
        dp = sympy.diff(p, X)
        for q, x in enumerate(points):
            V[q, i] = float(p.subs(X, sympy.Rational(float(x))))
            D[q, i] = float(dp.subs(X, sympy.Rational(float(x))))
    return V, D


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_cartesian_element_matrix_is_a_weighted_kronecker_sum(k):
    amp, Nc = 7.0, 3
    box = Box(Nc, k)
    n = k + 1
    xg, wg = gauss_legendre(n)
    xl, _ = gauss_lobatto(n)
    V, D = exact_basis_at(xl, xg)
    h = box.h
    cells = [0, 5, 13, 26]
    Ae = cg.element_matrices(box, cells=np.array(cells), kappa_fn=cg.cosine_coefficient(amp))
    for t, c in enumerate(cells):
        corner = [c % Nc, (c // Nc) % Nc, c // (Nc * Nc)]
        M, K, Mw, Kw = [], [], [], []
        for e in range(3):
            x = (corner[e] + xg) * h
            wt = np.cos(2 * np.pi * x + 0.1 * (e + 1)) ** 2
            M.append(h * (V.T * wg) @ V)
            K.append((D.T * wg) @ D / h)
            Mw.append(h * (V.T * (wg * wt)) @ V)
            Kw.append((D.T * (wg * wt)) @ D / h)
        # local index i + n j + n^2 l (x fastest): kron(z, kron(y, x))
        plain = (np.kron(M[2], np.kron(M[1], K[0])) + np.kron(M[2], np.kron(K[1], M[0])) +
                 np.kron(K[2], np.kron(M[1], M[0])))
        prod = (np.kron(Mw[2], np.kron(Mw[1], Kw[0])) + np.kron(Mw[2], np.kron(Kw[1], Mw[0])) +
                np.kron(Kw[2], np.kron(Mw[1], Mw[0])))
        ref = plain + amp * prod
        assert np.abs(Ae[t] - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("k", [1, 3])
def test_neumann_operator_annihilates_constants(k):
    box = Box(3, k, 0.1)
    A = cg.assemble(box, bc="neumann", kappa_fn=cg.cosine_coefficient(1e6))
    one = np.ones(box.n_dofs)
    assert np.abs(A @ one).max() <= 1e-11 * abs(A).max()


def test_symmetric_positive_definite_on_curved_mesh():
    box = Box(2, 2, 0.1)
    A = cg.assemble(box, kappa_fn=cg.cosine_coefficient(1e6)).toarray()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    inner = ~box.boundary_mask()
    ev = np.linalg.eigvalsh(A[np.ix_(inner, inner)])
    assert ev.min() > 0


def manufactured_forcing(amp):
    """f = -div(kappa grad u) = 3 pi^2 kappa u - grad kappa . grad u for u = sin sin sin."""
    def f(x):
        th = [2 * np.pi * x[..., e] + 0.1 * (e + 1) for e in range(3)]
        c2 = [np.cos(t) ** 2 for t in th]
        kap = 1.0 + amp * c2[0] * c2[1] * c2[2]
        s = [np.sin(np.pi * x[..., e]) for e in range(3)]
        c = [np.cos(np.pi * x[..., e]) for e in range(3)]
        u = s[0] * s[1] * s[2]
        gu = [np.pi * c[0] * s[1] * s[2], np.pi * s[0] * c[1] * s[2], np.pi * s[0] * s[1] * c[2]]
        out = 3.0 * np.pi ** 2 * kap * u
        for e in range(3):
            others = [c2[j] for j in range(3) if j != e]
            out -= amp * (-2.0 * np.pi * np.sin(2.0 * th[e])) * others[0] * others[1] * gu[e]
        return out
    return f


@pytest.mark.parametrize("k", [2, 3])
def test_l2_rate_with_variable_coefficient(k):
    amp = 1.0
    errs = []
    for nc in (4, 8):
        box = Box(nc, k, 0.1)
        A = cg.assemble(box, kappa_fn=cg.cosine_coefficient(amp))
        u = spla.spsolve(A.tocsc(), cg.rhs(box, manufactured_forcing(amp)))
        errs.append(cg.l2_error(box, u))
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - (k + 1)) <= 0.15, rate
