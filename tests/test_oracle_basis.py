"""Pins of the oracle's 1D rules, Lagrange bases and random streams (CPU only).

The expected values come from closed forms (monomial integrals, the 3-point
Lobatto rule), exact symbolic differentiation, and the published SplitMix64
reference outputs, none of which reuse the oracle's own code.
"""
import numpy as np
import pytest
import sympy

from oracle.basis import gauss_legendre, gauss_lobatto, lagrange_derivatives, lagrange_values
from oracle.rng import splitmix64, uniform_pm1


@pytest.mark.parametrize("n", range(1, 10))
def test_gauss_legendre_exact_to_degree_2n_minus_1(n):
    x, w = gauss_legendre(n)
    for p in range(2 * n):
        assert abs(w @ x ** p - 1.0 / (p + 1)) < 1e-14
    # degree 2n is not integrated exactly
    assert abs(w @ x ** (2 * n) - 1.0 / (2 * n + 1)) > 1e-13


def test_gauss_lobatto_three_points_closed_form():
    x, w = gauss_lobatto(3)
    np.testing.assert_allclose(x, [0.0, 0.5, 1.0], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 6, 2 / 3, 1 / 6], atol=1e-15)


@pytest.mark.parametrize("n", range(2, 10))
def test_gauss_lobatto_exact_to_degree_2n_minus_3(n):
    x, w = gauss_lobatto(n)
    assert x[0] == 0.0 and x[-1] == 1.0
    assert np.all(np.diff(x) > 0)
    np.testing.assert_allclose(x, 1.0 - x[::-1], atol=1e-15)     # symmetric
    for p in range(2 * n - 2):
        assert abs(w @ x ** p - 1.0 / (p + 1)) < 1e-14
    assert abs(w @ x ** (2 * n - 2) - 1.0 / (2 * n - 1)) > 1e-13


@pytest.mark.parametrize("n", [2, 4, 7])
def test_lagrange_against_symbolic(n):
    nodes, _ = gauss_lobatto(n)
    X = sympy.Symbol("X")
    pts = np.array([0.0, 0.13, 0.5, 0.77, 1.0])
    V = lagrange_values(nodes, pts)
    D = lagrange_derivatives(nodes, pts)
    for i in range(n):
        phi = sympy.Integer(1)
        for j in range(n):
            if j != i:
                phi *= (X - sympy.Float(nodes[j], 30)) / sympy.Float(nodes[i] - nodes[j], 30)
        dphi = sympy.diff(phi, X)
        for q, p in enumerate(pts):
            assert abs(float(phi.subs(X, p)) - V[q, i]) < 1e-12
            assert abs(float(dphi.subs(X, p)) - D[q, i]) < 1e-10
    np.testing.assert_allclose(lagrange_values(nodes, nodes), np.eye(n), atol=1e-14)


def test_splitmix64_reference_outputs():
    # first outputs of SplitMix64 seeded with 0 (published reference values)
    assert [int(v) for v in splitmix64(0, 3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                  0x06C45D188009454F]
    u = uniform_pm1(123, 100000)
    assert u.min() >= -1.0 and u.max() < 1.0
    assert abs(u.mean()) < 0.01 and abs(u.var() - 1.0 / 3.0) < 0.01
