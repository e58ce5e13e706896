"""One-dimensional quadrature rules and Lagrange bases on the reference interval [0, 1].

* Section 2.1: the continuous space uses tensor-product Lagrange polynomials in the
  k+1 Gauss-Lobatto-Legendre (GLL) nodes.
* Section 3, eq. (mf_eval): integrals are evaluated with k+1 Gauss-Legendre points
  per direction.
* The DG basis of the SIPG workload is the Lagrange basis in the Gauss-Legendre
  points themselves (a tensor-product basis, which the paper allows in Sec. 2.1).

Everything is written out directly: Lagrange polynomials as explicit products.
"""
import numpy as np
from numpy.polynomial import legendre as _leg


def gauss_legendre(n):
    """n-point Gauss-Legendre rule on [0, 1] (exact for degree 2n-1)."""
    x, w = _leg.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_lobatto(n):
    """n-point Gauss-Lobatto-Legendre nodes and weights on [0, 1], n >= 2.

    Nodes: the end points and the roots of P'_{n-1}; weights 2/(k(k+1) P_k(x)^2)
    on [-1, 1] with k = n-1 (exact for degree 2n-3).
    """
    if n < 2:
        raise ValueError("a Gauss-Lobatto rule needs at least two points")
    k = n - 1
    inner = np.sort(np.real(_leg.Legendre.basis(k).deriv().roots())) if n > 2 else np.zeros(0)
    # one Newton polish step per root on P'_k (roots of the companion matrix are ~1e-15 off)
    dP = _leg.Legendre.basis(k).deriv()
    ddP = dP.deriv()
    for _ in range(3):
        inner = inner - dP(inner) / ddP(inner)
    x = np.concatenate([[-1.0], inner, [1.0]])
    w = 2.0 / (k * (k + 1) * _leg.Legendre.basis(k)(x) ** 2)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_values(nodes, x):
    """V[q, i] = phi_i(x_q) for the Lagrange polynomials phi_i in `nodes`."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    V = np.ones((len(x), n))
    for i in range(n):
        for j in range(n):
            if j != i:
                V[:, i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    return V


def lagrange_derivatives(nodes, x):
    """D[q, i] = phi_i'(x_q), by the product rule over the factors of phi_i."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    D = np.zeros((len(x), n))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[m]))
            for j in range(n):
                if j != i and j != m:
                    term *= (x - nodes[j]) / (nodes[i] - nodes[j])
            D[:, i] += term
    return D
