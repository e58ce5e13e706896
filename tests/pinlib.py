"""Independent reference constructions used by the oracle pins (test code only)."""
import numpy as np
import sympy


def exact_1d_matrices(nodes):
    """Reference-interval [0,1] mass and stiffness matrices of the Lagrange basis in
    `nodes` by exact rational polynomial integration (sympy); the double-precision
    nodes are taken as exact rationals."""
    n = len(nodes)
    X = sympy.Symbol("X")
    r = [sympy.Rational(float(v)) for v in nodes]
    phis = []
    for i in range(n):
        p = sympy.Integer(1)
        for j in range(n):
            if j != i:
                p *= (X - r[j]) / (r[i] - r[j])
        phis.append(sympy.Poly(sympy.expand(p), X))
    M = np.zeros((n, n))
    K = np.zeros((n, n))
    for i in range(n):
        for j in range(i, n):
            pm = (phis[i] * phis[j]).integrate()
            pk = (phis[i].diff(X) * phis[j].diff(X)).integrate()
            M[i, j] = M[j, i] = float(pm.eval(1) - pm.eval(0))
            K[i, j] = K[j, i] = float(pk.eval(1) - pk.eval(0))
    return M, K


def exact_end_values(nodes):
    """phi_i(0), phi_i(1), phi_i'(0), phi_i'(1) in exact rational arithmetic."""
    n = len(nodes)
    X = sympy.Symbol("X")
    r = [sympy.Rational(float(v)) for v in nodes]
    out = np.zeros((4, n))
    for i in range(n):
        p = sympy.Integer(1)
        for j in range(n):
            if j != i:
                p *= (X - r[j]) / (r[i] - r[j])
        dp = sympy.diff(p, X)
        out[:, i] = [float(p.subs(X, 0)), float(p.subs(X, 1)), float(dp.subs(X, 0)), float(dp.subs(X, 1))]
    return out


def along(A, V, axis):
    """Apply the matrix A along `axis` of the array V."""
    return np.moveaxis(np.tensordot(A, V, axes=([1], [axis])), 0, axis)


def kron_sum_apply(Mx, Kx, U):
    """(K(x)M(x)M + M(x)K(x)M + M(x)M(x)K) U for U[z, y, x]."""
    return (along(Kx, along(Mx, along(Mx, U, 0), 1), 2) +
            along(Mx, along(Kx, along(Mx, U, 0), 1), 2) +
            along(Mx, along(Mx, along(Kx, U, 0), 1), 2))
