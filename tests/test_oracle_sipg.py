"""Pins of the SIPG oracle (CPU only).

The SIPG operator on a Cartesian mesh with a constant penalty is an exact
Kronecker sum A1(x)M1(x)M1 + M1(x)A1(x)M1 + M1(x)M1(x)A1 of a 1D SIPG operator and
the 1D DG mass matrix, up to the permutation between the cell-major DG layout and
tensor order.  The 1D operator is built here face by face from the symmetric
interior penalty form (each interior face once), with basis data from exact
rational arithmetic, independently of the oracle's element-centric transcription.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import cg, sipg
from seeded_inputs import uniform_vector
from tests.pinlib import exact_1d_matrices, exact_end_values, along


def sipg_1d(dg):
    """Global 1D SIPG matrix (Dirichlet) and DG mass, DoF index cell * n + i."""
    n, Nc, h, sig = dg.n, dg.Nc, dg.h, dg.sigma
    M, K = exact_1d_matrices(dg.nodes)
    v0, v1, d0, d1 = exact_end_values(dg.nodes)
    N = Nc * n
    A = np.zeros((N, N))
    Mg = np.zeros((N, N))
    for c in range(Nc):
        s = slice(c * n, (c + 1) * n)
        A[s, s] += K / h
        Mg[s, s] += h * M
    for f in range(1, Nc):                    # interior face between cells f-1 and f, normal +x
        jump = np.zeros(N)
        avg = np.zeros(N)
        jump[(f - 1) * n:f * n] = v1
        jump[f * n:(f + 1) * n] = -v0
        avg[(f - 1) * n:f * n] = 0.5 * d1 / h
        avg[f * n:(f + 1) * n] = 0.5 * d0 / h
        A += -np.outer(jump, avg) - np.outer(avg, jump) + sig * np.outer(jump, jump)
    for cell, val, dn in ((0, v0, -d0 / h), (Nc - 1, v1, d1 / h)):   # Dirichlet ends
        a = np.zeros(N)
        g = np.zeros(N)
        a[cell * n:(cell + 1) * n] = val
        g[cell * n:(cell + 1) * n] = dn
        A += -np.outer(a, g) - np.outer(g, a) + 2.0 * sig * np.outer(a, a)
    return A, Mg


def tensor_to_cell_major(dg):
    """perm[t] = cell-major index of tensor index t = X + N (Y + N Z), X = cx n + i."""
    n, Nc = dg.n, dg.Nc
    N = n * Nc
    Z, Y, X = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    cell = X // n + Nc * (Y // n + Nc * (Z // n))
    loc = X % n + n * (Y % n + n * (Z % n))
    return (cell * n ** 3 + loc).ravel()


def kron_apply(dg, u):
    A1, M1 = sipg_1d(dg)
    perm = tensor_to_cell_major(dg)
    N = dg.n * dg.Nc
    U = u[perm].reshape(N, N, N)
    Y = (along(A1, along(M1, along(M1, U, 0), 1), 2) + along(M1, along(A1, along(M1, U, 0), 1), 2)
         + along(M1, along(M1, along(A1, U, 0), 1), 2))
    y = np.empty_like(u)
    y[perm] = Y.ravel()
    return y


@pytest.mark.parametrize("Nc,k,cpen", [(3, 1, 1.0), (4, 2, 1.0), (3, 3, 3.0), (2, 5, 1.0)])
def test_sipg_matches_kronecker_sum(Nc, k, cpen):
    dg = sipg.DGBox(Nc, k, cpen)
    u = uniform_vector(dg.n_dofs, 3)
    y = kron_apply(dg, u)
    np.testing.assert_allclose(sipg.assemble(dg) @ u, y, rtol=0, atol=1e-12 * np.abs(y).max())


@pytest.mark.slow
def test_sipg_full_size_q3_sampled_rows_match_kronecker():
    dg = sipg.DGBox(32, 3)
    u = uniform_vector(dg.n_dofs, 3)
    y = kron_apply(dg, u)
    rows = np.random.default_rng(11).choice(dg.n_dofs, 200, replace=False)
    rows[:2] = [0, dg.n_dofs - 1]
    np.testing.assert_allclose(sipg.apply_rows(dg, u, rows), y[rows], rtol=0, atol=1e-11 * np.abs(y).max())


@pytest.mark.parametrize("k", [1, 2, 3])
def test_sipg_structure(k):
    dg = sipg.DGBox(3, k)
    An = sipg.assemble(dg, "neumann")
    assert np.abs(An @ np.ones(dg.n_dofs)).max() < 1e-12 * abs(An).max()
    A = sipg.assemble(dg).toarray()
    assert np.abs(A - A.T).max() < 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0.0


@pytest.mark.parametrize("k", [1, 2, 3])
def test_sipg_l2_rate(k):
    errs = []
    for Nc in ((2, 4) if k == 3 else (4, 8)):
        dg = sipg.DGBox(Nc, k)
        u = spla.spsolve(sipg.assemble(dg).tocsc(), sipg.rhs(dg, cg.sine_forcing))
        errs.append(sipg.l2_error(dg, u, cg.sine_solution))
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - (k + 1)) < 0.25, (errs, rate)
