"""Pins of the continuous-Galerkin oracle (CPU only).

Each test compares the oracle with something it does not compute itself:
* the closed-form Q1 stencil (h/3) {8, 0, -1/2, -1/4} (centre/face/edge/corner);
* Kronecker sums of 1D mass and stiffness matrices obtained by exact polynomial
  integration (Cartesian cells: tensor quadrature makes the operator separable);
* the divergence theorem on the curved mesh for linear functions, whose
  quadrature integrand is polynomial when enough Gauss points are used;
* symmetry, definiteness and the constant null space of the Neumann operator;
* the k+1 convergence rate of the L2 error (Section 4.3) on Cartesian and curved meshes;
* the DoF counts printed in the paper's matrix-vector product tables.
"""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla
from oracle import cg
from oracle.mesh import Box
from seeded_inputs import uniform_vector
from tests.pinlib import exact_1d_matrices, kron_sum_apply

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def assembled_1d(box, M, K):
    M1 = np.zeros((box.N1, box.N1))
    K1 = np.zeros((box.N1, box.N1))
    for c in range(box.Nc):
        s = slice(c * box.k, c * box.k + box.n)
        M1[s, s] += box.h * M
        K1[s, s] += K / box.h
    return M1, K1


def test_q1_stencil_closed_form():
    box = Box(2, 1)
    A = cg.assemble(box, bc="neumann").toarray()
    row = A[13].reshape(3, 3, 3) * 3.0 / box.h          # centre node of the 3^3 grid
    expect = np.empty((3, 3, 3))
    for z in range(3):
        for y in range(3):
            for x in range(3):
                off = abs(x - 1) + abs(y - 1) + abs(z - 1)
                expect[z, y, x] = {0: 8.0, 1: 0.0, 2: -0.5, 3: -0.25}[off]
    np.testing.assert_allclose(row, expect, atol=1e-13)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6])
def test_cartesian_element_matrix_is_kronecker_sum(k):
    box = Box(3, k)
    M, K = exact_1d_matrices(box.gll)
    expect = box.h * (np.kron(M, np.kron(M, K)) + np.kron(M, np.kron(K, M)) + np.kron(K, np.kron(M, M)))
    kap = np.linspace(0.5, 2.0, box.n_cells)
    Ae = cg.element_matrices(box, kap, cells=[0, 13])
    np.testing.assert_allclose(Ae[0], kap[0] * expect, rtol=0, atol=1e-12 * np.abs(expect).max())
    np.testing.assert_allclose(Ae[1], kap[13] * expect, rtol=0, atol=1e-12 * np.abs(expect).max())


@pytest.mark.parametrize("Nc,k", [(8, 2), (4, 4), (3, 5)])
def test_global_dirichlet_operator_matches_kronecker_sum(Nc, k):
    box = Box(Nc, k)
    M, K = exact_1d_matrices(box.gll)
    M1, K1 = assembled_1d(box, M, K)
    u = uniform_vector(box.n_dofs, 0)
    bm = box.boundary_mask()
    uz = np.where(bm, 0.0, u).reshape(box.N1, box.N1, box.N1)
    y = kron_sum_apply(M1, K1, uz).ravel()
    y[bm] = u[bm]
    A = cg.assemble(box)
    np.testing.assert_allclose(A @ u, y, rtol=0, atol=1e-12 * np.abs(y).max())


def test_sampled_rows_match_csr():
    box = Box(4, 3, 0.1)
    u = uniform_vector(box.n_dofs, 2)
    A = cg.assemble(box)
    rows = np.random.default_rng(0).choice(box.n_dofs, 60, replace=False)
    rows[:3] = [0, box.N1 + 1, box.n_dofs // 2]
    np.testing.assert_allclose(cg.apply_rows(box, u, rows), (A @ u)[rows], atol=1e-13)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_curved_linear_patch_test(k):
    """For u = c.x the FE function equals c.x exactly (isoparametric map), so
    (A u)_i = int grad phi_i . c dx = 0 for every interior i (divergence theorem);
    with 2k+1 Gauss points the quadrature of this polynomial integrand is exact."""
    box = Box(3, k, 0.1)
    A = cg.assemble(box, bc="neumann", n_quad=2 * k + 1)
    c = np.array([0.3, -1.1, 0.7])
    u = box.dof_points() @ c
    r = A @ u
    interior = ~box.boundary_mask()
    assert np.abs(r[interior]).max() < 1e-13 * np.abs(r).max() + 1e-14
    # boundary rows carry int_{dOmega} phi_i c.n, which sums to zero
    assert abs(r.sum()) < 1e-13


@pytest.mark.parametrize("a", [0.0, 0.1])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_structure_symmetric_definite_null_space(a, k):
    box = Box(3, k, a)
    kap = np.exp(np.random.default_rng(1).normal(0, 0.5, box.n_cells))
    An = cg.assemble(box, kap, bc="neumann")
    assert np.abs(An @ np.ones(box.n_dofs)).max() < 1e-13 * abs(An).max()
    A = cg.assemble(box, kap)
    Ad = A.toarray()
    assert np.abs(Ad - Ad.T).max() < 1e-14 * np.abs(Ad).max()
    assert np.linalg.eigvalsh(Ad).min() > 0.0
    np.linalg.cholesky(Ad)


def test_quadrature_order_converges_on_curved_cells():
    box = Box(2, 2, 0.1)
    mats = [cg.element_matrices(box, cells=[5], n_quad=m)[0] for m in (3, 5, 7, 11)]
    d = [np.abs(mats[i] - mats[-1]).max() for i in range(3)]
    assert d[0] > d[1] > d[2]
    # Cartesian: k+1 and k+3 points agree (exact integration)
    cart = Box(2, 3)
    np.testing.assert_allclose(cg.element_matrices(cart, cells=[1], n_quad=4),
                               cg.element_matrices(cart, cells=[1], n_quad=6), atol=1e-13)


def test_rhs_of_constant_forcing_is_lumped_gll_mass():
    """f = 1 on a Cartesian mesh: b_i = int phi_i = h^3 w_a w_b w_c summed over cells,
    because the k+1 point GLL rule integrates the degree-k basis exactly."""
    box = Box(3, 2)
    b = cg.rhs(box, f=lambda x: np.ones(x.shape[:-1]), zero_boundary=False)
    w1 = np.zeros(box.N1)
    for c in range(box.Nc):
        w1[c * box.k:c * box.k + box.n] += box.h * box.gll_w
    expect = np.einsum("z,y,x->zyx", w1, w1, w1).ravel()
    np.testing.assert_allclose(b, expect, atol=1e-15)


@pytest.mark.parametrize("a", [0.0, 0.1])
@pytest.mark.parametrize("k", [1, 2])
def test_l2_convergence_rate_k_plus_1(a, k):
    errs = []
    for Nc in (4, 8):
        box = Box(Nc, k, a)
        u = spla.spsolve(cg.assemble(box).tocsc(), cg.rhs(box))
        errs.append(cg.l2_error(box, u))
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - (k + 1)) < 0.25, (errs, rate)


def test_dof_counts_match_paper_tables():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "paper_matvec_dofs.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 16
    for fam, k, cells, dofs in rows:
        k, cells, dofs = int(k), int(cells), int(dofs)
        m = round(cells ** (1 / 3))
        assert m ** 3 == cells
        if fam == "cg":
            assert Box(m, k).n_dofs == dofs
        else:
            assert cells * (k + 1) ** 3 == dofs
