"""Pins of the multigrid / PCG / adjoint oracle (CPU only).

* PCG with the V-cycle reaches the sparse direct solution.
* The 15-step Lanczos estimate lies below the dense largest eigenvalue of D^{-1}A,
  and 1.2 times it lies above (Section 4.1's interval is safe).
* The smoother's error propagation operator has the eigenvalues of the scaled
  Chebyshev polynomial T_m((theta - mu)/delta) / T_m(theta/delta) at the
  eigenvalues mu of D^{-1}A (closed form of the Chebyshev iteration).
* The coarse solver meets its a-priori bound 1e-3 in the energy norm.
* 13 fine-level products per iteration (65 in 5 iterations, Section 4.3) and
  h-independent iteration counts near the paper's 5 (Table solver_times_3d).
* Embedding exactness: the prolongation of a coarse Q_k interpolant of a Q_k
  function equals its fine interpolant.
* Adjoint gradient against central finite differences of J.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import adjoint, cg, mg
from oracle.mesh import Box
from seeded_inputs import SEED_KAPPA_FIELD, SEED_KAPPA_PERTURB, gaussian_field


def test_pcg_reaches_direct_solution_and_counts_products():
    out = mg.solve(8, 2, tol=1e-10)
    fine = out["mg"].levels[-1]
    xs = spla.spsolve(fine["A"].tocsc(), cg.rhs(fine["box"]))
    assert np.linalg.norm(out["x"] - xs) <= 1e-9 * np.linalg.norm(xs)
    assert out["residual"] <= 1e-10
    assert out["fine_products"] == 13 * out["iterations"]
    assert 4 <= out["iterations"] <= 6


@pytest.mark.parametrize("k", [2, 3])
def test_iterations_h_independent(k):
    its = [mg.solve(Nc, k, tol=1e-10)["iterations"] for Nc in (4, 8)]
    assert max(its) - min(its) <= 1 and max(its) <= 7


@pytest.mark.parametrize("k", [2, 3])
def test_lanczos_estimate_brackets_dense_max(k):
    m = mg.Multigrid(4, k)
    lev = m.levels[-1]
    inner = ~lev["box"].boundary_mask()
    A = lev["A"][inner][:, inner].toarray()
    d = np.sqrt(lev["Dinv"][inner])
    lmax = np.linalg.eigvalsh(d[:, None] * A * d[None, :]).max()
    assert lev["lambda"] <= lmax * (1 + 1e-12)
    assert 1.2 * lev["lambda"] >= lmax


def test_smoother_error_polynomial():
    m = mg.Multigrid(2, 2, min_cells=1)
    lev = m.levels[-1]
    A, Dinv = lev["A"], lev["Dinv"]
    inner = np.nonzero(~lev["box"].boundary_mask())[0]
    n = A.shape[0]
    # smoother as a matrix: x = S b for b supported in the interior
    S = np.zeros((n, len(inner)))
    for j, i in enumerate(inner):
        e = np.zeros(n)
        e[i] = 1.0
        S[:, j] = mg.chebyshev(A, Dinv, e, None, lev["lo"], lev["hi"], m.cheb_updates)[0]
    Ai = A[inner][:, inner].toarray()
    E = np.eye(len(inner)) - S[inner] @ Ai
    d = np.sqrt(Dinv[inner])
    mu = np.linalg.eigvalsh(d[:, None] * Ai * d[None, :])
    theta = 0.5 * (lev["hi"] + lev["lo"])
    delta = 0.5 * (lev["hi"] - lev["lo"])
    p = np.array([np.polynomial.chebyshev.chebval((theta - x) / delta, [0] * m.cheb_updates + [1])
                  for x in mu]) / np.polynomial.chebyshev.chebval(theta / delta, [0] * m.cheb_updates + [1])
    ev = np.sort(np.linalg.eigvals(E).real)
    np.testing.assert_allclose(ev, np.sort(p), atol=1e-10)


def test_coarse_solver_meets_a_priori_bound():
    m = mg.Multigrid(4, 3)
    lev = m.levels[0]
    A = lev["A"]
    inner = ~lev["box"].boundary_mask()
    rng = np.random.default_rng(3)
    for _ in range(3):
        xs = np.where(inner, rng.uniform(-1, 1, A.shape[0]), 0.0)
        b = A @ xs
        x = mg.chebyshev(A, lev["Dinv"], b, None, lev["lmin"], lev["lmax"], lev["steps"])[0]
        e = x - xs
        assert np.sqrt(e @ (A @ e)) <= 1e-3 * np.sqrt(xs @ (A @ xs))


@pytest.mark.parametrize("k", [2, 3])
def test_prolongation_reproduces_qk_functions(k):
    def f(p):
        x, y, z = p[..., 0], p[..., 1], p[..., 2]
        return x * (1 - x) * (0.3 + x) ** (k - 2) * y * (1 - y) * z * (1 - z) * (0.7 - z) ** (k - 2)
    coarse, fine = Box(2, k), Box(4, k)
    P = mg.prolongation(coarse, fine)
    np.testing.assert_allclose(P @ cg.interpolate(coarse, f), cg.interpolate(fine, f), atol=1e-15)


def test_adjoint_gradient_against_finite_differences():
    Nc, k = 4, 2
    box = Box(Nc, k)
    g = gaussian_field(Nc ** 3, SEED_KAPPA_FIELD, 0.5)
    kap = np.exp(g)
    ut, _ = adjoint.solve_direct(box, np.exp(g + gaussian_field(Nc ** 3, SEED_KAPPA_PERTURB, 0.1)),
                                 cg.rhs(box))
    _, grad, u, lam = adjoint.objective_and_gradient(Nc, k, kap, ut)
    for c in (0, 9, 42, 63):
        eps = 1e-4 * kap[c]
        kp, km = kap.copy(), kap.copy()
        kp[c] += eps
        km[c] -= eps
        fd = (adjoint.objective_and_gradient(Nc, k, kp, ut)[0] -
              adjoint.objective_and_gradient(Nc, k, km, ut)[0]) / (2 * eps)
        assert abs(fd - grad[c]) <= 1e-6 * abs(grad).max()


def test_adjoint_gradient_curved_with_position_dependent_coefficient():
    """The gradient on curved cells with the cosine coefficient of Sec. 4.3 as a factor of the
    cellwise kappa, against central finite differences of J with direct solves."""
    Nc, k, amp = 3, 2, 50.0
    box = Box(Nc, k, 0.1)
    kfn = cg.cosine_coefficient(amp)
    g = gaussian_field(Nc ** 3, SEED_KAPPA_FIELD, 0.5)
    kap = np.exp(g)
    ut, _ = adjoint.solve_direct(box, np.exp(g + gaussian_field(Nc ** 3, SEED_KAPPA_PERTURB, 0.1)),
                                 cg.rhs(box), kfn)
    _, grad, u, lam = adjoint.objective_and_gradient(Nc, k, kap, ut, curve_amp=0.1, kappa_fn=kfn)
    for c in (0, 4, 13, 26):
        eps = 1e-4 * kap[c]
        kp, km = kap.copy(), kap.copy()
        kp[c] += eps
        km[c] -= eps
        fd = (adjoint.objective_and_gradient(Nc, k, kp, ut, 0.1, kfn)[0] -
              adjoint.objective_and_gradient(Nc, k, km, ut, 0.1, kfn)[0]) / (2 * eps)
        assert abs(fd - grad[c]) <= 1e-6 * abs(grad).max()
