"""GPU adjoint gradient dJ/dkappa (PoissonSolve autograd function) against the oracle and
finite differences.

J(kappa) = 1/2 ||u(kappa) - u_target||^2 with A(kappa) u = b (sine right-hand side),
kappa = exp(g) cellwise, g i.i.d. N(0, 0.5^2); u_target solves the problem with
kappa exp(delta), delta i.i.d. N(0, 0.1^2).
"""
import numpy as np
import pytest
import torch

import paper_1611_03029_amd as mfl
from oracle import adjoint as o_adj
from oracle import cg as o_cg
from oracle.mesh import Box
from seeded_inputs import (SEED_FD_CELLS, SEED_KAPPA_FIELD, SEED_KAPPA_PERTURB, choose_cells,
                           gaussian_field)

pytestmark = pytest.mark.gpu


def setup_problem(Nc, k, prec):
    g = gaussian_field(Nc ** 3, SEED_KAPPA_FIELD, 0.5)
    kap = np.exp(g)
    kap_t = np.exp(g + gaussian_field(Nc ** 3, SEED_KAPPA_PERTURB, 0.1))
    prob = mfl.Problem(k, Nc, build_mg=True, mg_precision=prec, kappa=kap)
    b = prob.rhs_sine()
    return prob, b, kap, kap_t


def objective(prob, b, kappa, u_t, rtol):
    prob.set_kappa(kappa)
    u, _, _ = prob.solve(b, rtol=rtol, maxit=200)
    return 0.5 * float(((u - u_t) ** 2).sum())


@pytest.mark.parametrize("prec", [mfl.F64, mfl.F32])
def test_gradient_matches_oracle_small(prec):
    Nc, k = 4, 3
    prob, b, kap, kap_t = setup_problem(Nc, k, prec)
    box = Box(Nc, k)
    ut_ref, _ = o_adj.solve_direct(box, kap_t, o_cg.rhs(box))
    J_ref, g_ref, _, _ = o_adj.objective_and_gradient(Nc, k, kap, ut_ref)
    kt = torch.tensor(kap, device="cuda", requires_grad=True)
    u = mfl.PoissonSolve.apply(kt, prob, b, 1e-13, 200)
    J = 0.5 * ((u - torch.tensor(ut_ref, device="cuda")) ** 2).sum()
    J.backward()
    assert abs(J.item() - J_ref) <= 1e-9 * J_ref
    g = kt.grad.cpu().numpy()
    assert np.abs(g - g_ref).max() <= 1e-8 * np.abs(g_ref).max()


def test_gradient_finite_differences_q3_32cubed():
    """CG Q3 on 32^3 cells, FP64 outer / FP32 multigrid, 20 random cells: central differences
    with step 1e-4 kappa_c, forward solves to 1e-14, agreement within 1e-5 of each cell's
    gradient."""
    Nc, k = 32, 3
    prob, b, kap, kap_t = setup_problem(Nc, k, mfl.F32)
    prob.set_kappa(kap_t)
    u_t, _, _ = prob.solve(b, rtol=1e-14, maxit=200)
    kt = torch.tensor(kap, device="cuda", requires_grad=True)
    u = mfl.PoissonSolve.apply(kt, prob, b, 1e-14, 200)
    (0.5 * ((u - u_t) ** 2).sum()).backward()
    g = kt.grad.cpu().numpy()
    cells = choose_cells(Nc ** 3, 20, SEED_FD_CELLS)
    errs = []
    for c in cells:
        eps = 1e-4 * kap[c]
        kp, km = kap.copy(), kap.copy()
        kp[c] += eps
        km[c] -= eps
        fd = (objective(prob, b, kp, u_t, 1e-14) - objective(prob, b, km, u_t, 1e-14)) / (2 * eps)
        errs.append(abs(fd - g[c]) / abs(g[c]))
        print("cell %d: gradient %.6e, central difference %.6e, relative deviation %.2e" % (
            c, g[c], fd, errs[-1]), flush=True)
    assert max(errs) <= 1e-5


def test_gradcheck_tiny():
    prob = mfl.Problem(2, 2, build_mg=True, min_level_cells=2)
    b = prob.rhs_sine()
    u_t = torch.zeros(prob.n_dofs, dtype=torch.float64, device="cuda")

    def J(kappa):
        u = mfl.PoissonSolve.apply(kappa, prob, b, 1e-15, 500)
        return 0.5 * ((u - u_t) ** 2).sum()

    kappa = torch.tensor(np.exp(gaussian_field(8, 11, 0.3)), device="cuda", requires_grad=True)
    # the Jacobi diagonal is assembled with atomics at setup, so two backward calls agree
    # to rounding (about 1e-15) rather than bitwise
    assert torch.autograd.gradcheck(J, (kappa,), eps=1e-6, atol=1e-7, rtol=1e-5, nondet_tol=1e-12)
