"""torch.autograd.Function around the multigrid-preconditioned solve.

forward(kappa) solves A(kappa) u = b; backward(grad_u) solves the adjoint system
A lambda = grad_u (A is symmetric; Dirichlet entries of grad_u are dropped) and
returns dJ/dkappa_c = -lambda_c^T A_c^{(1)} u_c from the per-cell gradient kernel.
"""
import torch


class PoissonSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kappa, problem, b, rtol=1e-10, maxit=100):
        problem.set_kappa(kappa.detach())
        u, _, _ = problem.solve(b, rtol=rtol, maxit=maxit)
        ctx.problem, ctx.rtol, ctx.maxit = problem, rtol, maxit
        ctx.save_for_backward(kappa, u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        kappa, u = ctx.saved_tensors
        problem = ctx.problem
        problem.set_kappa(kappa.detach())
        lam, _, _ = problem.adjoint_solve(grad_u.contiguous(), rtol=ctx.rtol, maxit=ctx.maxit)
        g = problem.kappa_gradient(u, lam)
        return g, None, None, None, None
