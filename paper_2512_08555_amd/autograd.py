"""Differentiable solve: forward = ups_solve, backward = ups_solve_adjoint.

The solve is linear, u = K f with K f = h^2 G1 * f, so dL/df = K^T dL/du;
K^T is applied by the library's adjoint entry point (the same five passes on
the incoming gradient, since G1 is even)."""
import torch


class PoissonSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, plan):
        ctx.plan = plan
        return plan.solve(f.contiguous())

    @staticmethod
    def backward(ctx, grad_u):
        return ctx.plan.adjoint(grad_u.contiguous()), None


def poisson_solve(f, plan):
    """u = K f with autograd support (grad via the hand-written adjoint)."""
    return PoissonSolve.apply(f, plan)
