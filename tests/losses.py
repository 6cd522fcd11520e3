"""Weighted gradient-energy loss of the differentiable workload (test and
benchmark harness, not part of the solver):

    L(u) = h^3 sum_{interior i} w[i] |D u[i]|^2,

D the second-order central-difference gradient, interior = points whose six
neighbours lie in the grid.  L is quadratic in u, hence in f for u = K f, so
a central finite difference of L is exact up to rounding."""
import torch


def grad_energy(u, w, h):
    inv = 1.0 / (2.0 * h)
    dx = (u[1:-1, 1:-1, 2:] - u[1:-1, 1:-1, :-2]) * inv
    dy = (u[1:-1, 2:, 1:-1] - u[1:-1, :-2, 1:-1]) * inv
    dz = (u[2:, 1:-1, 1:-1] - u[:-2, 1:-1, 1:-1]) * inv
    return h ** 3 * (w[1:-1, 1:-1, 1:-1] * (dx * dx + dy * dy + dz * dz)).sum()


def loss_grad_u(u, w, h):
    """dL/du, by torch autograd (any device and dtype)."""
    uu = u.detach().clone().requires_grad_(True)
    grad_energy(uu, w, h).backward()
    return uu.grad.detach()
