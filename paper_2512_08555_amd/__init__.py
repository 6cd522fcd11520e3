"""MI355X-native unbounded (free-space) Poisson solver: Python binding of the
``libups`` C-ABI library declared in include/ups.h.

    from paper_2512_08555_amd import Plan
    plan = Plan((nz, ny, nx), h, prec="f32")      # builds G_hat on the GPU
    u = plan.solve(f)                               # u = h^2 G1 * f

The HIP library is loaded on first use; importing the package alone (for
``workloads``) does not need it, and every solver call raises if it is not
built.
"""

__all__ = ["Plan", "Batch", "Multigrid", "solve", "PoissonSolve", "poisson_solve", "supported_length", "auto_pad"]


def __getattr__(name):
    if name in ("Plan", "Batch", "Multigrid", "solve"):
        from . import solver
        return getattr(solver, name)
    if name in ("PoissonSolve", "poisson_solve"):
        from . import autograd
        return getattr(autograd, name)
    if name in ("supported_length", "auto_pad"):
        from . import lengths
        return getattr(lengths, name)
    raise AttributeError(name)
