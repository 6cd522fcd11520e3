"""Plain FP64 CPU oracle for the unbounded (free-space) Poisson solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` use it.  It shares no code with the HIP library
(``paper_2512_08555_amd``) and imports nothing from it.

What it computes (Poncelet, Lambrechts, Gillis, Chatelain, "A scalable
high-order multigrid-FFT Poisson solver for unbounded domains on adaptive
multiresolution grids"):

* ``lgf``      -- the lattice Green's function G1 of the 7-point Laplacian,
                  the solution of L G = delta (Sec. 2.2, LGF definition;
                  stencil of eq. cross_discr2), by a separable Bessel
                  quadrature of its Fourier integral.
* ``spectrum`` -- the spectrum of the zero-padded, evenly periodised kernel
                  (Sec. 2.2, u_hat = G_hat f_hat), as a DCT-I of the octant.
* ``solve``    -- u = h^2 (G1 * f) on the box: the zero-padded FFT
                  convolution, the same product without pruning, and the
                  brute-force lattice sum that defines it.
* ``bc``       -- the solve with a boundary condition per axis (unbounded,
                  periodic, even, odd; Sec. 2.2 and eq. 2unbkernel), by one
                  plain transform per axis, and the lower-dimensional lattice
                  Green's functions it needs.
* ``mehrstellen`` -- the fourth- and sixth-order Mehrstellen pairs (eqs.
                  mehrstellen_discr4/6): the LGF of L by the 7-point LGF plus
                  a graded quadrature of the bounded difference of the inverse
                  symbols, the kernel R G_L, and the solve with it.
* ``multigrid`` -- the V(eta1, eta2) full-approximation cycle around the
                  unbounded solve (Sec. 3.1, Alg. amg_vcycle) on a hierarchy
                  of nested refined boxes, and the composite equations its
                  fixed point satisfies, solved directly for small grids.
* ``analytic`` -- closed forms used as pins: Watson's constant, the Gaussian
                  charge potential, the paper's compact manufactured solution
                  (Sec. 4.2, unbounded domains).

Every routine runs in float64 on the CPU.
"""

from .lgf import (watson_g0, lgf_table, lgf_point_adaptive, lgf_far_field,
                  lgf_tail, quadrature_nodes, hankel_coefficients)
from .spectrum import green_spectrum_raw, green_spectrum_rfft, green_spectrum_scaled
from .solve import (solve, solve_full, brute_force, brute_force_adjoint,
                    adjoint, laplacian7_interior)
from . import analytic, bc, mehrstellen, multigrid

__all__ = [
    "watson_g0", "lgf_table", "lgf_point_adaptive", "lgf_far_field", "lgf_tail",
    "quadrature_nodes", "hankel_coefficients",
    "green_spectrum_raw", "green_spectrum_rfft", "green_spectrum_scaled",
    "solve", "solve_full", "brute_force", "brute_force_adjoint", "adjoint",
    "laplacian7_interior", "analytic", "bc", "mehrstellen", "multigrid",
]
