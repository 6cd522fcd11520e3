"""Free-space Poisson solve u = h^2 (G1 * f) on a uniform box -- ORACLE, test
infrastructure only (see ``oracle/__init__.py``).

Problem (eq. poisson_problem with unbounded conditions, Sec. 1 and Sec. 2.2):
the Laplacian of u equals f, u -> 0 at infinity.  Discretised with the
7-point stencil of eq. cross_discr2 and solved with the LGF of that stencil
(Sec. 2.2 and Sec. 3.3: the kernel must be the LGF of the operator), the
discrete free-space solution for a source f given on the box and zero
outside it is the lattice sum

    u[i] = h^2 sum_{j in box} G1[i - j] f[j],      i in box,

which is the unique decaying solution of (1/h^2) L u = f 1_box on Z^3.
Arrays are indexed [z, y, x] (x fastest); h is the isotropic spacing.
"""

import os

import numpy as np
import scipy.fft as sfft

from .lgf import lgf_table
from .spectrum import green_spectrum_raw


def _default_M(shape):
    return tuple(2 * int(n) for n in shape)


def _check_M(shape, M):
    for n, m in zip(shape, M):
        if m % 2 or m < 2 * n - 2:
            raise ValueError("padded length %d invalid for %d points" % (m, n))


def _workers(workers):
    if workers is not None:
        return int(workers)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _mirror(M):
    k = np.arange(M)
    return np.minimum(k, M - k)


def solve_full(f, h, M=None):
    """Circular convolution on the padded (Mz, My, Mx) torus by the
    convolution theorem, without pruning: zero-pad f, real DFT, multiply by
    h^2 times the DFT of the periodised kernel, inverse DFT, crop.
    Small grids only."""
    f = np.asarray(f, dtype=np.float64)
    N = f.shape
    M = _default_M(N) if M is None else tuple(M)
    _check_M(N, M)
    Gh = green_spectrum_raw(M)
    full = Gh[np.ix_(_mirror(M[0]), _mirror(M[1]), np.arange(M[2] // 2 + 1))]
    fh = np.fft.rfftn(f, s=M, axes=(0, 1, 2))
    u = np.fft.irfftn(fh * (float(h) ** 2 * full), s=M, axes=(0, 1, 2))
    return u[: N[0], : N[1], : N[2]]


def solve(f, h, M=None, G_hat_raw=None, workers=None, chunk=64):
    """The pad-to-M FFT convolution taken one axis at a time, skipping what
    is known to be zero (padded inputs) or discarded (cropped outputs):

      1. real DFT along x of the zero-padded rows           (Nz, Ny, Mx/2+1)
      2. DFT along y of the zero-padded columns             (Nz, My, Mx/2+1)
      3. along z: DFT of the zero-padded lines, times h^2 G_hat, inverse DFT,
         keep z < Nz
      4. inverse DFT along y, keep y < Ny
      5. inverse real DFT along x, keep x < Nx.

    Same arithmetic as ``solve_full`` up to rounding order; bounded memory
    at 512^3.  ``G_hat_raw`` may pass a precomputed ``green_spectrum_raw(M)``."""
    f = np.asarray(f, dtype=np.float64)
    Nz, Ny, Nx = f.shape
    M = _default_M(f.shape) if M is None else tuple(M)
    _check_M(f.shape, M)
    Mz, My, Mx = M
    w = _workers(workers)
    Gh = green_spectrum_raw(M) if G_hat_raw is None else np.asarray(G_hat_raw)
    h2 = float(h) ** 2
    F = sfft.rfft(f, n=Mx, axis=2, workers=w)
    F = sfft.fft(F, n=My, axis=1, workers=w)
    iz = _mirror(Mz)
    iy = _mirror(My)
    for y0 in range(0, My, chunk):
        y1 = min(My, y0 + chunk)
        line = sfft.fft(F[:, y0:y1, :], n=Mz, axis=0, workers=w)
        line *= h2 * Gh[np.ix_(iz, iy[y0:y1], np.arange(Gh.shape[2]))]
        F[:, y0:y1, :] = sfft.ifft(line, axis=0, workers=w)[:Nz]
        del line
    F = sfft.ifft(F, axis=1, workers=w)[:, :Ny, :]
    u = sfft.irfft(F, n=Mx, axis=2, workers=w)[:, :, :Nx]
    return np.ascontiguousarray(u)


def adjoint(g, h, M=None, G_hat_raw=None, workers=None):
    """Adjoint of f -> u: (K^T g)[j] = h^2 sum_i G1[i - j] g[i].  G1 is even
    in every index (the stencil is symmetric), so K^T = K and the adjoint
    is the same convolution applied to g."""
    return solve(g, h, M=M, G_hat_raw=G_hat_raw, workers=workers)


def _offset_table(shape):
    return lgf_table(*shape)


def brute_force(f, h):
    """The defining lattice sum, evaluated directly: O(N^6), tiny grids only."""
    f = np.asarray(f, dtype=np.float64)
    Nz, Ny, Nx = f.shape
    G1 = _offset_table(f.shape)
    jz, jy, jx = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    u = np.empty_like(f)
    for iz in range(Nz):
        for iy in range(Ny):
            for ix in range(Nx):
                k = G1[np.abs(iz - jz), np.abs(iy - jy), np.abs(ix - jx)]
                u[iz, iy, ix] = np.sum(k * f)
    return float(h) ** 2 * u


def brute_force_adjoint(g, h):
    """(K^T g)[j] = h^2 sum_i G1[i - j] g[i], the transpose of ``brute_force``
    written out directly."""
    g = np.asarray(g, dtype=np.float64)
    Nz, Ny, Nx = g.shape
    # G1 on Z^3 is read from its octant at |offset| (the Fourier integral of
    # the LGF is even in every k_i); the sum runs over the output index i.
    G1 = _offset_table(g.shape)
    iz, iy, ix = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    out = np.empty_like(g)
    for jz in range(Nz):
        for jy in range(Ny):
            for jx in range(Nx):
                k = G1[np.abs(iz - jz), np.abs(iy - jy), np.abs(ix - jx)]
                out[jz, jy, jx] = np.sum(k * g)
    return float(h) ** 2 * out


def laplacian7_interior(u, h):
    """(1/h^2) [d_xx + d_yy + d_zz] u with d = [1 -2 1] (eq. cross_discr2), on
    the points whose six neighbours all lie in the array: shape (N-2)^3."""
    u = np.asarray(u, dtype=np.float64)
    c = u[1:-1, 1:-1, 1:-1]
    lap = (u[2:, 1:-1, 1:-1] + u[:-2, 1:-1, 1:-1]
           + u[1:-1, 2:, 1:-1] + u[1:-1, :-2, 1:-1]
           + u[1:-1, 1:-1, 2:] + u[1:-1, 1:-1, :-2] - 6.0 * c)
    return lap / float(h) ** 2
