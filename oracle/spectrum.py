"""Spectrum of the zero-padded lattice Green's function -- ORACLE, test
infrastructure only (see ``oracle/__init__.py``).

Sec. 2.2 states the solve in spectral space as u_hat = G_hat f_hat.  On a
box of N_i points per axis the free-space lattice convolution is reproduced
exactly by a circular convolution of length M_i >= 2 N_i - 2 when the kernel
is periodised evenly (the paper is silent on this; it is the classical
Hockney-Eastwood construction it cites):

    Gp[i] = G1[min(i_z, M_z - i_z), min(i_y, M_y - i_y), min(i_x, M_x - i_x)].

Gp is real and even, so its DFT is real and even and is fully described by
the octant k_i in [0, M_i/2]; on that octant it equals the type-I DCT of the
G1 octant [0, M_i/2] (scipy's unnormalised DCT-I).
"""

import numpy as np
import scipy.fft as sfft

from .lgf import lgf_table


def _octant_extents(M):
    M = tuple(int(m) for m in M)
    if any(m % 2 for m in M):
        raise ValueError("padded lengths must be even")
    return M, tuple(m // 2 + 1 for m in M)


def green_spectrum_raw(M, G1=None):
    """DFT of the evenly periodised G1 on the (Mz, My, Mx) torus, octant
    [0, Mz/2] x [0, My/2] x [0, Mx/2], computed as dctn(G1 octant, type=1).
    Unscaled: it multiplies f_hat when the inverse DFT carries 1/(Mz My Mx)."""
    M, K = _octant_extents(M)
    if G1 is None:
        G1 = lgf_table(*K)
    G1 = np.asarray(G1)[: K[0], : K[1], : K[2]]
    return sfft.dctn(G1, type=1)


def green_spectrum_rfft(M):
    """The same octant computed the long way: build the full periodised
    kernel Gp on the torus and take its real-input DFT.  For small M only."""
    M, K = _octant_extents(M)
    G1 = lgf_table(*K)
    iz = np.minimum(np.arange(M[0]), M[0] - np.arange(M[0]))
    iy = np.minimum(np.arange(M[1]), M[1] - np.arange(M[1]))
    ix = np.minimum(np.arange(M[2]), M[2] - np.arange(M[2]))
    Gp = G1[np.ix_(iz, iy, ix)]
    full = np.fft.rfftn(Gp)
    return full[: K[0], : K[1], :]


def green_spectrum_scaled(M, h, G1=None):
    """h^2 / (Mz My Mx) times the raw octant: the spectrum that, with
    unnormalised forward and inverse DFTs, maps f to u = h^2 G1 * f."""
    M = tuple(int(m) for m in M)
    return (float(h) ** 2 / float(M[0] * M[1] * M[2])) * green_spectrum_raw(M, G1)
