r"""Poisson solve with a boundary condition per axis -- ORACLE, test
infrastructure only (see ``oracle/__init__.py``).

Sec. 2.2 lists the conditions a direction may carry: unbounded, periodic,
even (homogeneous Neumann) and odd (homogeneous Dirichlet).  Periodic
directions use the spectral expression of the lattice Green's function,
even and odd ones the cosine and sine transforms, unbounded ones the LGF of
the operator.  For two unbounded directions eq. 2unbkernel fixes the kernel:
the two-dimensional LGF's spectrum on the zero wavenumber of the third
direction, the inverse symbol 1/sigma everywhere else.  Sec. 3.3 states that
the LGFs for one and for three unbounded directions are known; for one, the
lattice Green's function of the one-dimensional operator screened by the
other directions' symbol is closed-form (below).

The discrete problem on a box of N_i cells per axis (arrays [z, y, x],
cell-centred, spacing h, 7-point operator L of eq. cross_discr2):

    (1/h^2) (L u)[i] = f[i]   for every cell i of the box,

where a neighbour outside the box is
  * periodic:  u[i + N] = u[i];
  * even:      the mirror image about the box face, u[-1] = u[0], u[N] = u[N-1];
  * odd:       the negated mirror image, u[-1] = -u[0], u[N] = -u[N-1];
  * unbounded: the value of the free-space solution (no boundary; u is the
    convolution of f, zero outside the box, with the mixed Green's function).

When no direction is unbounded and no direction is odd the problem is
singular: the solve returns the solution of zero mean for the source with
its mean removed (the spectral kernel is 0 at wavenumber 0).  The
one-dimensional LGF (one unbounded direction, zero transverse wavenumber) is
|n|/2 and the two-dimensional one is normalised by G[0, 0] = 0; both grow
at infinity, and the constant they leave open only shifts u by a multiple of
the source's total.

The solve is the plain route, one transform per axis: a length-N DFT along a
periodic axis, the DFT of the even (or odd) extension to length 2N along an
even (or odd) axis, and the DFT of the zero-padded data of length M >= 2N
along an unbounded axis; the product with the kernel sampled on that
frequency grid; the inverse DFT; the box.
"""

from math import pi

import numpy as np

from .lgf import lgf_table, quadrature_nodes, hankel_coefficients, default_T
from scipy import special

BCS = ("unb", "per", "even", "odd")


# ---- lower-dimensional lattice Green's functions ------------------------------

def _tail2_moment(m, T):
    # \int_T^inf (4 pi t)^-1 (2t)^-m dt, m >= 1
    return (4.0 * pi) ** -1.0 * 2.0 ** (-m) * T ** (-float(m)) / m


def lgf2d_table(k0, k1, T=None, K=6):
    r"""Two-dimensional LGF of the 5-point Laplacian normalised by G[0,0] = 0,
    on the quadrant 0 <= n0 < k0, 0 <= n1 < k1:

        G[n] = (2 pi)^-2 \int (cos(k.n) - 1) / (-sigma(k)) dk
             = - \int_0^inf (e^{-4t} I_{n0}(2t) I_{n1}(2t) - e^{-4t} I_0(2t)^2) dt,

    sigma = sum (2 - 2 cos k_i).  The same composite Gauss-Legendre rule in
    ln t as the three-dimensional table on [0, T]; on [T, inf) the product of
    the two Hankel series minus its value at n = 0 (the leading terms cancel),
    integrated term by term."""
    k0, k1 = int(k0), int(k1)
    n_max = max(k0, k1) - 1
    T = default_T(max(n_max, 1)) if T is None else float(T)
    t, w = quadrature_nodes(T)
    B0 = special.ive(np.arange(k0)[:, None], 2.0 * t[None, :])
    B1 = special.ive(np.arange(k1)[:, None], 2.0 * t[None, :])
    b00 = special.ive(0, 2.0 * t) ** 2
    quad = (B0 * w[None, :]) @ B1.T - np.sum(w * b00)
    c0 = hankel_coefficients(np.arange(k0), K)
    c1 = hankel_coefficients(np.arange(k1), K)
    cz = hankel_coefficients(np.array([0]), K)[:, 0]
    tail = np.zeros((k0, k1))
    for a in range(K + 1):
        for b in range(K + 1 - a):
            m = a + b
            if m == 0:
                continue
            g = _tail2_moment(m, T)
            tail += g * (np.outer(c0[a], c1[b]) - cz[a] * cz[b])
    return -(quad + tail)


def lgf1d_screened(n, s):
    r"""The decaying solution of G[n+1] - 2 G[n] + G[n-1] - s G[n] = delta[n]
    (s > 0): G[n] = -rho^|n| / sqrt(s (s + 4)), rho the root of
    rho^2 - (2 + s) rho + 1 = 0 inside the unit circle.  For s = 0 the
    one-dimensional LGF |n| / 2."""
    n = np.abs(np.asarray(n, dtype=np.float64))
    s = np.asarray(s, dtype=np.float64)
    n, s = np.broadcast_arrays(n, s)
    out = np.empty(np.broadcast(n, s).shape)
    z = s == 0
    out[z] = 0.5 * n[z]
    sp = s[~z]
    root = np.sqrt(sp * (sp + 4.0))
    # rho = 1 / (1 + s/2 + sqrt(s + s^2/4)), log taken without cancellation
    log_rho = -np.log1p(0.5 * sp + 0.5 * root)
    out[~z] = -np.exp(n[~z] * log_rho) / root
    return out


# ---- the kernel on the solve's frequency grid ----------------------------------

def _check_bc(bc):
    bc = tuple(str(b) for b in bc)
    if len(bc) != 3 or any(b not in BCS for b in bc):
        raise ValueError("bc must be three of %s in (z, y, x) order" % (BCS,))
    return bc


def transform_lengths(shape, bc, M=None):
    """Length of the transform along each axis: N (periodic), 2N (even,
    odd), the padded M >= 2N (unbounded; default 2N)."""
    bc = _check_bc(bc)
    out = []
    for i, (n, b) in enumerate(zip(shape, bc)):
        if b == "per":
            out.append(int(n))
        elif b in ("even", "odd"):
            out.append(2 * int(n))
        else:
            m = 2 * int(n) if M is None else int(M[i])
            if m % 2 or m < 2 * int(n) - 2:
                raise ValueError("padded length %d invalid for %d points" % (m, n))
            out.append(m)
    return tuple(out)


def _symbol_1d(L):
    k = np.arange(L)
    return 4.0 * np.sin(pi * k / L) ** 2


def _even_embed(g, L):
    """Kernel values g[0 .. L/2] of an even function -> the L-torus sequence
    g[min(i, L - i)]."""
    i = np.arange(L)
    return g[np.minimum(i, L - i)]


def kernel_spectrum(L, bc, shape=None):
    """G_tilde on the full frequency grid of shape L = transform_lengths(...),
    for unit spacing: u = IDFT(G_tilde DFT(f_ext)) h^2 solves the problem
    (the DFTs unnormalised, the inverse carrying 1 / prod L)."""
    bc = _check_bc(bc)
    L = tuple(int(v) for v in L)
    unb = [i for i in range(3) if bc[i] == "unb"]
    spec = [i for i in range(3) if bc[i] != "unb"]
    s = [_symbol_1d(L[i]) for i in range(3)]
    grids = np.meshgrid(*s, indexing="ij")
    sigma = grids[0] + grids[1] + grids[2]
    if len(unb) == 3:
        K = tuple(l // 2 + 1 for l in L)
        G = lgf_table(*K)
        Gp = G[np.ix_(*[np.minimum(np.arange(l), l - np.arange(l)) for l in L])]
        return np.real(np.fft.fftn(Gp))
    if len(unb) == 0:
        out = np.zeros(L)
        nz = sigma != 0
        out[nz] = -1.0 / sigma[nz]
        return out
    if len(unb) == 2:
        a, b = unb
        c = spec[0]
        out = np.zeros(L)
        nz = sigma != 0
        out[nz] = -1.0 / sigma[nz]
        # zero wavenumber of the third direction: the 2-D LGF's spectrum
        G2 = lgf2d_table(L[a] // 2 + 1, L[b] // 2 + 1)
        ia = np.minimum(np.arange(L[a]), L[a] - np.arange(L[a]))
        ib = np.minimum(np.arange(L[b]), L[b] - np.arange(L[b]))
        plane = np.real(np.fft.fft2(G2[np.ix_(ia, ib)]))
        idx = [slice(None)] * 3
        idx[c] = 0
        # plane is indexed (a, b) with a < b in axis order
        out[tuple(idx)] = plane
        return out
    # one unbounded direction a: per transverse wavenumber, the screened 1-D LGF
    a = unb[0]
    la = L[a]
    ia = np.minimum(np.arange(la), la - np.arange(la))
    st = sigma.take(0, axis=a)          # transverse symbol (a-wavenumber 0 term is 0)
    tab = lgf1d_screened(ia[:, None], st.reshape(1, -1))      # (la, ntrans)
    spec_a = np.real(np.fft.fft(tab, axis=0))                  # (la, ntrans)
    shp = list(L)
    shp.pop(a)
    spec_a = spec_a.reshape([la] + shp)
    return np.moveaxis(spec_a, 0, a)


def extend(f, bc, L):
    """The source on the transform grid: zero padding (unbounded), itself
    (periodic), its even or odd extension to 2N about the box face."""
    bc = _check_bc(bc)
    g = np.asarray(f, dtype=np.float64)
    for ax in range(3):
        n = g.shape[ax]
        if bc[ax] == "unb":
            pad = [(0, 0)] * 3
            pad[ax] = (0, L[ax] - n)
            g = np.pad(g, pad)
        elif bc[ax] == "even":
            g = np.concatenate([g, np.flip(g, axis=ax)], axis=ax)
        elif bc[ax] == "odd":
            g = np.concatenate([g, -np.flip(g, axis=ax)], axis=ax)
    return g


def solve_bc(f, h, bc, M=None):
    """u on the box (arrays [z, y, x], bc in the same order)."""
    f = np.asarray(f, dtype=np.float64)
    bc = _check_bc(bc)
    L = transform_lengths(f.shape, bc, M)
    G = kernel_spectrum(L, bc)
    F = np.fft.fftn(extend(f, bc, L))
    u = np.fft.ifftn(F * (float(h) ** 2 * G))
    N = f.shape
    return np.ascontiguousarray(np.real(u[: N[0], : N[1], : N[2]]))


# ---- the discrete operator with the boundary rules, for checks ------------------

def ghost_pad(u, bc):
    """u with one ghost layer per side along every non-unbounded axis, filled
    by the boundary rule; unbounded axes are left without ghosts."""
    bc = _check_bc(bc)
    g = np.asarray(u, dtype=np.float64)
    for ax in range(3):
        b = bc[ax]
        if b == "unb":
            continue
        first = np.take(g, [0], axis=ax)
        last = np.take(g, [g.shape[ax] - 1], axis=ax)
        if b == "per":
            lo, hi = last, first
        elif b == "even":
            lo, hi = first, last
        else:
            lo, hi = -first, -last
        g = np.concatenate([lo, g, hi], axis=ax)
    return g


def laplacian_bc(u, h, bc):
    """(1/h^2) L u on the cells whose neighbours exist: every cell along
    periodic, even and odd axes (through the ghosts), the interior cells
    along unbounded axes."""
    bc = _check_bc(bc)
    g = ghost_pad(u, bc)
    c = g[1:-1, 1:-1, 1:-1]
    lap = (g[2:, 1:-1, 1:-1] + g[:-2, 1:-1, 1:-1] + g[1:-1, 2:, 1:-1] + g[1:-1, :-2, 1:-1]
           + g[1:-1, 1:-1, 2:] + g[1:-1, 1:-1, :-2] - 6.0 * c)
    return lap / float(h) ** 2


def interior_cells(shape, bc):
    """The box cells laplacian_bc returns, as slices of the box."""
    bc = _check_bc(bc)
    return tuple(slice(1, n - 1) if b == "unb" else slice(0, n) for n, b in zip(shape, bc))
