r"""Mehrstellen kernels (eqs. mehrstellen_discr4 and mehrstellen_discr6) --
ORACLE, test infrastructure only (see ``oracle/__init__.py``).

The compact fourth- and sixth-order discretisations of Sec. 3.2 apply one
stencil to u and another to f (unit spacing; d2 the 3-point second
difference along an axis, d4 = d2 d2):

    L4 = sum d2 + (1/6) sum_{i<j} d2_i d2_j
    L6 = L4 + (1/30) d2_x d2_y d2_z
    R4 = 1 + (1/12) sum d2
    R6 = R4 + (1/90) sum_{i<j} d2_i d2_j - (1/240) sum d4

(the paper prints "delta_y delta_z^2" in the second R6 term; the symmetric
d2_y d2_z is the reading taken, as in the stencil figure).  With
s_i = 4 sin^2(k_i / 2) the symbol of d2 is -s_i, so L has the symbol
-sigma and R the symbol rho:

    sigma4 = sum s - (1/6) sum_{i<j} s_i s_j,    sigma6 = sigma4 + (1/30) s_x s_y s_z
    rho4 = 1 - (1/12) sum s,    rho6 = rho4 + (1/90) sum_{i<j} s_i s_j - (1/240) sum s^2.

The discrete problem (1/h^2) L u = R (f 1_box), u decaying, has the solution
u = h^2 G_L * (R f) = h^2 (R G_L) * f, with G_L the LGF of L (L G_L = delta;
Sec. 3.3: the kernel must be the LGF of the operator).  So the unbounded
solve of Sec. 2.2 runs unchanged with the kernel K = R G_L.

G_L is computed as G1 (the 7-point LGF of ``lgf``) plus

    D[n] = -(2 pi)^-3 \int_{[-pi, pi]^3} cos(k.n) (1/sigma_L(k) - 1/sigma_2(k)) dk,

whose integrand is bounded (its only irregularity is a direction-dependent
limit at k = 0).  The integral over [0, pi]^3 (the integrand is even in
each k_i) uses the tensor cube of a one-dimensional composite 16-point
Gauss-Legendre rule whose panels halve towards 0 (breakpoints pi 2^-j,
j = 0 .. J, and the panel [0, pi 2^-J]) and are split further so that no
panel spans more than one period of cos(n_max k).  Every box of that grid
away from the origin sees an integrand analytic on a neighbourhood of its
own size; only the corner box [0, pi 2^-J]^3 is not, and its whole
contribution is below 1e-17 for J = 20.
"""

from math import pi

import numpy as np
import scipy.fft as sfft

from .lgf import lgf_table

ORDERS = (4, 6)
J_GRADE = 20
PANEL = 16


def symbols(s, order):
    """(sigma, rho) of the order-4 or order-6 Mehrstellen pair for
    s = (s_x, s_y, s_z) arrays (broadcastable)."""
    sx, sy, sz = s
    S = sx + sy + sz
    P = sx * sy + sy * sz + sz * sx
    sigma = S - P / 6.0
    rho = 1.0 - S / 12.0
    if order == 6:
        sigma = sigma + sx * sy * sz / 30.0
        rho = rho + P / 90.0 - (sx * sx + sy * sy + sz * sz) / 240.0
    elif order != 4:
        raise ValueError("order must be 4 or 6")
    return sigma, rho


def rule_1d(n_max, J=None):
    """Nodes and weights of the graded composite Gauss-Legendre rule on [0, pi]."""
    J = J_GRADE if J is None else int(J)
    x, w = np.polynomial.legendre.leggauss(PANEL)
    edges = [0.0] + [pi * 2.0 ** (-j) for j in range(J, -1, -1)]
    nodes, weights = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        m = max(1, int(np.ceil((b - a) * max(n_max, 1) / (2 * pi))))
        sub = np.linspace(a, b, m + 1)
        for c, d in zip(sub[:-1], sub[1:]):
            half, mid = 0.5 * (d - c), 0.5 * (d + c)
            nodes.append(mid + half * x)
            weights.append(half * w)
    return np.concatenate(nodes), np.concatenate(weights)


def lgf_difference(kz, ky, kx, order):
    """D on the octant [0, kz) x [0, ky) x [0, kx): G_L = G1 + D."""
    n_max = max(kz, ky, kx) - 1
    k, w = rule_1d(n_max)
    s = 4.0 * np.sin(0.5 * k) ** 2
    # cos(n k_a) w_a per axis
    Cz = np.cos(np.outer(np.arange(kz), k)) * w[None, :]
    Cy = np.cos(np.outer(np.arange(ky), k)) * w[None, :]
    Cx = np.cos(np.outer(np.arange(kx), k)) * w[None, :]
    sy = s[:, None]
    sx = s[None, :]
    D = np.zeros((kz, ky, kx))
    for a in range(k.size):
        sig, _ = symbols((sx, sy, s[a]), order)
        sig2 = sx + sy + s[a]
        with np.errstate(divide="ignore", invalid="ignore"):
            delta = np.where(sig2 > 0, 1.0 / sig - 1.0 / sig2, 0.0)
        # plane [ky, kx] = Cy delta Cx^T, accumulated with weight Cz[:, a]
        plane = Cy @ delta @ Cx.T
        D += Cz[:, a, None, None] * plane[None, :, :]
    return -D / pi ** 3


def lgf_table_mehrstellen(kz, ky, kx, order):
    """G_L on the octant: the LGF of L4 or L6."""
    return lgf_table(kz, ky, kx) + lgf_difference(kz, ky, kx, order)


def _mirror_full(G):
    f = np.concatenate([G[:0:-1], G], 0)
    f = np.concatenate([f[:, :0:-1], f], 1)
    return np.concatenate([f[:, :, :0:-1], f], 2)


def _d2(a, axis):
    """Second difference along `axis`, shrinking that extent by 2."""
    n = a.shape[axis]
    lo = np.take(a, range(0, n - 2), axis=axis)
    mid = np.take(a, range(1, n - 1), axis=axis)
    hi = np.take(a, range(2, n), axis=axis)
    return lo - 2.0 * mid + hi


def _crop(a, r):
    """Remove r layers on every side of a 3-D array."""
    return a[r:a.shape[0] - r, r:a.shape[1] - r, r:a.shape[2] - r]


def apply_stencil(a, kind, order):
    """L or R of the given order applied to a full (mirrored) array; the
    result loses the stencil radius (1, or 2 for R6) on every side."""
    r = 2 if (kind == "R" and order == 6) else 1
    d2 = [_d2(a, ax) for ax in range(3)]

    def fit(b):           # crop an array that lost 2 layers along one axis to radius r
        out = b
        for ax in range(3):
            lost = (a.shape[ax] - out.shape[ax]) // 2
            sl = [slice(None)] * 3
            sl[ax] = slice(r - lost, out.shape[ax] - (r - lost))
            out = out[tuple(sl)]
        return out

    d2d2 = {}
    for i in range(3):
        for j in range(i + 1, 3):
            d2d2[(i, j)] = _d2(d2[i], j)
    if kind == "L":
        out = sum(fit(d2[i]) for i in range(3)) + sum(fit(v) for v in d2d2.values()) / 6.0
        if order == 6:
            out = out + fit(_d2(d2d2[(0, 1)], 2)) / 30.0
        return out
    out = _crop(a, r) + sum(fit(d2[i]) for i in range(3)) / 12.0
    if order == 6:
        out = out + sum(fit(v) for v in d2d2.values()) / 90.0
        out = out - sum(fit(_d2(d2[i], i)) for i in range(3)) / 240.0
    return out


def kernel_table(kz, ky, kx, order):
    """K = R G_L on the octant [0, kz) x [0, ky) x [0, kx)."""
    r = 2 if order == 6 else 1
    G = lgf_table_mehrstellen(kz + r, ky + r, kx + r, order)
    K = apply_stencil(_mirror_full(G), "R", order)
    cz, cy, cx = K.shape[0] // 2, K.shape[1] // 2, K.shape[2] // 2
    return K[cz:cz + kz, cy:cy + ky, cx:cx + kx]


def green_spectrum_raw(M, order):
    """DFT of the evenly periodised K on the (Mz, My, Mx) torus, octant
    [0, M_i/2], as the DCT-I of the K octant (unscaled, as
    ``spectrum.green_spectrum_raw``)."""
    K = tuple(int(m) // 2 + 1 for m in M)
    return sfft.dctn(kernel_table(*K, order), type=1)


def solve(f, h, order, M=None):
    """u = h^2 K * f on the box by the zero-padded FFT convolution (no
    pruning; small grids)."""
    f = np.asarray(f, dtype=np.float64)
    N = f.shape
    M = tuple(2 * n for n in N) if M is None else tuple(int(m) for m in M)
    Gh = green_spectrum_raw(M, order)
    mir = [np.minimum(np.arange(m), m - np.arange(m)) for m in M]
    full = Gh[np.ix_(mir[0], mir[1], np.arange(M[2] // 2 + 1))]
    fh = np.fft.rfftn(f, s=M, axes=(0, 1, 2))
    u = np.fft.irfftn(fh * (float(h) ** 2 * full), s=M, axes=(0, 1, 2))
    return np.ascontiguousarray(u[: N[0], : N[1], : N[2]])
