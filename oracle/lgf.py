r"""Lattice Green's function (LGF) of the 7-point Laplacian -- ORACLE, test
infrastructure only (see ``oracle/__init__.py``).

Definition followed (Sec. 2.2, the LGF paragraph): G1 is the solution of
L G1[n] = delta[n] on the infinite unit lattice Z^3, decaying at infinity
(Sec. 2.2, unbounded directions), where L is the second-order cross stencil
of eq. cross_discr2 with h = 1:

    (L u)[n] = sum_i (u[n + e_i] - 2 u[n] + u[n - e_i]).

Fourier integral.  The symbol of L is -sigma(k), sigma(k) = sum_i (2 - 2 cos k_i),
so G1[n] = -(2 pi)^-3 \int e^{i k.n} / sigma(k) dk.  Writing
1/sigma = \int_0^inf e^{-sigma t} dt and using the Bessel generating integral
(1/2pi) \int e^{i k n} e^{2 t cos k} dk = I_n(2t) gives the separable form

    G1[n] = - \int_0^inf  prod_i  e^{-2t} I_{n_i}(2t)  dt.

Evaluation (the reading of the paper's unstated LGF construction):
  * [0, T]: composite Gauss-Legendre in s = ln t, panels of width 1 with 16
    nodes each, on s in [-40, ln T] (the last panel ends exactly at ln T);
    e^{-2t} I_n(2t) is scipy.special.ive(n, 2t).
  * [T, inf): the large-argument (Hankel) expansion
    e^{-x} I_nu(x) ~ (2 pi x)^{-1/2} sum_k (-1)^k a_k(nu) x^{-k},
    a_k(nu) = prod_{m=1..k} (4 nu^2 - (2m-1)^2) / (k! 8^k)
    (Abramowitz & Stegun 9.7.1), multiplied out over the three axes and
    integrated term by term:  \int_T^inf (4 pi t)^{-3/2} (2t)^{-m} dt
    = (4 pi)^{-3/2} 2^{-m} T^{-1/2-m} / (m + 1/2).
    T = max(400, 40 n_max^2) keeps every term ratio below ~1/160.
"""

from math import factorial, gamma, pi, sqrt

import numpy as np
from scipy import integrate, special

S_LO = -40.0          # lower end of the s = ln t range; e^{-40} ~ 4e-18
PANEL_WIDTH = 1.0
PANEL_ORDER = 16
TAIL_TERMS = 6        # Hankel terms kept in the product series


def watson_g0():
    """G1[0,0,0] = -W/6 with Watson's simple-cubic integral
    W = (sqrt 6 / (32 pi^3)) Gamma(1/24) Gamma(5/24) Gamma(7/24) Gamma(11/24)
    (Glasser & Zucker's closed form of Watson's integral).  Independent of
    every routine below; used to pin them."""
    w = sqrt(6.0) / (32.0 * pi ** 3) * gamma(1 / 24) * gamma(5 / 24) * gamma(7 / 24) * gamma(11 / 24)
    return -w / 6.0


def default_T(n_max):
    return max(400.0, 40.0 * float(n_max) ** 2)


def quadrature_nodes(T):
    """Nodes t_j and weights w_j (including the Jacobian dt = t ds) of the
    composite Gauss-Legendre rule on s = ln t in [S_LO, ln T]."""
    s_hi = np.log(T)
    npan = int(np.ceil((s_hi - S_LO) / PANEL_WIDTH))
    edges = np.linspace(S_LO, s_hi, npan + 1)
    x, w = np.polynomial.legendre.leggauss(PANEL_ORDER)
    half = 0.5 * (edges[1:] - edges[:-1])
    mid = 0.5 * (edges[1:] + edges[:-1])
    s = (mid[:, None] + half[:, None] * x[None, :]).ravel()
    ws = (half[:, None] * w[None, :]).ravel()
    t = np.exp(s)
    return t, ws * t


def hankel_coefficients(nu, K=TAIL_TERMS):
    """c_k(nu) = (-1)^k a_k(nu), k = 0..K, of e^{-x} I_nu(x) ~ (2 pi x)^{-1/2}
    sum_k c_k x^{-k}.  ``nu`` may be an integer array; returns (K+1, len(nu))."""
    nu = np.atleast_1d(np.asarray(nu, dtype=np.float64))
    mu = 4.0 * nu * nu
    out = np.empty((K + 1, nu.size))
    prod = np.ones_like(nu)
    out[0] = 1.0
    for k in range(1, K + 1):
        prod = prod * (mu - (2 * k - 1) ** 2)
        out[k] = (-1) ** k * prod / (factorial(k) * 8.0 ** k)
    return out


def _tail_moment(m, T):
    # \int_T^inf (4 pi t)^{-3/2} (2t)^{-m} dt
    return (4.0 * pi) ** -1.5 * 2.0 ** (-m) * T ** (-0.5 - m) / (m + 0.5)


def lgf_tail(n, T, K=TAIL_TERMS):
    """\\int_T^inf prod_i e^{-2t} I_{n_i}(2t) dt for one lattice point n (3-tuple),
    by the term-by-term integral of the product Hankel series (total degree <= K)."""
    c = [hankel_coefficients(ni, K)[:, 0] for ni in n]
    tot = 0.0
    for a in range(K + 1):
        for b in range(K + 1 - a):
            for d in range(K + 1 - a - b):
                tot += c[0][a] * c[1][b] * c[2][d] * _tail_moment(a + b + d, T)
    return tot


def lgf_table(kz, ky, kx, T=None):
    """G1[nz, ny, nx] for 0 <= nz < kz, 0 <= ny < ky, 0 <= nx < kx (float64).

    G1 is even in every index, so this octant holds the whole function on
    the box  |n_i| < k_i.  The separable quadrature sum is a product of three
    per-axis tables B_i[n, j] = ive(n, 2 t_j), contracted over j one
    nz-slab at a time; the tail is the same triple Hankel sum as
    ``lgf_tail`` with its inner two sums grouped per (a, nz)."""
    kz, ky, kx = int(kz), int(ky), int(kx)
    n_max = max(kz, ky, kx) - 1
    T = default_T(n_max) if T is None else float(T)
    t, w = quadrature_nodes(T)
    Bz = special.ive(np.arange(kz)[:, None], 2.0 * t[None, :])
    By = special.ive(np.arange(ky)[:, None], 2.0 * t[None, :])
    Bx = special.ive(np.arange(kx)[:, None], 2.0 * t[None, :])
    K = TAIL_TERMS
    cz = hankel_coefficients(np.arange(kz), K)
    cy = hankel_coefficients(np.arange(ky), K)
    cx = hankel_coefficients(np.arange(kx), K)
    g = np.array([_tail_moment(m, T) for m in range(K + 1)])
    # tail[nz,ny,nx] = sum_{a+b+d<=K} cz[a,nz] cy[b,ny] cx[d,nx] g[a+b+d]
    E = np.zeros((K + 1, ky, kx))
    for a in range(K + 1):
        for b in range(K + 1 - a):
            dx = sum(cx[d] * g[a + b + d] for d in range(K + 1 - a - b))
            E[a] += np.outer(cy[b], dx)
    G = np.empty((kz, ky, kx))
    ByT = By
    BxT = Bx.T.copy()
    for iz in range(kz):
        quad = (ByT * (w * Bz[iz])[None, :]) @ BxT
        tail = np.tensordot(cz[:, iz], E, axes=(0, 0))
        G[iz] = -(quad + tail)
    return G


def lgf_point_adaptive(n, T=None):
    """G1[n] for one point by adaptive quadrature (scipy.integrate.quad) of
    the same Bessel integral on [0, T] in s = ln t (subintervals of width 2),
    plus ``lgf_tail``.  Slow; an independent check of the panel rule."""
    n = tuple(int(abs(v)) for v in n)
    T = default_T(max(max(n), 1)) if T is None else float(T)

    def integrand(s):
        t = np.exp(s)
        return t * special.ive(n[0], 2 * t) * special.ive(n[1], 2 * t) * special.ive(n[2], 2 * t)

    edges = list(np.arange(S_LO, np.log(T), 2.0)) + [np.log(T)]
    tot = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        if b <= a:
            continue
        v, _ = integrate.quad(integrand, a, b, epsabs=1e-300, epsrel=1e-14, limit=200)
        tot += v
    return -(tot + lgf_tail(n, T))


def lgf_far_field(n):
    """Two-term far-field expansion of G1 (the continuous -1/(4 pi r) plus the
    lattice correction): -(1/(4 pi r)) [1 + (5 sum n_i^4 / r^4 - 3) / (8 r^2)].
    The remainder is O(r^-5)."""
    n = np.asarray(n, dtype=np.float64)
    r = np.sqrt(np.sum(n * n, axis=-1))
    q = np.sum(n ** 4, axis=-1) / r ** 4
    return -(1.0 / (4.0 * pi * r)) * (1.0 + (5.0 * q - 3.0) / (8.0 * r * r))
