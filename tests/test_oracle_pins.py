"""Pins of the CPU oracle against facts fixed by the paper and by mathematics,
independently of the oracle's own formulas (no GPU)."""
import os

import numpy as np
import pytest

import oracle
from oracle import analytic
from paper_2512_08555_amd import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


def _mirror_full(G):
    """Octant [0, K)^3 of an even function -> values on (-K, K)^3."""
    f = np.concatenate([G[:0:-1], G], 0)
    f = np.concatenate([f[:, :0:-1], f], 1)
    return np.concatenate([f[:, :, :0:-1], f], 2)


# --- lattice Green's function -------------------------------------------------

def test_g0_is_watson_closed_form():
    # G1[0] = -W/6, Watson's integral in Gamma-function closed form.
    g0 = oracle.lgf_table(1, 1, 1)[0, 0, 0]
    assert abs(g0 - oracle.watson_g0()) <= 2e-16
    assert abs(oracle.watson_g0() - (-0.252731009858663)) < 1e-15


@pytest.mark.parametrize("K", [9, 33])
def test_lgf_solves_lattice_poisson_with_delta(K):
    # Sec. 2.2: L G = delta with the 7-point stencil of eq. cross_discr2.
    G = _mirror_full(oracle.lgf_table(K, K, K))
    lap = oracle.laplacian7_interior(G, 1.0)
    c = lap.shape[0] // 2
    lap[c, c, c] -= 1.0
    assert np.abs(lap).max() < 1e-15


def test_lgf_noncubic_table_matches_cubic():
    G = oracle.lgf_table(9, 9, 9)
    Gn = oracle.lgf_table(5, 9, 7)
    # the quadrature split T depends on the table's extent: rounding-level change only
    assert np.abs(Gn - G[:5, :9, :7]).max() < 2e-16
    # symmetric under permutation of the axes
    assert np.abs(G - G.transpose(1, 0, 2)).max() < 1e-16
    assert np.abs(G - G.transpose(2, 1, 0)).max() < 1e-16


def test_lgf_far_field():
    # G1 -> -1/(4 pi r) [1 + (5 sum n^4/r^4 - 3)/(8 r^2)] + O(r^-5)
    pts = np.array([[60, 0, 0], [40, 40, 40], [100, 30, 7], [200, 200, 0], [400, 10, 300]])
    G = oracle.lgf_table(401, 401, 401)[pts[:, 2], pts[:, 1], pts[:, 0]]
    r = np.sqrt((pts.astype(float) ** 2).sum(1))
    resid = (G - oracle.lgf_far_field(pts)) * r ** 5
    assert np.all(np.abs(resid) < 0.1), resid
    # the leading term alone is off by O(r^-3): the correction is really there
    lead = -1.0 / (4 * np.pi * r)
    assert np.all(np.abs((G - lead) * r ** 3) > 1e-3)


def test_lgf_table_matches_golden_adaptive_points():
    path = os.path.join(HERE, "golden", "lgf_points.txt")
    rows = np.loadtxt(path)
    T = 40.0 * 512 ** 2
    for nx, ny, nz, val in rows:
        nx, ny, nz = int(nx), int(ny), int(nz)
        # the table code path on a small slab that contains the point
        tab = oracle.lgf_table(nz + 1, ny + 1, nx + 1, T=T)[nz, ny, nx]
        assert abs(tab - val) <= 4e-15 * abs(val), (nx, ny, nz, tab, val)


def test_tail_formula_against_quadrature_of_ive():
    from scipy import integrate, special
    T, T2 = 40.0 * 512 ** 2, 4e8
    for n in [(0, 0, 0), (512, 0, 0), (300, 200, 100)]:
        def f(s):
            t = np.exp(s)
            return t * special.ive(n[0], 2 * t) * special.ive(n[1], 2 * t) * special.ive(n[2], 2 * t)
        e = np.linspace(np.log(T), np.log(T2), 30)
        mid = sum(integrate.quad(f, a, b, epsabs=1e-300, epsrel=1e-14, limit=200)[0]
                  for a, b in zip(e[:-1], e[1:]))
        ref = mid + oracle.lgf_tail(n, T2)
        assert abs(oracle.lgf_tail(n, T) - ref) < 1e-19 + 1e-13 * abs(ref)


# --- Green's spectrum -----------------------------------------------------------

@pytest.mark.parametrize("M", [(16, 20, 24), (48, 48, 48), (8, 6, 10)])
def test_spectrum_dct_equals_rfft_of_periodisation(M):
    a = oracle.green_spectrum_raw(M)
    b = oracle.green_spectrum_rfft(M)
    assert np.abs(b.imag).max() < 1e-13 * np.abs(a).max()
    assert np.abs(a - b.real).max() < 1e-14 * np.abs(a).max()


def test_spectrum_negative_and_nyquist_limit():
    M = (48, 48, 48)
    a = oracle.green_spectrum_raw(M)
    assert np.all(a < 0)
    # at the Nyquist corner sigma(k) = 12, and the padded kernel's spectrum
    # approaches the infinite-lattice value -1/sigma as M grows
    assert abs(a[-1, -1, -1] + 1.0 / 12.0) < 1e-7
    # DFT identities: G_hat(0) = sum of the periodised kernel; mean of G_hat = Gp[0]
    iz = np.minimum(np.arange(48), 48 - np.arange(48))
    G1 = oracle.lgf_table(25, 25, 25)
    Gp = G1[np.ix_(iz, iz, iz)]
    assert abs(a[0, 0, 0] - Gp.sum()) < 1e-12 * abs(Gp.sum())
    full = a[np.ix_(iz, iz, iz)]
    assert abs(full.mean() - G1[0, 0, 0]) < 1e-14


# --- the solve ------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(8, 8, 8), (6, 10, 7), (5, 3, 9)])
def test_solve_equals_brute_force_lattice_sum(shape):
    rng = np.random.default_rng(11)
    f = rng.standard_normal(shape)
    h = 0.37
    ub = oracle.brute_force(f, h)
    us = oracle.solve(f, h)
    uf = oracle.solve_full(f, h)
    s = np.abs(ub).max()
    assert np.abs(us - ub).max() < 1e-14 * s * 10
    assert np.abs(uf - ub).max() < 1e-14 * s * 10


def test_solve_with_larger_padding_is_the_same():
    rng = np.random.default_rng(12)
    f = rng.standard_normal((6, 7, 5))
    u0 = oracle.solve(f, 0.5)
    u1 = oracle.solve(f, 0.5, M=(18, 14, 20))
    u2 = oracle.solve(f, 0.5, M=(10, 12, 8))     # M = 2N - 2, the smallest exact length
    assert np.abs(u0 - u1).max() < 1e-13 * np.abs(u0).max()
    assert np.abs(u0 - u2).max() < 1e-13 * np.abs(u0).max()
    with pytest.raises(ValueError):
        oracle.solve(f, 0.5, M=(10, 12, 6))


def test_solve_satisfies_discrete_poisson_inside_box():
    rng = np.random.default_rng(13)
    f = rng.standard_normal((20, 18, 22))
    h = 1.0 / 20
    u = oracle.solve(f, h)
    r = oracle.laplacian7_interior(u, h) - f[1:-1, 1:-1, 1:-1]
    assert np.abs(r).max() < 1e-11 * np.abs(f).max()


def test_delta_source_gives_scaled_lgf():
    N = 12
    f = np.zeros((N, N, N))
    c = (5, 3, 7)  # (z, y, x)
    f[c] = 1.0
    h = 0.25
    u = oracle.solve(f, h)
    G1 = oracle.lgf_table(N, N, N)
    i = np.arange(N)
    ref = h * h * G1[np.ix_(np.abs(i - c[0]), np.abs(i - c[1]), np.abs(i - c[2]))]
    assert np.abs(u - ref).max() < 1e-15


def test_translation_equivariance_and_linearity():
    rng = np.random.default_rng(14)
    N = 16
    f = np.zeros((N, N, N))
    f[3:9, 4:10, 2:8] = rng.standard_normal((6, 6, 6))
    g = np.roll(f, (2, 1, 3), axis=(0, 1, 2))
    uf = oracle.solve(f, 0.1)
    ug = oracle.solve(g, 0.1)
    assert np.abs(ug[2:, 1:, 3:] - uf[:-2, :-1, :-3]).max() < 1e-14 * np.abs(uf).max() * 10
    a, b = 1.7, -0.4
    uab = oracle.solve(a * f + b * g, 0.1)
    assert np.abs(uab - (a * uf + b * ug)).max() < 1e-14 * np.abs(uab).max() * 10


def test_adjoint_dot_product_and_transpose():
    rng = np.random.default_rng(15)
    f = rng.standard_normal((7, 6, 8))
    g = rng.standard_normal((7, 6, 8))
    h = 0.3
    lhs = np.vdot(oracle.solve(f, h), g)
    rhs = np.vdot(f, oracle.adjoint(g, h))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    assert np.abs(oracle.brute_force_adjoint(g, h) - oracle.adjoint(g, h)).max() < 1e-14 * 10


def test_paper_compact_solution_second_order():
    # Sec. 4.2: u_ref = u_unb(x) u_unb(y) u_unb(z) is the exact free-space
    # solution; the error of the second-order scheme falls as h^2 (Sec. 4).
    errs = []
    for N in (32, 64):
        h = 1.0 / N
        x = (np.arange(N) + 0.5) * h
        u = oracle.solve(analytic.bump_source(x, x, x), h)
        errs.append(np.abs(u - analytic.bump_solution(x, x, x)).max())
    order = np.log2(errs[0] / errs[1])
    assert 1.9 < order < 2.1, (errs, order)
    assert 1.0e-2 < errs[0] < 1.2e-2


def test_gaussian_closed_form_second_order():
    sig = 0.08
    c = (0.5, 0.5, 0.5)
    errs = []
    for N in (32, 64, 128):   # sigma = 2.6 cells at N = 32: in the asymptotic range
        h = 1.0 / N
        x = (np.arange(N) + 0.5) * h
        Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
        f = analytic.gaussian_source(X, Y, Z, c, sig, 1.0)
        uref = analytic.gaussian_potential(X, Y, Z, c, sig, 1.0)
        u = oracle.solve(f, h)
        errs.append(np.abs(u - uref).max() / np.abs(uref).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((orders > 1.85) & (orders < 2.15)), (errs, orders)
    # the computed potential is negative for a positive source (G < 0)
    assert u.max() < 0


def test_bump_second_derivative_matches_finite_difference():
    x = np.linspace(0.05, 0.95, 37)
    e = 1e-4
    fd = (analytic.bump_1d(x + e) - 2 * analytic.bump_1d(x) + analytic.bump_1d(x - e)) / e ** 2
    assert np.allclose(fd, analytic.bump_1d_dd(x), rtol=1e-5, atol=1e-6)


# --- synthetic inputs -------------------------------------------------------------

def test_workloads_are_seeded_and_shaped():
    a = workloads.config_c1()["f"]
    b = workloads.config_c1()["f"]
    assert a.shape == (32, 32, 32) and np.array_equal(a, b)
    f = workloads.blob_source((12, 10, 14), 0.1, seed=3, nblobs=4, sigma=(0.02, 0.1), noise=1e-3)
    assert f.shape == (12, 10, 14)
    s = workloads.batch_sizes()
    assert len(s) == 48 and all(32 <= v <= 192 for t in s for v in t)
    v = workloads.curl_source(16, 1 / 16, seed=1)
    assert v.shape == (3, 16, 16, 16)
    # a curl is divergence-free: central-difference divergence is small
    # relative to the field (second-order truncation only)
    h = 1 / 16
    div = ((v[0][1:-1, 1:-1, 2:] - v[0][1:-1, 1:-1, :-2]) + (v[1][1:-1, 2:, 1:-1] - v[1][1:-1, :-2, 1:-1])
           + (v[2][2:, 1:-1, 1:-1] - v[2][:-2, 1:-1, 1:-1])) / (2 * h)
    grad_scale = np.abs(v).max() / h
    assert np.abs(div).max() < 0.5 * grad_scale


def test_blob_sum_matches_direct_evaluation():
    shape = (5, 6, 7)
    h = 0.2
    c = np.array([[0.3, 0.5, 0.4], [0.8, 0.2, 0.6]])
    s = np.array([0.3, 0.5])
    a = np.array([1.5, -0.7])
    f = workloads.blob_sum(shape, h, c, s, a)
    z = (np.arange(5) + 0.5) * h
    y = (np.arange(6) + 0.5) * h
    x = (np.arange(7) + 0.5) * h
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    ref = sum(analytic.gaussian_source(X, Y, Z, c[b], s[b], a[b]) for b in range(2))
    assert np.abs(f - ref).max() < 1e-14
