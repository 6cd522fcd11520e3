"""Pins of the oracle's mixed-boundary solve (oracle/bc.py) against facts
fixed by the mathematics and by the paper, independently of its own
formulas (no GPU)."""
import itertools
from math import pi

import numpy as np
import pytest

import oracle
from oracle import analytic, bc as obc

EULER_GAMMA = 0.57721566490153286061


def _mirror2(G):
    f = np.concatenate([G[:0:-1], G], 0)
    return np.concatenate([f[:, :0:-1], f], 1)


# --- the two-dimensional LGF ----------------------------------------------------

def test_lgf2d_nearest_values_are_textbook():
    # With G[0,0] = 0, L G = delta at the origin and the square symmetry give
    # G[1,0] = 1/4; G[1,1] = 1/pi is the classical value of the square
    # lattice (the random walk's potential kernel a(1,1) = 4/pi, G = a/4).
    G = obc.lgf2d_table(4, 4)
    assert G[0, 0] == 0.0 or abs(G[0, 0]) < 1e-17
    assert abs(G[1, 0] - 0.25) < 2e-15
    assert abs(G[0, 1] - 0.25) < 2e-15
    assert abs(G[1, 1] - 1.0 / pi) < 2e-15


@pytest.mark.parametrize("K", [9, 40])
def test_lgf2d_solves_lattice_poisson_with_delta(K):
    G = _mirror2(obc.lgf2d_table(K, K))
    lap = G[2:, 1:-1] + G[:-2, 1:-1] + G[1:-1, 2:] + G[1:-1, :-2] - 4.0 * G[1:-1, 1:-1]
    c = lap.shape[0] // 2
    lap[c, c] -= 1.0
    assert np.abs(lap).max() < 2e-14


def test_lgf2d_far_field():
    # G -> (1/2pi) (ln r + gamma + (3/2) ln 2) + O(r^-2)
    G = obc.lgf2d_table(121, 121)
    pts = np.array([[30, 0], [20, 20], [60, 17], [100, 90], [120, 3]])
    r = np.sqrt((pts.astype(float) ** 2).sum(1))
    lead = (np.log(r) + EULER_GAMMA + 1.5 * np.log(2.0)) / (2 * pi)
    g = G[pts[:, 0], pts[:, 1]]
    assert np.all(np.abs((g - lead) * r ** 2) < 0.05)
    # the constant is really there
    assert np.all(np.abs(g - np.log(r) / (2 * pi)) > 0.25)


# --- the screened one-dimensional LGF ---------------------------------------------

@pytest.mark.parametrize("s", [1e-6, 0.01, 0.3, 2.0, 11.5])
def test_lgf1d_screened_solves_its_equation(s):
    n = np.arange(-30, 31)
    G = obc.lgf1d_screened(n, s)
    res = G[2:] - 2 * G[1:-1] + G[:-2] - s * G[1:-1]
    d = np.zeros_like(res)
    d[29] = 1.0
    assert np.abs(res - d).max() < 1e-12 * max(1.0, 1.0 / np.sqrt(s))
    assert np.all(np.diff(np.abs(G[30:])) <= 0)   # decays away from the source


def test_lgf1d_screened_tends_to_the_1d_lgf():
    # G(n; s) - G(0; s) -> |n|/2 as s -> 0, and s = 0 is |n|/2 itself
    n = np.arange(0, 12)
    for s in (1e-8, 1e-10):
        g = obc.lgf1d_screened(n, s)
        assert np.abs((g - g[0]) - 0.5 * n).max() < 20 * np.sqrt(s) * n.max() ** 2
    assert np.array_equal(obc.lgf1d_screened(n, 0.0), 0.5 * n)


# --- the solve against a dense solve of the boundary-value problem -----------------

def _dense_operator(shape, bc):
    """The 7-point operator with the boundary rules as a dense matrix."""
    Nz, Ny, Nx = shape
    n = Nz * Ny * Nx
    A = np.zeros((n, n))
    idx = np.arange(n).reshape(shape)
    for z, y, x in itertools.product(range(Nz), range(Ny), range(Nx)):
        i = idx[z, y, x]
        A[i, i] -= 6.0
        for ax, d in itertools.product(range(3), (-1, 1)):
            p = [z, y, x]
            p[ax] += d
            N = shape[ax]
            sgn = 1.0
            if p[ax] < 0 or p[ax] >= N:
                b = bc[ax]
                if b == "per":
                    p[ax] %= N
                elif b == "even":
                    p[ax] = 0 if p[ax] < 0 else N - 1
                else:
                    p[ax] = 0 if p[ax] < 0 else N - 1
                    sgn = -1.0
            A[i, idx[tuple(p)]] += sgn
    return A


SPECTRAL = list(itertools.product(("per", "even", "odd"), repeat=3))


@pytest.mark.parametrize("bc", SPECTRAL)
def test_spectral_solve_equals_dense_solve(bc):
    shape = (4, 5, 3)
    h = 0.25
    rng = np.random.default_rng(hash(bc) % 1000)
    f = rng.standard_normal(shape)
    singular = "odd" not in bc
    if singular:
        f -= f.mean()
    u = obc.solve_bc(f, h, bc)
    A = _dense_operator(shape, bc) / h ** 2
    ref = np.linalg.lstsq(A, f.ravel(), rcond=None)[0].reshape(shape)
    if singular:
        ref -= ref.mean()
        assert abs(u.mean()) < 1e-14
    assert np.abs(u - ref).max() < 1e-12 * np.abs(ref).max()


# --- mixed unbounded / spectral directions ----------------------------------------

MIXED = [b for b in itertools.product(obc.BCS, repeat=3) if 0 < sum(x == "unb" for x in b) < 3]


@pytest.mark.parametrize("bc", MIXED)
def test_mixed_solve_satisfies_the_discrete_equation(bc):
    shape = (9, 8, 10)
    h = 1.0 / 10
    rng = np.random.default_rng(7)
    f = rng.standard_normal(shape)
    u = obc.solve_bc(f, h, bc)
    lap = obc.laplacian_bc(u, h, bc)
    inner = f[obc.interior_cells(shape, bc)]
    assert np.abs(lap - inner).max() < 1e-11 * np.abs(f).max()


def test_all_unbounded_is_the_free_space_solve():
    rng = np.random.default_rng(3)
    f = rng.standard_normal((6, 7, 5))
    a = obc.solve_bc(f, 0.1, ("unb",) * 3)
    b = oracle.solve(f, 0.1)
    assert np.abs(a - b).max() < 1e-15 * 100 * np.abs(b).max()


@pytest.mark.parametrize("c", ["per", "even"])
def test_two_unbounded_z_independent_source_is_the_2d_lattice_sum(c):
    # f(x, y, z) = g(x, y): only the zero wavenumber of z is present, and the
    # solution is h^2 sum_j G2[i - j] g[j], the 2-D LGF sum written out
    shape = (6, 7, 5)
    h = 0.2
    rng = np.random.default_rng(11)
    g = rng.standard_normal(shape[1:])
    f = np.broadcast_to(g, shape).copy()
    u = obc.solve_bc(f, h, (c, "unb", "unb"))
    G2 = obc.lgf2d_table(shape[1], shape[2])
    ref = np.zeros(shape[1:])
    for i0, i1 in itertools.product(range(shape[1]), range(shape[2])):
        for j0, j1 in itertools.product(range(shape[1]), range(shape[2])):
            ref[i0, i1] += G2[abs(i0 - j0), abs(i1 - j1)] * g[j0, j1]
    ref *= h * h
    assert np.abs(u - ref[None]).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("tb", [("per", "per"), ("even", "per"), ("even", "even")])
def test_one_unbounded_transverse_constant_is_the_1d_lattice_sum(tb):
    # f depends on the unbounded axis only: u = h^2 sum_j |i - j|/2 g[j]
    shape = (9, 4, 6)
    h = 0.3
    rng = np.random.default_rng(5)
    g = rng.standard_normal(shape[0])
    f = np.broadcast_to(g[:, None, None], shape).copy()
    u = obc.solve_bc(f, h, ("unb",) + tb)
    i = np.arange(shape[0])
    ref = h * h * (0.5 * np.abs(i[:, None] - i[None, :])) @ g
    assert np.abs(u - ref[:, None, None]).max() < 1e-13 * np.abs(ref).max()


def test_periodic_direction_translation():
    # periodic in z: shifting the source cyclically along z shifts u
    rng = np.random.default_rng(9)
    f = rng.standard_normal((8, 6, 7))
    bc = ("per", "unb", "unb")
    u = obc.solve_bc(f, 0.1, bc)
    v = obc.solve_bc(np.roll(f, 3, axis=0), 0.1, bc)
    assert np.abs(np.roll(u, 3, axis=0) - v).max() < 1e-13 * np.abs(u).max()


# --- second order against the paper's manufactured solutions (Sec. 4.2) ------------

def _uper(x):
    return np.exp(np.sin(2 * pi * x)) - 1.0


def _uper_dd(x):
    s, c = np.sin(2 * pi * x), np.cos(2 * pi * x)
    return (2 * pi) ** 2 * (c * c - s) * np.exp(s)


def _factor(kind):
    if kind == "unb":
        return analytic.bump_1d, analytic.bump_1d_dd
    if kind == "per":
        return _uper, _uper_dd
    if kind == "even":     # zero slope at the faces x = 0, 1
        return (lambda x: np.cos(2 * pi * x) + 0.5 * np.cos(4 * pi * x),
                lambda x: -(2 * pi) ** 2 * np.cos(2 * pi * x) - 0.5 * (4 * pi) ** 2 * np.cos(4 * pi * x))
    return (lambda x: np.sin(pi * x) + 0.3 * np.sin(3 * pi * x),   # odd: zero at the faces
            lambda x: -pi ** 2 * np.sin(pi * x) - 0.3 * (3 * pi) ** 2 * np.sin(3 * pi * x))


def _manufactured(bc, n):
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    fac = [_factor(b) for b in bc]
    u = [fa[0](x) for fa in fac]
    d = [fa[1](x) for fa in fac]
    U = u[0][:, None, None] * u[1][None, :, None] * u[2][None, None, :]
    F = (d[0][:, None, None] * u[1][None, :, None] * u[2][None, None, :]
         + u[0][:, None, None] * d[1][None, :, None] * u[2][None, None, :]
         + u[0][:, None, None] * u[1][None, :, None] * d[2][None, None, :])
    return h, U, F


@pytest.mark.parametrize("bc", [("per", "unb", "unb"), ("unb", "per", "per"), ("per", "per", "per"),
                                ("even", "unb", "odd"), ("odd", "even", "per")])
def test_second_order_convergence(bc):
    errs = []
    for n in (16, 32, 64):
        h, U, F = _manufactured(bc, n)
        u = obc.solve_bc(F, h, bc)
        if "unb" not in bc and "odd" not in bc:
            u = u - u.mean()
            U = U - U.mean()
        errs.append(np.abs(u - U).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    # measured 1.86-1.90 from 16 to 32 (pre-asymptotic), 1.97 from 32 to 64
    assert orders[0] > 1.8 and 1.93 < orders[1] < 2.07, (errs, orders)


def test_vortex_tube_second_order():
    # the paper's Biot-Savart benchmark (Sec. 5): unbounded in x and y,
    # periodic in z; the discrete velocity converges to the closed form
    from paper_2512_08555_amd import workloads
    errs = []
    for n in (32, 64, 128):
        f = workloads.vortex_tube_source(n, nz=4)
        ref = analytic.vortex_tube_velocity(n, nz=4)
        u = np.stack([obc.solve_bc(f[c], 1.0 / n, ("per", "unb", "unb")) for c in range(2)])
        errs.append(np.abs(u - ref[:2]).max() / np.abs(ref[:2]).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    # measured 7.4e-3, 1.6e-3, 3.7e-4: orders 2.23, 2.09 (approaching 2)
    assert 1.95 < orders[-1] < 2.2, (errs, orders)
    assert errs[-1] < 5e-4
