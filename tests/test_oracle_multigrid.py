"""Pins of the oracle's multigrid cycle (oracle/multigrid.py; Sec. 3.1, Alg.
amg_vcycle) against facts fixed by the mathematics and the paper (no GPU),
and planted mistakes each of them must catch."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import analytic, mehrstellen, multigrid as mg


# --- the operators ---------------------------------------------------------------

def test_prolongation_is_exact_on_trilinear_functions():
    # trilinear interpolation reproduces every function a + b x + c y + d z
    # + e xy + f yz + g zx + k xyz (Sec. 3.1: block-wise trilinear)
    rng = np.random.default_rng(1)
    a = rng.standard_normal(8)

    def fun(z, y, x):
        return (a[0] + a[1] * x + a[2] * y + a[3] * z + a[4] * x * y + a[5] * y * z
                + a[6] * z * x + a[7] * x * y * z)
    mz, my, mx = 3, 4, 2
    cz, cy, cx = np.meshgrid(np.arange(mz + 1), np.arange(my + 1), np.arange(mx + 1), indexing="ij")
    fz, fy, fx = np.meshgrid(np.arange(2 * mz + 1) / 2, np.arange(2 * my + 1) / 2, np.arange(2 * mx + 1) / 2,
                             indexing="ij")
    assert np.abs(mg.prolong(fun(cz, cy, cx)) - fun(fz, fy, fx)).max() < 1e-13


def test_ghost_reconstruction_is_exact_on_cubics():
    # the 4-point rule (-1, 9, 9, -1)/16 reproduces cubics along each axis,
    # so its tensor product reproduces every product of cubics
    rng = np.random.default_rng(11)
    cz, cy, cx = rng.standard_normal((3, 4))

    def fun(z, y, x):
        return np.polyval(cz, z) * np.polyval(cy, y) * np.polyval(cx, x) + np.polyval(cx, z) * np.polyval(cz, x)
    m = (3, 2, 4)
    ext = [np.arange(-1, v + 2) for v in m]
    E = fun(*np.meshgrid(*ext, indexing="ij"))
    fine = [np.arange(2 * v + 1) / 2 for v in m]
    assert np.abs(mg.interp_cubic(E) - fun(*np.meshgrid(*fine, indexing="ij"))).max() < 1e-11
    # and the ghost layer takes those values, the unknowns are left alone
    u = np.zeros(tuple(2 * v + 1 for v in m))
    parent = np.zeros((8, 7, 9))
    c = (2, 2, 3)
    parent[1:1 + m[0] + 3, 1:1 + m[1] + 3, 2:2 + m[2] + 3] = E
    mg.fill_ghosts(u, parent, c, m)
    want = fun(*np.meshgrid(*fine, indexing="ij"))
    assert np.abs(u[0] - want[0]).max() < 1e-11 and np.abs(u[:, :, -1] - want[:, :, -1]).max() < 1e-11
    assert not u[1:-1, 1:-1, 1:-1].any()


def _prolongation_matrix(m):
    n = int(np.prod([v + 1 for v in m]))
    cols = []
    for t in range(n):
        e = np.zeros(n)
        e[t] = 1.0
        cols.append(mg.prolong(e.reshape(tuple(v + 1 for v in m))).ravel())
    return np.array(cols).T                     # fine x coarse


def test_full_weighting_is_the_scaled_transpose_of_the_prolongation():
    # the tensor product of (1/4)[1 2 1] equals P^T / 2^3 at the interior
    # coarse nodes (the variational pair of the textbook two-grid method)
    m = (3, 4, 3)
    P = _prolongation_matrix(m)
    rng = np.random.default_rng(2)
    r = rng.standard_normal(tuple(2 * v + 1 for v in m))
    fw = mg.restrict_full_weighting(r)
    full = (P.T @ r.ravel() / 8.0).reshape(tuple(v + 1 for v in m))
    assert np.abs(fw - full[1:-1, 1:-1, 1:-1]).max() < 1e-14
    # weights sum to one; a quadratic x^2 gains h^2/2 per axis (h = 1 fine)
    assert abs(mg.restrict_full_weighting(np.ones((7, 7, 7))).max() - 1.0) < 1e-15
    x = np.arange(7, dtype=float)
    q = np.broadcast_to(x[None, None, :] ** 2, (7, 7, 7))
    assert np.allclose(mg.restrict_full_weighting(q)[0, 0, :], x[2:-2:2] ** 2 + 0.5)


def test_laplacian_is_exact_on_quadratics():
    z, y, x = np.meshgrid(*(np.arange(6) * 0.3,) * 3, indexing="ij")
    u = x ** 2 + 2 * y ** 2 - 0.5 * z ** 2 + x * y - z
    assert np.abs(mg.laplacian(u, 0.3) - 5.0).max() < 1e-12


def test_smoothing_is_red_black_gauss_seidel():
    # against plain loops: every red unknown (even index sum), then every
    # black one, set to the value that zeroes its own residual
    rng = np.random.default_rng(3)
    u = rng.standard_normal((5, 6, 7))
    f = rng.standard_normal(u.shape)
    h = 0.25
    ref = u.copy()
    for color in (0, 1):
        for i, j, k in itertools.product(range(1, 4), range(1, 5), range(1, 6)):
            if (i + j + k) % 2 != color:
                continue
            nb = (ref[i + 1, j, k] + ref[i - 1, j, k] + ref[i, j + 1, k] + ref[i, j - 1, k]
                  + ref[i, j, k + 1] + ref[i, j, k - 1])
            ref[i, j, k] = (nb - h * h * f[i, j, k]) / 6.0
    out = mg.smooth(u.copy(), f, h)
    assert np.abs(out - ref).max() < 1e-15
    # the ghost layer is not touched
    assert np.array_equal(out[0], u[0]) and np.array_equal(out[:, :, -1], u[:, :, -1])


def test_hierarchy_validation():
    assert mg.level_shapes((10, 10, 10), [((1, 2, 3), (4, 4, 5))])[1] == (9, 9, 11)
    for bad in [((0, 2, 2), (4, 4, 4)), ((2, 2, 2), (7, 4, 4)), ((2, 2, 2), (1, 4, 4))]:
        with pytest.raises(ValueError):
            mg.level_shapes((10, 10, 10), [bad])


# --- the cycle --------------------------------------------------------------------

N0, H0 = (12, 11, 13), 0.1
PATCH = ((3, 2, 4), (4, 5, 4))


def _random_sources(n0, patches, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(s) for s in mg.level_shapes(n0, patches)]


def test_without_refinement_a_cycle_is_the_direct_solve():
    f = _random_sources(N0, [], 4)
    u = mg.solve(f, [], H0, 1)
    assert np.abs(u[0] - oracle.solve(f[0], H0)).max() < 1e-15
    assert np.abs(mg.laplacian(u[0], H0) - f[0][1:-1, 1:-1, 1:-1]).max() < 1e-11


def test_fixed_point_is_the_composite_solution():
    # the cycle converges to the solution of the composite equations,
    # assembled and solved directly (no smoothing, no transfers of the cycle)
    fs = _random_sources(N0, [PATCH], 5)
    u0, u1 = mg.composite_dense(fs, PATCH, H0)
    us = mg.solve(fs, [PATCH], H0, 14)
    scale = np.abs(u1).max()
    assert np.abs(us[0] - u0).max() < 1e-11 * scale
    assert np.abs(us[1] - u1).max() < 1e-11 * scale


def test_composite_equations_hold_at_convergence_on_three_levels():
    patches = [((3, 3, 3), (6, 5, 7)), ((2, 2, 3), (6, 6, 5))]
    fs = _random_sources((13, 12, 14), patches, 6)
    us = mg.solve(fs, patches, H0, 16)
    res = mg.composite_residuals(us, fs, patches, H0)
    assert max(res) < 1e-10 * max(np.abs(f).max() for f in fs)
    for k, (c, m) in enumerate(patches):      # injection consistency
        inner = tuple(slice(ci + 1, ci + mi) for ci, mi in zip(c, m))
        assert np.abs(us[k][inner] - us[k + 1][2:-2:2, 2:-2:2, 2:-2:2]).max() < 1e-14 * np.abs(us[k]).max()


def _rates(n, cycles, nu=(2, 2)):
    h0 = 1.0 / n
    patch = ((n // 4,) * 3, (n // 2,) * 3)
    fs = _random_sources((n + 1,) * 3, [patch], 7)
    us = [np.zeros(s) for s in mg.level_shapes((n + 1,) * 3, [patch])]
    res = []
    for _ in range(cycles):
        mg.vcycle(us, fs, [patch], h0, *nu)
        res.append(max(mg.composite_residuals([u.copy() for u in us], fs, [patch], h0)))
    return np.array(res[1:]) / np.array(res[:-1])


def test_contraction_is_independent_of_the_spacing():
    # the defining property of a multigrid cycle: a residual reduction per
    # cycle bounded away from 1 independently of h
    r16, r32 = _rates(16, 7)[-3:].max(), _rates(32, 7)[-3:].max()
    assert r16 < 0.1 and r32 < 0.1 and abs(np.log(r32 / r16)) < np.log(1.6)
    assert _rates(16, 7, (1, 1))[-3:].max() < 0.25


def _gaussian_levels(n, boxes):
    h0 = 1.0 / n
    patches = [((n // 4,) * 3, (n // 2,) * 3)] * boxes
    shapes = mg.level_shapes((n + 1,) * 3, patches)
    fs, ref = [], []
    o, h = 0.0, h0
    for k, s in enumerate(shapes):
        a = o + np.arange(s[0]) * h
        Z, Y, X = np.meshgrid(a, a, a, indexing="ij")
        fs.append(analytic.gaussian_source(X, Y, Z, (0.5, 0.5, 0.5), 0.1, 1.0))
        ref.append(analytic.gaussian_potential(X, Y, Z, (0.5, 0.5, 0.5), 0.1, 1.0))
        o, h = o + (n // 4) * h, h / 2
    return fs, ref, patches, h0


@pytest.mark.parametrize("boxes", [1, 2])
def test_second_order_on_a_gaussian(boxes):
    # the composite solution of nested boxes around a Gaussian charge (the
    # closed-form erf potential) converges at second order in h0
    errs = []
    for n in (16, 32):
        fs, ref, patches, h0 = _gaussian_levels(n, boxes)
        us = mg.solve(fs, patches, h0, 10)
        errs.append(max(np.abs(u - r).max() for u, r in zip(us, ref)) / np.abs(ref[0]).max())
    p = np.log2(errs[0] / errs[1])
    assert 1.9 < p < 2.4, (errs, p)


def test_second_order_on_the_paper_bump():
    # Sec. 4 manufactured solution, level 0 on [0, 1]^3 and a box on
    # [1/4, 3/4]^3: the composite error falls as h^2
    errs = []
    for n in (32, 64):
        h0 = 1.0 / n
        patches = [((n // 4,) * 3, (n // 2,) * 3)]
        axes = [np.arange(n + 1) * h0, 0.25 + np.arange(n + 1) * (h0 / 2)]
        fs = [analytic.bump_source(a, a, a) for a in axes]
        us = mg.solve(fs, patches, h0, 10)
        errs.append(max(np.abs(u - analytic.bump_solution(a, a, a)).max() for u, a in zip(us, axes)))
    p = np.log2(errs[0] / errs[1])
    assert 1.8 < p < 2.2 and errs[1] < 1.5e-3, (errs, p)


def test_incompatible_kernel_does_not_converge():
    # Sec. 3.3: the coarse kernel must be the LGF of the cycle's operator;
    # the Mehrstellen kernel (the LGF of another stencil) leaves the
    # composite residual at the level of the first cycle
    fs = _random_sources(N0, [PATCH], 8)
    good = mg.solve(fs, [PATCH], H0, 8)
    bad = mg.solve(fs, [PATCH], H0, 8, coarse_solve=lambda f, h: mehrstellen.solve(f, h, 4))
    rg = max(mg.composite_residuals(good, fs, [PATCH], H0))
    rb = max(mg.composite_residuals(bad, fs, [PATCH], H0))
    assert rg < 1e-8 and rb > 1e-2, (rg, rb)


# --- planted mistakes -------------------------------------------------------------------

def _bad_prolong(e):
    out = np.asarray(e, dtype=float)
    for a in range(3):                # piecewise constant instead of linear
        out = np.repeat(out, 2, axis=a)
        s = [slice(None)] * 3
        s[a] = slice(0, -1)
        out = out[tuple(s)]
    return out


def _jacobi(u, f, h):
    inner = (slice(1, -1),) * 3
    nb = (u[2:, 1:-1, 1:-1] + u[:-2, 1:-1, 1:-1] + u[1:-1, 2:, 1:-1] + u[1:-1, :-2, 1:-1]
          + u[1:-1, 1:-1, 2:] + u[1:-1, 1:-1, :-2])
    u[inner] = (nb - h * h * f[inner]) / 6.0
    return u


_REAL = {k: getattr(mg, k) for k in ("correction", "inject", "restrict_full_weighting", "prolong",
                                      "smooth", "laplacian", "interp_cubic")}

PLANTS = {
    # the correction taken as stored minus new, as the algorithm prints it
    "correction_sign": ("correction", lambda a, b: b - a),
    # the solution restricted by full weighting instead of injection
    "u_full_weighting": ("inject", lambda u: _REAL["restrict_full_weighting"](u)),
    # full weighting whose weights do not sum to one
    "fw_weights": ("restrict_full_weighting", lambda r: 1.3 * _REAL["restrict_full_weighting"](r)),
    # piecewise-constant prolongation of the correction
    "prolong_constant": ("prolong", _bad_prolong),
    # ghost layers by trilinear interpolation instead of the cubic rule
    "ghost_trilinear": ("interp_cubic", lambda E: _REAL["prolong"](np.asarray(E)[1:-1, 1:-1, 1:-1])),
    # Jacobi sweeps instead of Gauss-Seidel
    "jacobi": ("smooth", _jacobi),
    # the Laplacian with the wrong sign
    "laplacian_sign": ("laplacian", lambda u, h: -_REAL["laplacian"](u, h)),
}


@pytest.mark.parametrize("name", sorted(PLANTS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, val = PLANTS[name]
    monkeypatch.setattr(mg, attr, val)
    caught = 0
    for pin in (test_fixed_point_is_the_composite_solution, test_contraction_is_independent_of_the_spacing,
                lambda: test_second_order_on_a_gaussian(1)):
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught > 0, name
