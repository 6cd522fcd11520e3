"""Pins of the oracle's Mehrstellen kernels (oracle/mehrstellen.py) against
facts fixed by the paper and the mathematics (no GPU), and planted
mistakes each of them must catch."""
import numpy as np
import pytest

import oracle
from oracle import analytic, mehrstellen as ms


# --- the stencils ---------------------------------------------------------------

@pytest.mark.parametrize("order", [4, 6])
def test_symbol_ratio_has_the_stated_order(order):
    # sigma / rho = |k|^2 + O(|k|^(order + 2)): the pair is consistent to the
    # order eqs. mehrstellen_discr4/6 state (this also fixes the reading of
    # the misprinted term of R6)
    ratios = []
    for kk in (0.1, 0.05, 0.025):
        k = np.array([kk, 0.7 * kk, 0.3 * kk])
        sig, rho = ms.symbols(4.0 * np.sin(0.5 * k) ** 2, order)
        k2 = float((k ** 2).sum())
        ratios.append((sig / rho - k2) / k2 ** (order / 2 + 1))
    assert abs(ratios[0]) > 1e-6
    assert abs(ratios[2] / ratios[1] - 1.0) < 0.01 and abs(ratios[1] / ratios[0] - 1.0) < 0.03


def test_stencil_coefficients():
    # L4: centre -24/6, faces 2/6, edges 1/6 (the 19-point stencil); L6:
    # centre -128/30, faces 14/30, edges 3/30, corners 1/30 (27 points);
    # R4: centre 1/2, faces 1/12
    d = np.zeros((5, 5, 5))
    d[2, 2, 2] = 1.0
    L4 = ms.apply_stencil(d, "L", 4)
    assert np.allclose([L4[1, 1, 1], L4[0, 1, 1], L4[0, 0, 1], L4[0, 0, 0]], [-4.0, 1 / 3, 1 / 6, 0.0])
    L6 = ms.apply_stencil(d, "L", 6)
    assert np.allclose([L6[1, 1, 1], L6[0, 1, 1], L6[0, 0, 1], L6[0, 0, 0]],
                       [-128 / 30, 14 / 30, 3 / 30, 1 / 30])
    R4 = ms.apply_stencil(d, "R", 4)
    assert np.allclose([R4[1, 1, 1], R4[0, 1, 1], R4[0, 0, 1]], [0.5, 1 / 12, 0.0])
    one = np.ones((5, 5, 5))
    for kind, order, val in (("R", 4, 1.0), ("R", 6, 1.0), ("L", 4, 0.0), ("L", 6, 0.0)):
        assert abs(ms.apply_stencil(one, kind, order).max() - val) < 1e-15   # rho(0) = 1, sigma(0) = 0


# --- the lattice Green's functions ----------------------------------------------------

@pytest.mark.parametrize("order", [4, 6])
def test_lgf_solves_the_mehrstellen_equation(order):
    # L G_L = delta (Sec. 3.3: the kernel is the LGF of the operator)
    G = ms.lgf_table_mehrstellen(10, 10, 10, order)
    L = ms.apply_stencil(ms._mirror_full(G), "L", order)
    c = L.shape[0] // 2
    L[c, c, c] -= 1.0
    assert np.abs(L).max() < 1e-15


@pytest.mark.parametrize("order", [4, 6])
def test_lgf_far_field(order):
    # G_L -> -1/(4 pi r): the difference to the 7-point LGF decays as r^-3
    K = 41
    D = ms.lgf_difference(K, K, 1, order)[:, :, 0]
    pts = [(40, 0), (28, 28), (40, 13), (20, 0), (14, 14)]
    r = np.array([np.hypot(*p) for p in pts])
    dr3 = np.array([D[p] for p in pts]) * r ** 3
    assert np.all(np.abs(dr3) < 0.05)
    # along an axis the r^-3 law holds to the next order: D(40)/D(20) ~ 1/8
    assert abs(D[40, 0] / D[20, 0] * 8.0 - 1.0) < 0.02


def test_difference_is_converged_in_the_grading_and_panels():
    a = ms.lgf_difference(9, 9, 9, 4)
    real = ms.rule_1d

    def finer(n_max, J=None):
        return real(2 * n_max + 8, J=ms.J_GRADE + 4)
    try:
        ms.rule_1d = finer
        b = ms.lgf_difference(9, 9, 9, 4)
    finally:
        ms.rule_1d = real
    assert np.abs(a - b).max() < 1e-16


# --- the solve ----------------------------------------------------------------------

@pytest.mark.parametrize("order", [4, 6])
def test_solve_satisfies_the_mehrstellen_problem(order):
    # (1/h^2) L u = R (f 1_box) at every cell whose stencils stay in the box
    rng = np.random.default_rng(order)
    shape, h = (12, 10, 11), 0.1
    f = rng.standard_normal(shape)
    u = ms.solve(f, h, order)
    r = 2 if order == 6 else 1
    Rf = ms.apply_stencil(np.pad(f, r), "R", order)      # R(f 1_box) on the whole box
    Lu = ms.apply_stencil(u, "L", order) / h ** 2        # cells 1 .. N-2
    rhs = Rf[1:-1, 1:-1, 1:-1]
    assert np.abs(Lu - rhs).max() < 1e-11 * np.abs(rhs).max()


def test_solve_equals_lattice_sum_with_the_kernel():
    rng = np.random.default_rng(1)
    shape, h = (5, 6, 4), 0.2
    f = rng.standard_normal(shape)
    K = ms.kernel_table(*shape, 4)
    ref = np.zeros(shape)
    idx = np.indices(shape).reshape(3, -1).T
    for i in idx:
        d = np.abs(idx - i)
        ref[tuple(i)] = np.sum(K[d[:, 0], d[:, 1], d[:, 2]] * f.ravel())
    ref *= h * h
    assert np.abs(ms.solve(f, h, 4) - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("order,lo,hi", [(4, 3.9, 4.1), (6, 5.6, 6.2)])
def test_convergence_order_on_the_paper_bump(order, lo, hi):
    # Sec. 4: E_inf proportional to h^M; measured 5.9e-4 -> 3.7e-5 (order 4)
    # and 1.7e-4 -> 3.1e-6 (order 6) from 16^3 to 32^3
    errs = []
    for n in (16, 32):
        h = 1.0 / n
        x = (np.arange(n) + 0.5) * h
        u = ms.solve(analytic.bump_source(x, x, x), h, order)
        errs.append(np.abs(u - analytic.bump_solution(x, x, x)).max())
    p = np.log2(errs[0] / errs[1])
    assert lo < p < hi, (errs, p)


# --- planted mistakes ---------------------------------------------------------------

def _rhs_unfolded(f, h, order, M=None):
    # R applied to nothing: the Mehrstellen LGF alone as the kernel
    real = ms.kernel_table
    try:
        ms.kernel_table = lambda kz, ky, kx, o: ms.lgf_table_mehrstellen(kz, ky, kx, o)
        return _real_solve(f, h, order, M)
    finally:
        ms.kernel_table = real


_real_solve = ms.solve


PLANTS = {
    # the cross term of L4 with the wrong sign
    "cross_term_sign": ("symbols", lambda s, o: (lambda sg, rh: (sg + (s[0] * s[1] + s[1] * s[2] + s[2] * s[0]) / 3.0,
                                                                 rh))(*REAL_SYMBOLS(s, o))),
    # the R6 cross term read literally as d_y d2_z (dropped here)
    "r6_cross_dropped": ("symbols", lambda s, o: (lambda sg, rh: (sg, rh - ((s[0] * s[1] + s[1] * s[2] + s[2] * s[0])
                                                                          / 90.0 if o == 6 else 0.0)))(*REAL_SYMBOLS(s, o))),
    # the grading stopped early: the corner box near k = 0 is too large
    "grading_short": ("J_GRADE", 3),
}
REAL_SYMBOLS = ms.symbols


@pytest.mark.parametrize("name", sorted(PLANTS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, val = PLANTS[name]
    monkeypatch.setattr(ms, attr, val)
    caught = 0
    for pin in (lambda: test_lgf_solves_the_mehrstellen_equation(4),
                lambda: test_lgf_solves_the_mehrstellen_equation(6),
                lambda: test_symbol_ratio_has_the_stated_order(6)):
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught > 0, name


def test_kernel_without_the_rhs_stencil_loses_the_order():
    # u = h^2 G_L * f without R is only second order
    errs = []
    for n in (16, 32):
        h = 1.0 / n
        x = (np.arange(n) + 0.5) * h
        u = _rhs_unfolded(analytic.bump_source(x, x, x), h, 4)
        errs.append(np.abs(u - analytic.bump_solution(x, x, x)).max())
    assert np.log2(errs[0] / errs[1]) < 2.5
