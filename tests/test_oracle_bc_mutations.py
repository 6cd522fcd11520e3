"""The mixed-boundary pins must be able to fail: each case plants one
plausible mistake in oracle/bc.py with monkeypatch and requires every pin
named for it to fail.  No GPU."""
import numpy as np
import pytest

from oracle import bc as obc
from tests import test_oracle_bc as pins

REAL = {n: getattr(obc, n) for n in ("lgf1d_screened", "lgf2d_table", "_symbol_1d", "extend",
                                     "kernel_spectrum", "transform_lengths")}


def screened_sign_flipped(mp):
    mp.setattr(obc, "lgf1d_screened", lambda n, s: -REAL["lgf1d_screened"](n, s))


def lgf2d_tail_dropped(mp):
    mp.setattr(obc, "lgf2d_table", lambda k0, k1, T=None, K=6: REAL["lgf2d_table"](k0, k1, T, K=0))


def symbol_not_squared(mp):
    # 2 |sin(pi k / L)| in place of 4 sin^2(pi k / L)
    mp.setattr(obc, "_symbol_1d", lambda L: 2.0 * np.abs(np.sin(np.pi * np.arange(L) / L)))


def even_mirror_about_cell_centre(mp):
    # the even extension mirrored about the last cell centre instead of the
    # box face: [f0 .. f(N-1), f(N-2) .. f0, f0]
    def bad(f, bc, L):
        g = np.asarray(f, dtype=np.float64)
        for ax in range(3):
            n = g.shape[ax]
            if bc[ax] == "unb":
                pad = [(0, 0)] * 3
                pad[ax] = (0, L[ax] - n)
                g = np.pad(g, pad)
            elif bc[ax] == "even":
                g = np.concatenate([g, np.flip(np.take(g, range(n - 1), axis=ax), axis=ax),
                                    np.take(g, [0], axis=ax)], axis=ax)
            elif bc[ax] == "odd":
                g = np.concatenate([g, -np.flip(g, axis=ax)], axis=ax)
        return g
    mp.setattr(obc, "extend", bad)


def two_unbounded_without_2d_lgf(mp):
    # 1/sigma everywhere, also on the zero wavenumber of the third direction
    def bad(L, bc, shape=None):
        if sum(b == "unb" for b in bc) == 2:
            s = [obc._symbol_1d(l) for l in L]
            g = np.meshgrid(*s, indexing="ij")
            sig = g[0] + g[1] + g[2]
            out = np.zeros(tuple(L))
            nz = sig != 0
            out[nz] = -1.0 / sig[nz]
            return out
        return REAL["kernel_spectrum"](L, bc, shape)
    mp.setattr(obc, "kernel_spectrum", bad)


def periodic_axis_zero_padded(mp):
    # a periodic direction transformed like an unbounded one, zero-padded to
    # 2N, with the periodic symbol on that grid: the images of the source
    # are missing
    def bad_len(shape, bc, M=None):
        return tuple(2 * int(n) if b == "per" else l
                     for n, b, l in zip(shape, bc, REAL["transform_lengths"](shape, bc, M)))

    def bad_ext(f, bc, L):
        g = REAL["extend"](f, bc, L)
        for ax in range(3):
            if bc[ax] == "per":
                pad = [(0, 0)] * 3
                pad[ax] = (0, L[ax] - g.shape[ax])
                g = np.pad(g, pad)
        return g
    mp.setattr(obc, "transform_lengths", bad_len)
    mp.setattr(obc, "extend", bad_ext)


DENSE = lambda: pins.test_spectral_solve_equals_dense_solve(("per", "even", "odd"))  # noqa: E731
DENSE_EVEN = lambda: pins.test_spectral_solve_equals_dense_solve(("even", "even", "per"))  # noqa: E731
SCREENED = lambda: pins.test_lgf1d_screened_solves_its_equation(0.3)  # noqa: E731
G2_NEAR = pins.test_lgf2d_nearest_values_are_textbook
MIXED_RES = lambda: pins.test_mixed_solve_satisfies_the_discrete_equation(("unb", "per", "even"))  # noqa: E731
LATTICE_2D = lambda: pins.test_two_unbounded_z_independent_source_is_the_2d_lattice_sum("per")  # noqa: E731
ORDER_2UNB = lambda: pins.test_second_order_convergence(("per", "unb", "unb"))  # noqa: E731

CASES = {
    "screened_sign_flipped": (screened_sign_flipped, [SCREENED, MIXED_RES]),
    "lgf2d_tail_dropped": (lgf2d_tail_dropped, [G2_NEAR, LATTICE_2D]),
    "symbol_not_squared": (symbol_not_squared, [DENSE, MIXED_RES]),
    "even_mirror_about_cell_centre": (even_mirror_about_cell_centre, [DENSE_EVEN]),
    "two_unbounded_without_2d_lgf": (two_unbounded_without_2d_lgf, [LATTICE_2D, ORDER_2UNB]),
    "periodic_axis_zero_padded": (periodic_axis_zero_padded, [DENSE, ORDER_2UNB]),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_planted_mistake_is_caught(name, monkeypatch):
    plant, expected = CASES[name]
    plant(monkeypatch)
    missed = []
    for pin in expected:
        try:
            pin()
        except AssertionError:
            continue
        missed.append(getattr(pin, "__name__", repr(pin)))
    assert not missed, "%s passed under the planted mistake %s" % (missed, name)


def test_pins_pass_without_a_mistake():
    for pin in (DENSE, DENSE_EVEN, SCREENED, G2_NEAR, MIXED_RES, LATTICE_2D, ORDER_2UNB):
        pin()
