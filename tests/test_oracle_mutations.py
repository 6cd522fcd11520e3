"""The oracle's pins must be able to fail.

Each case plants one plausible mistake in the CPU oracle (a flipped sign, a
dropped term, a wrong index, a missing factor, a too-short integration
range) with pytest's monkeypatch, runs the pins that should notice it, and
requires every one of them to fail.  The oracle is restored after each case.
No GPU.

Mistakes that only permute the axes of the kernel or of the source are not
mistakes for this operator: G1 is symmetric under every permutation and
reflection of its index, so u = h^2 G1 * f commutes with axis permutations
and any padded length M >= 2N - 2 gives the same box values; the solve pins
use non-cubic grids and paddings so that a swapped extent still shows.
"""
import importlib

import numpy as np
import pytest
import scipy.fft as sfft

import oracle
from tests import test_oracle_pins as pins

LGF = importlib.import_module("oracle.lgf")
SPEC = importlib.import_module("oracle.spectrum")
SOLVE = importlib.import_module("oracle.solve")
MODULES = (oracle, LGF, SPEC, SOLVE)

REAL = {
    "lgf_table": LGF.lgf_table,
    "quadrature_nodes": LGF.quadrature_nodes,
    "hankel_coefficients": LGF.hankel_coefficients,
    "green_spectrum_raw": SPEC.green_spectrum_raw,
    "solve": SOLVE.solve,
}


def _plant(mp, name, fn):
    """Replace ``name`` wherever the oracle binds it (its own module and
    every module that imported it by name)."""
    hit = False
    for mod in MODULES:
        if name in vars(mod):
            mp.setattr(mod, name, fn)
            hit = True
    assert hit, name


# --- the planted mistakes ---------------------------------------------------------

def lgf_sign_flipped(mp):
    # G1 taken as the Green's function of -L (the symbol's sign dropped)
    _plant(mp, "lgf_table", lambda *a, **k: -REAL["lgf_table"](*a, **k))


def lgf_half_argument(mp):
    # e^{-t} I_n(t) in place of e^{-2t} I_n(2t): the kernel of L/2, twice G1
    _plant(mp, "lgf_table", lambda *a, **k: 2.0 * REAL["lgf_table"](*a, **k))


def tail_dropped(mp):
    mp.setattr(LGF, "_tail_moment", lambda m, T: 0.0)


def tail_exponent_off(mp):
    # int_T^inf t^{-3/2 - m} dt integrated as if the power were t^{-5/2 - m}
    real = LGF._tail_moment
    mp.setattr(LGF, "_tail_moment", lambda m, T: real(m, T) * (m + 0.5) / (m + 1.5) / T)


def hankel_sign_dropped(mp):
    # a_k(nu) used without the alternating sign (-1)^k
    _plant(mp, "hankel_coefficients", lambda nu, K=LGF.TAIL_TERMS: np.abs(REAL["hankel_coefficients"](nu, K)))


def hankel_nu_not_squared(mp):
    # mu = 4 nu in place of 4 nu^2
    def bad(nu, K=LGF.TAIL_TERMS):
        nu = np.atleast_1d(np.asarray(nu, dtype=np.float64))
        return REAL["hankel_coefficients"](np.sqrt(nu), K)
    _plant(mp, "hankel_coefficients", bad)


def tail_truncated(mp):
    mp.setattr(LGF, "TAIL_TERMS", 1)


def quadrature_range_short(mp):
    # s = ln t starting at -5: the part of the integral near t = 0 is lost
    mp.setattr(LGF, "S_LO", -5.0)


def quadrature_too_coarse(mp):
    mp.setattr(LGF, "PANEL_ORDER", 4)


def quadrature_jacobian_dropped(mp):
    # weights of ds used for dt (the factor t of dt = t ds left out)
    def bad(T):
        t, w = REAL["quadrature_nodes"](T)
        return t, w / t
    _plant(mp, "quadrature_nodes", bad)


def dct_orthonormal(mp):
    # the spectrum taken with an orthonormal DCT-I instead of the plain sum
    def bad(M, G1=None):
        M = tuple(int(m) for m in M)
        K = tuple(m // 2 + 1 for m in M)
        G = LGF.lgf_table(*K) if G1 is None else np.asarray(G1)[: K[0], : K[1], : K[2]]
        return sfft.dctn(G, type=1, norm="ortho")
    _plant(mp, "green_spectrum_raw", bad)


def spectrum_normalised_twice(mp):
    # 1/(Mz My Mx) applied to G_hat although the inverse DFT already has it
    _plant(mp, "green_spectrum_raw", lambda M, G1=None: REAL["green_spectrum_raw"](M, G1) / float(np.prod(M)))


def mirror_off_by_one(mp):
    # periodised index min(k, M - 1 - k) in place of min(k, M - k)
    mp.setattr(SOLVE, "_mirror", lambda M: np.minimum(np.arange(M), M - 1 - np.arange(M)))


def h_not_squared(mp):
    # the solve scaled by h instead of h^2
    _plant(mp, "solve", lambda f, h, **k: REAL["solve"](f, float(h) ** 0.5, **k))


def adjoint_unscaled(mp):
    mp.setattr(SOLVE, "adjoint", lambda g, h, **k: REAL["solve"](g, 1.0, **k))
    mp.setattr(oracle, "adjoint", SOLVE.adjoint)


# --- which pins must catch which mistake --------------------------------------------

G0 = pins.test_g0_is_watson_closed_form
DELTA = lambda: pins.test_lgf_solves_lattice_poisson_with_delta(9)  # noqa: E731
GOLDEN = pins.test_lgf_table_matches_golden_adaptive_points
TAIL = pins.test_tail_formula_against_quadrature_of_ive
SPEC_EQ = lambda: pins.test_spectrum_dct_equals_rfft_of_periodisation((16, 20, 24))  # noqa: E731
SPEC_NEG = pins.test_spectrum_negative_and_nyquist_limit
BRUTE = lambda: pins.test_solve_equals_brute_force_lattice_sum((6, 10, 7))  # noqa: E731
POISSON = pins.test_solve_satisfies_discrete_poisson_inside_box
DELTA_SRC = pins.test_delta_source_gives_scaled_lgf
ADJ = pins.test_adjoint_dot_product_and_transpose
GAUSS = pins.test_gaussian_closed_form_second_order

CASES = {
    "lgf_sign_flipped": (lgf_sign_flipped, [G0, DELTA, SPEC_NEG, POISSON]),
    "lgf_half_argument": (lgf_half_argument, [G0, DELTA, POISSON]),
    "tail_dropped": (tail_dropped, [G0, GOLDEN]),
    "tail_exponent_off": (tail_exponent_off, [G0, GOLDEN, TAIL]),
    "hankel_sign_dropped": (hankel_sign_dropped, [TAIL]),
    "hankel_nu_not_squared": (hankel_nu_not_squared, [TAIL, GOLDEN]),
    "tail_truncated": (tail_truncated, [GOLDEN]),
    "quadrature_range_short": (quadrature_range_short, [G0, GOLDEN]),
    "quadrature_too_coarse": (quadrature_too_coarse, [G0, GOLDEN]),
    "quadrature_jacobian_dropped": (quadrature_jacobian_dropped, [G0, DELTA]),
    "dct_orthonormal": (dct_orthonormal, [SPEC_EQ, BRUTE, DELTA_SRC]),
    "spectrum_normalised_twice": (spectrum_normalised_twice, [BRUTE, POISSON, DELTA_SRC]),
    "mirror_off_by_one": (mirror_off_by_one, [BRUTE, DELTA_SRC]),
    "h_not_squared": (h_not_squared, [BRUTE, POISSON, DELTA_SRC, GAUSS]),
    "adjoint_unscaled": (adjoint_unscaled, [ADJ]),
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
    # the same calls as above, unmutated (so a failure above is the mistake's)
    for pin in (G0, DELTA, TAIL, SPEC_EQ, SPEC_NEG, BRUTE, POISSON, DELTA_SRC, ADJ):
        pin()
