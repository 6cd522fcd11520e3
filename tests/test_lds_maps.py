"""The LDS exchange maps of the wave-per-line transforms (csrc/zwave.hpp),
checked on the host for line lengths M = 64 E, E = 8, 16, 32.

Each exchange stores register i of lane l at waddr(l, i) and loads register
i of lane l from raddr(l, i), once for the real parts and once for the
imaginary parts.  For every exchange this test checks, against the index
algebra written in the header comment of zwave.hpp:

* the stores of one exchange are injective (no two values share a word);
* every load reads the word that holds the element the next stage expects;
* every address lies inside the wave's slot;
* for 32-bit words (FP32), the 32 lanes of each half-wave touch 32 distinct
  banks for every register (32 banks of 4 bytes).

The maps are restated here from zwave.hpp (the strides S1, P2, S4 and the
swizzle of the second inverse exchange)."""
import pytest

BANKS = 32


def consts(E):
    A = 64 // E
    E2 = E * E
    S1 = 64 + 32 // E
    P2 = E2 + ((E % 32) - (E2 % 32) + 32) % 32
    S4 = 65
    xfloats = max(E * S1, A * P2, (E - 1) * S4 + 64)
    return A, E2, S1, P2, S4, xfloats


def slot_complex(E, CW):
    # zwave_slot<E, CW>(): room for the M/2 tile rows and one exchange
    _, _, _, _, _, xf = consts(E)
    need = max(32 * E, (xf + 1) // 2)
    r = (16 // CW) % 16
    while need % 16 != r:
        need += 1
    return need


def exchanges(E):
    """(name, waddr, welem, raddr, relem): addresses and the element each
    (lane, register) stores / must receive, per the zwave.hpp index algebra."""
    A, E2, S1, P2, S4, _ = consts(E)
    HE = E // 2
    out = []

    # forward exchange 1: lane l stores k1 = i at k1 S1 + l; lane (k1, l1)
    # = (L % E, L / E) loads l2 = i, element (k1, l = l1 + A l2)
    out.append(("fwd1",
                lambda l, i: l + i * S1, lambda l, i: (i, l),
                lambda L, i: (L % E) * S1 + L // E + A * i, lambda L, i: (L % E, L // E + A * i)))

    # forward exchange 2: lane (k1, l1) = (L % E, L / E) stores m1 = i as
    # a = k1 + E m1 at l1 P2 + a; lane L loads register r A + l1' as
    # element (a = L + 64 r, l1')
    out.append(("fwd2",
                lambda L, i: (L // E) * P2 + L % E + E * i, lambda L, i: (L % E + E * i, L // E),
                lambda L, i: L + (i % A) * P2 + 64 * (i // A), lambda L, i: (L + 64 * (i // A), i % A)))

    # inverse exchange 1: lane L stores register i = r A + n0 as element
    # (a = L + 64 r, n0) at n0 P2 + a; lane (b, n0) = (L % E, L / E) loads
    # c = i, element (a = b + E c, n0)
    out.append(("inv1",
                lambda L, i: L + (i % A) * P2 + 64 * (i // A), lambda L, i: (L + 64 * (i // A), i % A),
                lambda L, i: (L // E) * P2 + L % E + E * i, lambda L, i: (L % E + E * i, L // E)))

    # inverse exchange 2: lane (b, n0) = (L % E, L / E) stores e = i at
    # e S4 + E n0 + (b ^ swz(n0)); lane (n0, e) = (L % A, L / A) loads
    # b = i, element (b, n0, e)
    def swz(n0):
        return HE if n0 >= A // 2 else 0

    out.append(("inv2",
                lambda L, i: E * (L // E) + ((L % E) ^ swz(L // E)) + S4 * i,
                lambda L, i: (L % E, L // E, i),
                lambda L, i: (L // A) * S4 + E * (L % A) + (i ^ swz(L % A)),
                lambda L, i: (i, L % A, L // A)))
    return out


@pytest.mark.parametrize("E", [8, 16, 32])
def test_exchange_maps_injective_and_correct(E):
    xfloats = consts(E)[5]
    for name, wa, we, ra, re_ in exchanges(E):
        word = {}
        for L in range(64):
            for i in range(E):
                a = wa(L, i)
                assert 0 <= a < xfloats, (name, E, L, i, a)
                assert a not in word, "%s E=%d: two stores to word %d" % (name, E, a)
                word[a] = we(L, i)
        assert len(word) == 64 * E
        for L in range(64):
            for i in range(E):
                a = ra(L, i)
                assert a in word, "%s E=%d: lane %d reg %d loads unwritten word %d" % (name, E, L, i, a)
                assert word[a] == re_(L, i), (name, E, L, i, word[a], re_(L, i))


@pytest.mark.parametrize("E", [8, 16, 32])
def test_exchange_maps_bank_conflict_free_fp32(E):
    for name, wa, _, ra, _ in exchanges(E):
        for kind, f in (("store", wa), ("load", ra)):
            for i in range(E):
                for half in (range(0, 32), range(32, 64)):
                    banks = {f(L, i) % BANKS for L in half}
                    assert len(banks) == 32, "%s %s E=%d reg %d: %d banks" % (name, kind, E, i, len(banks))


@pytest.mark.parametrize("E,CW", [(8, 16), (8, 8), (8, 4), (8, 1), (16, 16), (16, 8), (16, 4), (16, 1)])
def test_slot_holds_tile_and_exchange(E, CW):
    s = slot_complex(E, CW)
    assert s >= 32 * E                          # the M/2 rows of the column
    assert 2 * s >= consts(E)[5]                # one exchange (floats)
    assert s % 16 == (16 // CW) % 16            # slot stride modulo 16 complex words


@pytest.mark.parametrize("E", [8, 16])
@pytest.mark.parametrize("sign", [1, -1])
def test_mirrored_fill_maps(E, sign):
    # The wave-per-line forward kernels along an even or odd direction:
    # lane l, register j >= E/2 holds row n = l + 64 j of the line of
    # M = 64 E points, which is sign times row M - 1 - n, read from lane
    # 63 - l, register E - 1 - j (a register below E/2, loaded as usual).
    import numpy as np
    M = 64 * E
    lanes = np.arange(64)
    for j in range(E // 2, E):
        n = lanes + 64 * j
        src = (63 - lanes) + 64 * (E - 1 - j)
        assert np.array_equal(src, M - 1 - n) and src.max() < M // 2 and src.min() >= 0
    # x: the packed complex line Z[m] = x[2m] + i x[2m+1] (L = M/2 = 32 E
    # complex points, nx = L reals mirrored to 2 L) has
    # Z[m] = sign * (Im Z[L-1-m] + i Re Z[L-1-m]) for m >= L/2
    rng = np.random.default_rng(E)
    L = 32 * E
    x = rng.standard_normal(L)
    ext = np.concatenate([x, sign * x[::-1]])
    Z = ext[0::2] + 1j * ext[1::2]
    m = np.arange(L // 2, L)
    Zr = Z[L - 1 - m]
    assert np.allclose(Z[m], sign * (Zr.imag + 1j * Zr.real), rtol=0, atol=0)
    # the x kernel holds the packed line of Lx = 64 E complex points (2 Lx
    # reals: E = 8 for 1024-point lines) as m = lane + 64 j; register
    # j >= E/2 reads m' = Lx - 1 - m = (63 - lane) + 64 (E - 1 - j)
    Lx = 64 * E
    for j in range(E // 2, E):
        mm = lanes + 64 * j
        assert np.array_equal((63 - lanes) + 64 * (E - 1 - j), Lx - 1 - mm)
