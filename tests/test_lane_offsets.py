"""32-bit per-lane byte offsets of the pass kernels, checked on the host.

Every kernel addresses W, G_hat and the twiddle tables as a wave-uniform
64-bit base plus a 32-bit per-lane byte offset (ld_at / st_at in
passes_impl.hpp).  A per-lane offset that reaches 2^32 wraps silently and
reads or writes another line's data, so each such product in the kernel
sources must stay below 2^32 for every shape the C ABI accepts.

The test finds every `unsigned(X) * unsigned(Y)` product in csrc/, maps it to
a row of the table below (the bound of X, the stride Y and the element size
of that formula), and evaluates the largest value at the extreme accepted
geometry of every precision and padded length.  A product that is not in the
table fails the test, so a new addressing formula must be added to it."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2512_08555_amd", "csrc")

POW2 = [32, 64, 128, 256, 512, 1024]
MIXED_F32 = [80, 96, 144, 160, 192, 288, 320, 384]


def lengths(prec):
    return POW2 + (MIXED_F32 if prec == "f32" else [])


def align16(v):
    return (v + 15) // 16 * 16


def geometry(prec, mx, my, mz):
    """The geometry the ABI builds (plan_layout): n = M/2 on every axis, the
    largest accepted for these padded lengths."""
    elem = 8 if prec == "f64" else 4
    kx = mx // 2 + 1
    px = align16(kx)
    gz = align16(mz // 2 + 1)
    return dict(elem=elem, cb=2 * elem, mx=mx, my=my, mz=mz, nx=mx // 2, ny=my // 2, nz=mz // 2,
                kx=kx, px=px, plane=my * px, gz=gz)


# (file, X, Y) -> largest byte offset at geometry g.  Column/tile widths are
# at most 16 columns, four-step split factors at most 64, and the wave-per-
# line kernels move rows tr < 64 of a 64-row block (the block itself goes
# into the 64-bit base).
def _col(g, rows, stride):
    return ((rows - 1) * stride + 15) * g["cb"]


FORMULAS = {
    # four-step column kernels: line position q or n2 < Q <= 64; stride = px
    # (y passes) or plane (z pass)
    ("passes_impl.hpp", "q", "stride"): lambda g: _col(g, 64, max(g["px"], g["plane"])),
    ("passes_impl.hpp", "n2", "stride"): lambda g: _col(g, 64, max(g["px"], g["plane"])),
    # y-pass spectrum rows k1 < P <= 64 (stores of yfwd, loads of yinv)
    ("passes_impl.hpp", "k1", "a.px"): lambda g: _col(g, 64, g["px"]),
    # z four-step G_hat loads: column c < 16 lines of gz reals, iz <= mz/2
    ("passes_impl.hpp", "c", "a.gz"): lambda g: (15 * g["gz"] + g["mz"] // 2) * g["elem"],
    # block count of the y-pass map (not an address): z lines x components
    ("passes_impl.hpp", "nz", "ncomp"): lambda g: g["nz"] * 8,
    # wave-per-line y passes: tile row tr < 64, or a ragged row < ny
    ("ywave.hpp", "tr", "a.px"): lambda g: _col(g, 64, g["px"]),
    ("ywave.hpp", "rowc", "a.px"): lambda g: _col(g, g["ny"], g["px"]),
    # wave-per-line z pass: tile row tr < 64 of a 64-row block
    ("zwave.hpp", "tr", "a.plane"): lambda g: _col(g, 64, g["plane"]),
}

PRODUCT = re.compile(r"unsigned\(([^()]*)\) \* unsigned\(([^()]*)\)")


def source_products():
    found = []
    for fn in sorted(os.listdir(CSRC)):
        if not fn.endswith((".hpp", ".hip", ".cpp")):
            continue
        with open(os.path.join(CSRC, fn)) as fh:
            for ln, line in enumerate(fh, 1):
                for m in PRODUCT.finditer(line):
                    found.append((fn, m.group(1).strip(), m.group(2).strip(), ln))
    return found


def test_every_offset_product_is_in_the_table():
    found = source_products()
    assert found, "no 32-bit offset products found: the scan is broken"
    for fn, x, y, ln in found:
        assert (fn, x, y) in FORMULAS, "%s:%d: unsigned(%s) * unsigned(%s) has no bound in this test" % (
            fn, ln, x, y)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_offsets_fit_32_bits_at_every_accepted_length(prec):
    worst = {}
    for mx in lengths(prec):
        for my in lengths(prec):
            for mz in lengths(prec):
                g = geometry(prec, mx, my, mz)
                for key, f in FORMULAS.items():
                    v = f(g)
                    worst[key] = max(worst.get(key, 0), v)
    for key, v in worst.items():
        assert v < 2 ** 32, "%s: %s offset %d reaches 2^32" % (prec, key, v)


def test_row_times_plane_would_wrap():
    """The form a z-pass offset must not take: a ragged row index (up to
    nz - 1 = 511) times the plane in 32 bits wraps for FP64 at 1024^2 x 528
    planes -- e.g. the (500, 260, 260) grid padded to 1024 per axis."""
    g = geometry("f64", 1024, 1024, 1024)
    assert (499 * g["plane"] + 15) * g["cb"] >= 2 ** 32
    assert FORMULAS[("zwave.hpp", "tr", "a.plane")](g) < 2 ** 32


def test_library_plans_the_extreme_shapes():
    """validate_problem refuses a plan whose per-lane offsets could reach
    2^32; none of the compiled lengths does, so the extreme shapes plan."""
    from paper_2512_08555_amd import _capi as capi
    if not os.path.exists(capi.LIB_PATH):
        pytest.skip("libups.so not built")
    import ctypes as C
    from paper_2512_08555_amd.solver import make_problem
    L = capi.lib()
    for prec in ("f32", "f64"):
        for shape in ((512, 512, 512), (500, 260, 260), (511, 512, 3)):
            pad = (1024, 1024, 1024)
            p = make_problem(shape, 0.01, prec, ncomp=8, pad=pad)
            h = C.c_void_p()
            assert L.ups_plan_create(C.byref(p), C.byref(h)) == capi.UPS_OK, L.ups_last_error()
            L.ups_plan_destroy(h)
