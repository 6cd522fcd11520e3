"""Which plans carry the Nyquist column in column 0 of W, and what that does
to the work buffer and to kernel choice (host only, no GPU)."""
import pytest

from paper_2512_08555_amd import _capi as capi
from paper_2512_08555_amd.lengths import auto_pad
from paper_2512_08555_amd.solver import Plan


def _plan(shape, prec, **kw):
    kw.setdefault("pad", auto_pad(shape, prec))
    return Plan(shape, 1.0 / max(shape), prec, setup=False, **kw)


@pytest.mark.parametrize("shape,prec,kw,packed", [
    ((512, 512, 512), "f32", {}, True),
    ((200, 30, 500), "f32", {}, True),               # mz 512, my 64, mx 1024
    ((300, 20, 400), "f32", {}, True),               # mz 1024
    ((512, 512, 512), "f64", {}, False),             # FP64: column slabs
    ((256, 256, 256), "f32", {}, False),             # mx 512
    ((100, 30, 500), "f32", {}, False),              # mz 256
    ((64, 16, 512), "f32", dict(bc=("unb", "unb", "even"), pad=(128, 32, 1024)), False),
    ((256, 16, 512), "f32", dict(bc=("odd", "unb", "unb"), pad=(512, 32, 1024)), False),
    ((256, 16, 500), "f32", dict(bc=("unb", "per", "unb"), pad=(512, 32, 1024)), True),
    ((256, 30, 500), "f32", dict(green="mehr4"), True),
])
def test_which_plans_pack(shape, prec, kw, packed):
    assert _plan(shape, prec, **kw).nyquist_packed is packed


def test_packed_plans_keep_the_unpacked_buffers():
    # packing changes what column 0 holds, not the layout or the sizes
    p = _plan((200, 30, 500), "f32", ncomp=3)
    lay = p.layout()
    assert lay["pitch"] >= 513
    assert p.work_bytes >= 8 * lay["comp_stride"] * 3
    assert capi.lib().ups_plan_nyquist_packed(None) == -1


def test_packed_plans_refuse_four_step_x_and_z_kernels_and_slabs():
    from paper_2512_08555_amd.solver import kernel_variants
    p = _plan((512, 512, 512), "f32")
    assert p.kernel(0).startswith("xfwd_float_w") and p.kernel(2).startswith("zconv_float_w")
    four_step = [v for v in kernel_variants(0, "f32", 1024) if "_w" not in v]
    assert four_step
    with pytest.raises(capi.UpsError) as ei:
        p.set_kernel(0, four_step[0])
    assert ei.value.status == capi.UPS_ERR_UNSUPPORTED
    with pytest.raises(capi.UpsError) as ei:
        p.set_kernel(2, [v for v in kernel_variants(2, "f32", 1024) if "_w" not in v][0])
    assert ei.value.status == capi.UPS_ERR_UNSUPPORTED
    p.set_kernel(1, kernel_variants(1, "f32", 1024)[-1])        # y passes: any variant
    st = capi.lib().ups_plan_set_slab(p._h, 128)
    assert st == capi.UPS_ERR_UNSUPPORTED
    assert capi.lib().ups_plan_set_slab(p._h, 0) == capi.UPS_OK


def test_nyquist_pair_identity():
    # The identity the column-0 pair launch evaluates: for a real source the
    # x-frequencies 0 and mx/2 of its spectrum are real along x, so after the
    # y and z transforms F_0 and F_N are Hermitian in (ky, kz); with
    # F_C = F_0 + i F_N and real G_hat lines G0, GN,
    #   R(ky, kz) = F_C(ky, kz) (G0 + GN) / 2 + conj F_C(-ky, -kz) (G0 - GN) / 2
    # equals G0 F_0 + i GN F_N, and the inverse of R is the solve's kx = 0
    # part plus i times its kx = mx/2 part.  Checked with numpy FFTs on a
    # random real field, independently of the kernels.
    import numpy as np
    rng = np.random.default_rng(7)
    mz, my, mx = 12, 10, 16
    f = rng.standard_normal((mz, my, mx))
    X = np.fft.rfft(f, axis=2)                  # [z, y, kx], kx = 0 .. mx/2
    F = np.fft.fft(np.fft.fft(X, axis=1), axis=0)
    F0, FN = F[:, :, 0], F[:, :, mx // 2]
    G0 = rng.standard_normal((mz, my))
    GN = rng.standard_normal((mz, my))
    # G_hat is even: G(-ky, -kz) = G(ky, kz)
    rev = lambda a: np.roll(a[::-1, ::-1], 1, axis=(0, 1))
    G0 = (G0 + rev(G0)) / 2
    GN = (GN + rev(GN)) / 2
    FC = F0 + 1j * FN
    R = FC * (G0 + GN) / 2 + np.conj(rev(FC)) * (G0 - GN) / 2
    assert np.allclose(R, G0 * F0 + 1j * GN * FN, rtol=0, atol=1e-12 * np.abs(F).max())
    # the inverse: kx = 0 part plus i times the kx = mx/2 part, both real
    r = np.fft.ifft(np.fft.ifft(R, axis=0), axis=1)
    p0 = np.fft.ifft(np.fft.ifft(G0 * F0, axis=0), axis=1)
    pN = np.fft.ifft(np.fft.ifft(GN * FN, axis=0), axis=1)
    assert np.abs(p0.imag).max() < 1e-12 and np.abs(pN.imag).max() < 1e-12
    assert np.allclose(r, p0.real + 1j * pN.real, rtol=0, atol=1e-12)
    # a planted mistake (the conjugate of the unmirrored line) breaks it
    Rbad = FC * (G0 + GN) / 2 + np.conj(FC) * (G0 - GN) / 2
    assert not np.allclose(Rbad, G0 * F0 + 1j * GN * FN, rtol=0, atol=1e-6 * np.abs(F).max())
