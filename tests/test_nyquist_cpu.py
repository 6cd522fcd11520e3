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
