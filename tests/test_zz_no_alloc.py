"""ups_solve_noalloc (W in the library's per-device array) against ups_solve
(W in the plan's work buffer), through the C ABI: two calls in a row, the
second on a smaller grid, in FP64 and FP32, plus the size limit."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2512_08555_amd import _capi as capi
from paper_2512_08555_amd import workloads
from paper_2512_08555_amd.solver import Plan, _stream_handle

pytestmark = pytest.mark.gpu


def _rel_inf(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _via_capi(plan, fname, f):
    u = plan.empty_like_io()
    fn = getattr(capi.lib(), fname)
    capi.check(fn(plan._h, C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()), _stream_handle()))
    torch.cuda.synchronize()
    return u


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 2e-6)])
def test_noalloc_matches_solve_two_calls(prec, tol):
    # the first grid's W fills most of the array; the second is smaller, so
    # it runs over what the first call left behind
    cases = ([((100, 120, 110), (256, 256, 256)), ((30, 20, 25), (64, 64, 64))] if prec == "f64" else
             [((120, 112, 128), (256, 256, 256)), ((40, 48, 36), (80, 96, 80))])
    for k, (shape, pad) in enumerate(cases):
        print("noalloc %s call %d shape %s pad %s" % (prec, k, shape, pad), flush=True)
        h = 1.0 / max(shape)
        plan = Plan(shape, h, prec, pad=pad)
        wbytes = 2 * (8 if prec == "f64" else 4) * plan.layout()["comp_stride"]
        assert wbytes <= capi.UPS_NOALLOC_MAX_WORK
        f = workloads.blob_source(shape, h, seed=30 + k, nblobs=6, sigma=(0.05, 0.1), noise=1e-3)
        ft = torch.from_numpy(f).to("cuda", plan.dtype)
        ref = _via_capi(plan, "ups_solve", ft).double().cpu().numpy()
        got = _via_capi(plan, "ups_solve_noalloc", ft).double().cpu().numpy()
        err = _rel_inf(got, ref)
        print("  rel Linf vs ups_solve %.3e" % err, flush=True)
        assert err < tol
        # the same kernels on the same schedule: identical values
        assert np.array_equal(got, ref)


def test_noalloc_vector_rhs_and_in_place():
    shape, h = (48, 40, 45), 1.0 / 48
    print("noalloc f32 3 components %s, in place" % (shape,), flush=True)
    plan = Plan(shape, h, "f32", ncomp=3, pad=(96, 80, 96))
    f = np.stack([workloads.blob_source(shape, h, seed=40 + c, nblobs=4, sigma=(0.05, 0.1), noise=0.0)
                  for c in range(3)])
    ft = torch.from_numpy(f).to("cuda", torch.float32)
    ref = _via_capi(plan, "ups_solve", ft)
    x = ft.clone()
    capi.check(capi.lib().ups_solve_noalloc(plan._h, C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()),
                                            _stream_handle()))
    torch.cuda.synchronize()
    assert torch.equal(x, ref)


def test_noalloc_rejects_plans_above_the_limit():
    shape = (160, 160, 160)
    print("noalloc limit: f32 %s" % (shape,), flush=True)
    plan = Plan(shape, 1.0 / 160, "f32")
    assert 2 * 4 * plan.layout()["comp_stride"] > capi.UPS_NOALLOC_MAX_WORK
    f = torch.zeros(shape, dtype=torch.float32, device="cuda")
    u = torch.empty_like(f)
    st = capi.lib().ups_solve_noalloc(plan._h, C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()),
                                      _stream_handle())
    assert st == capi.UPS_ERR_UNSUPPORTED
    assert b"at most" in capi.lib().ups_last_error()
