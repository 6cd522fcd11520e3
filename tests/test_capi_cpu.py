"""The C-ABI library on a machine without a GPU: it loads, exports every
symbol include/ups.h declares, validates problems and fails cleanly."""
import ctypes as C
import os
import re

import pytest

from paper_2512_08555_amd import _capi as capi
from paper_2512_08555_amd.solver import make_problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    if not os.path.exists(capi.LIB_PATH):
        pytest.skip("libups.so not built")
    return capi.lib()


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "ups.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ups_[a-z_]+)\s*\(", txt)))


def test_header_symbols_exported():
    L = _lib_or_skip()
    names = _declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
        assert n in capi.SIGNATURES, "binding lacks " + n


def test_abi_version_and_lengths():
    L = _lib_or_skip()
    assert L.ups_abi_version() == 2
    for m in (32, 64, 128, 256, 512, 1024):
        assert L.ups_supported_length(m, capi.UPS_F64) == 1
        assert L.ups_supported_length(m, capi.UPS_F32) == 1
    assert L.ups_supported_length(33, capi.UPS_F64) == 0
    assert L.ups_supported_length(0, capi.UPS_F64) == 0


def _create(p):
    L = capi.lib()
    h = C.c_void_p()
    s = L.ups_plan_create(C.byref(p), C.byref(h))
    return s, h, L.ups_last_error().decode()


def test_validation_errors():
    L = _lib_or_skip()
    p = make_problem((32, 32, 32), 1 / 32)
    s, h, _ = _create(p)
    assert s == capi.UPS_OK
    L.ups_plan_destroy(h)

    p = make_problem((32, 32, 1), 1 / 32)
    s, h, msg = _create(p)
    assert s == capi.UPS_ERR_INVALID_ARG and "n[0]" in msg and not h.value

    p = make_problem((32, 32, 32), 1 / 32)
    p.h[1] = 0.5
    assert _create(p)[0] == capi.UPS_ERR_UNSUPPORTED

    p = make_problem((32, 32, 32), 1 / 32)
    p.h[2] = -1.0
    assert _create(p)[0] == capi.UPS_ERR_INVALID_ARG

    # boundary conditions: the same on both sides of an axis; periodic
    # directions padded to exactly 2 n; even and odd directions not solved
    p = make_problem((32, 32, 32), 1 / 32)
    p.bc[1][0] = capi.UPS_BC_PER
    s, _, msg = _create(p)
    assert s == capi.UPS_ERR_UNSUPPORTED and "both sides" in msg
    p = make_problem((32, 32, 32), 1 / 32, bc=("per", "unb", "unb"))
    s, h, _ = _create(p)
    assert s == capi.UPS_OK
    L.ups_plan_destroy(h)
    p = make_problem((32, 32, 32), 1 / 32, bc=("per", "per", "per"))
    s, h, _ = _create(p)
    assert s == capi.UPS_OK
    L.ups_plan_destroy(h)
    p = make_problem((30, 32, 32), 1 / 32, pad=(64, 64, 64), bc=("per", "unb", "unb"))
    s, _, msg = _create(p)
    assert s == capi.UPS_ERR_INVALID_ARG and "periodic" in msg
    for b in ("even", "odd"):
        p = make_problem((32, 32, 32), 1 / 32, bc=("unb", b, "unb"))
        s, h, _ = _create(p)
        assert s == capi.UPS_OK
        assert L.ups_plan_kernel(h, 1).decode().endswith("_e")        # mirrored-fill y-forward
        assert not L.ups_plan_kernel(h, 3).decode().endswith("_e")    # inverse unchanged
        L.ups_plan_destroy(h)
        p = make_problem((32, 32, 32), 1 / 32, bc=("unb", b, "unb"))
        p.center = capi.UPS_NODE
        s, _, msg = _create(p)
        assert s == capi.UPS_ERR_UNSUPPORTED and "cell faces" in msg
    p = make_problem((32, 32, 31), 1 / 32, pad=(64, 64, 62), bc=("unb", "unb", "even"))
    s, _, msg = _create(p)
    assert s == capi.UPS_ERR_UNSUPPORTED and "even n[0]" in msg
    p = make_problem((32, 32, 40), 1 / 40, bc=("unb", "unb", "odd"))   # 80: no mirrored-fill kernel
    s, _, msg = _create(p)
    assert s == capi.UPS_ERR_UNSUPPORTED and "mirrored-fill" in msg
    p = make_problem((32, 32, 32), 1 / 32, bc=("per", "unb", "unb"))
    p.green = capi.UPS_GREEN_LGF4_MEHR
    assert _create(p)[0] == capi.UPS_ERR_UNSUPPORTED

    for g in ("mehr4", "mehr6"):
        p = make_problem((32, 32, 32), 1 / 32, green=g)
        s, h, _ = _create(p)
        assert s == capi.UPS_OK
        L.ups_plan_destroy(h)

    p = make_problem((32, 32, 32), 1 / 32, ncomp=9)
    assert _create(p)[0] == capi.UPS_ERR_INVALID_ARG

    p = make_problem((20, 20, 20), 1 / 20, pad=(36, 40, 40))   # 36 < 2*20-2
    assert _create(p)[0] == capi.UPS_ERR_INVALID_ARG
    # 2n - 2 is exact for the convolution but the pruned kernels need 2n
    p = make_problem((33, 20, 20), 1 / 33, pad=(64, 64, 64))
    s, _, msg = _create(p)
    assert s == capi.UPS_ERR_INVALID_ARG and ">= 2 n" in msg
    p = make_problem((20, 20, 20), 1 / 20, pad=(40, 40, 41))   # odd
    assert _create(p)[0] == capi.UPS_ERR_INVALID_ARG
    p = make_problem((20, 20, 20), 1 / 20)                      # 40: no kernel
    assert _create(p)[0] == capi.UPS_ERR_UNSUPPORTED
    p = make_problem((20, 20, 20), 1 / 20, pad=(64, 64, 64))
    s, h, _ = _create(p)
    assert s == capi.UPS_OK
    L.ups_plan_destroy(h)

    assert L.ups_plan_create(None, C.byref(C.c_void_p())) == capi.UPS_ERR_INVALID_ARG
    assert L.ups_plan_create(C.byref(p), None) == capi.UPS_ERR_INVALID_ARG


def test_sizes_model_bytes_and_kernels():
    L = _lib_or_skip()
    p = make_problem((512, 512, 512), 1 / 512, prec="f32")
    s, h, _ = _create(p)
    assert s == capi.UPS_OK
    g, w = C.c_size_t(), C.c_size_t()
    assert L.ups_plan_sizes(h, C.byref(g), C.byref(w)) == capi.UPS_OK
    N = 512
    # work holds W = N * 2N * pitch complex float, pitch >= N + 1
    assert w.value >= N * 2 * N * (N + 1) * 8
    assert g.value >= (N + 1) ** 3 * 4
    # byte model: s [2 N^3 + 24 (N+1) N^2 + (N+1)^3], s = 4
    ref = 4.0 * (2 * N ** 3 + 24 * (N + 1) * N ** 2 + (N + 1) ** 3)
    assert abs(L.ups_plan_model_bytes(h, -1) - ref) < 1e-6 * ref
    assert sum(L.ups_plan_model_bytes(h, k) for k in range(5)) == pytest.approx(ref)
    assert L.ups_plan_model_bytes(h, 7) == 0.0
    names = [L.ups_plan_kernel(h, k).decode() for k in range(5)]
    assert names[0].startswith("xfwd_float") and names[2].startswith("zconv_float")
    assert L.ups_plan_kernel(h, 5) is None
    assert L.ups_plan_set_kernel(h, 2, b"nonexistent") == capi.UPS_ERR_INVALID_ARG
    assert L.ups_plan_set_kernel(h, 2, names[2].encode()) == capi.UPS_OK
    L.ups_plan_destroy(h)


def test_calls_before_setup_and_without_device_fail_cleanly():
    L = _lib_or_skip()
    p = make_problem((32, 32, 32), 1 / 32)
    s, h, _ = _create(p)
    assert s == capi.UPS_OK
    assert L.ups_solve(h, C.c_void_p(4096), C.c_void_p(8192), None) == capi.UPS_ERR_STATE
    assert L.ups_solve_adjoint(h, C.c_void_p(4096), C.c_void_p(8192), None) == capi.UPS_ERR_STATE
    assert L.ups_solve_noalloc(h, C.c_void_p(4096), C.c_void_p(8192), None) == capi.UPS_ERR_STATE
    assert L.ups_solve_noalloc(None, C.c_void_p(4096), C.c_void_p(8192), None) == capi.UPS_ERR_INVALID_ARG
    assert L.ups_run_pass(h, 0, C.c_void_p(4096), C.c_void_p(8192), None) == capi.UPS_ERR_STATE
    assert L.ups_run_pass(h, 9, None, None, None) == capi.UPS_ERR_INVALID_ARG
    g, w = C.c_size_t(), C.c_size_t()
    L.ups_plan_sizes(h, C.byref(g), C.byref(w))
    # size and alignment checks come before any device access
    assert L.ups_plan_setup(h, C.c_void_p(256), g.value - 1, C.c_void_p(1 << 20), w.value,
                            None) == capi.UPS_ERR_WORKSPACE
    assert L.ups_plan_setup(h, C.c_void_p(256), g.value, C.c_void_p(1 << 20), w.value - 1,
                            None) == capi.UPS_ERR_WORKSPACE
    assert L.ups_plan_setup(h, C.c_void_p(257), g.value, C.c_void_p(1 << 20), w.value,
                            None) == capi.UPS_ERR_INVALID_ARG
    assert L.ups_plan_setup(h, None, g.value, C.c_void_p(1 << 20), w.value, None) == capi.UPS_ERR_INVALID_ARG
    import torch
    if not torch.cuda.is_available():
        s = L.ups_plan_setup(h, C.c_void_p(256), g.value, C.c_void_p(1 << 20), w.value, None)
        assert s == capi.UPS_ERR_DEVICE
        assert "device" in L.ups_last_error().decode()
    L.ups_plan_destroy(h)


def test_batch_validation_without_device():
    L = _lib_or_skip()
    good = make_problem((20, 30, 40), 0.05, prec="f32", pad=(64, 64, 80))
    bad = make_problem((20, 30, 1), 0.05)
    arr = (capi.ups_problem * 2)(good, bad)
    h = C.c_void_p()
    assert L.ups_batch_create(arr, 2, C.byref(h)) == capi.UPS_ERR_INVALID_ARG
    assert L.ups_batch_create(arr, 0, C.byref(h)) == capi.UPS_ERR_INVALID_ARG
    many = (capi.ups_problem * 201)(*([good] * 201))
    assert L.ups_batch_create(many, 201, C.byref(h)) == capi.UPS_ERR_UNSUPPORTED
    arr = (capi.ups_problem * 3)(good, make_problem((16, 16, 16), 1 / 16, prec="f64"),
                                  make_problem((24, 24, 24), 1 / 24, prec="f32", ncomp=3, pad=(64, 64, 64)))
    assert L.ups_batch_create(arr, 3, C.byref(h)) == capi.UPS_OK
    g, w = C.c_size_t(), C.c_size_t()
    assert L.ups_batch_sizes(h, C.byref(g), C.byref(w)) == capi.UPS_OK
    assert g.value > 0 and w.value > 0
    assert all(L.ups_batch_launches(h, k) >= 1 for k in range(5))
    assert L.ups_batch_launches(h, 5) == 0
    fp = (C.c_void_p * 3)(4096, 8192, 12288)
    assert L.ups_batch_solve(h, fp, fp, None) == capi.UPS_ERR_STATE
    assert L.ups_batch_setup(h, C.c_void_p(256), g.value - 1, C.c_void_p(512), w.value,
                             None) == capi.UPS_ERR_WORKSPACE
    import torch
    if not torch.cuda.is_available():
        assert L.ups_batch_setup(h, C.c_void_p(256), g.value, C.c_void_p(512), w.value,
                                 None) == capi.UPS_ERR_DEVICE
    assert L.ups_batch_destroy(h) == capi.UPS_OK


def test_autotune_requires_setup():
    L = _lib_or_skip()
    p = make_problem((32, 32, 32), 1 / 32)
    s, h, _ = _create(p)
    assert s == capi.UPS_OK
    f, u = C.c_void_p(4096), C.c_void_p(8192)
    assert L.ups_autotune(h, f, u, None, 10.0) == capi.UPS_ERR_STATE
    assert L.ups_autotune(None, f, u, None, 10.0) == capi.UPS_ERR_INVALID_ARG
    L.ups_plan_destroy(h)


def test_debug_switches_without_device():
    L = _lib_or_skip()
    p = make_problem((32, 32, 32), 1 / 32)
    s, h, _ = _create(p)
    assert s == capi.UPS_OK
    assert L.ups_plan_set_check_finite(h, 1) == capi.UPS_OK
    assert L.ups_plan_set_check_finite(None, 1) == capi.UPS_ERR_INVALID_ARG
    assert L.ups_plan_guard_mode(h) in (0, 1)
    assert L.ups_plan_guard_mode(None) == -1
    L.ups_plan_destroy(h)


_GUARD_SCRIPT = r"""
import ctypes as C, sys
sys.path.insert(0, %r)
from paper_2512_08555_amd import _capi as capi
from paper_2512_08555_amd.solver import make_problem
L = capi.lib()
p = make_problem((32, 32, 32), 1 / 32, prec="f32")
h = C.c_void_p()
assert L.ups_plan_create(C.byref(p), C.byref(h)) == 0
g, w = C.c_size_t(), C.c_size_t()
L.ups_plan_sizes(h, C.byref(g), C.byref(w))
print(L.ups_plan_guard_mode(h), L.ups_plan_work_offset(h), w.value)
"""


def _run(env_extra, script):
    import subprocess
    import sys
    env = dict(os.environ)
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return r.stdout.split()


def test_guard_mode_layout():
    """UPS_DEBUG_GUARDS at plan creation: W moves past a 64 KiB canary band
    and the work buffer grows by two bands."""
    _lib_or_skip()
    off = _run({"UPS_DEBUG_GUARDS": "0"}, _GUARD_SCRIPT % ROOT)
    on = _run({"UPS_DEBUG_GUARDS": "1"}, _GUARD_SCRIPT % ROOT)
    assert off[:2] == ["0", "0"] and on[:2] == ["1", str(64 * 1024)]
    # 32^3 FP32: W = 32 * 64 * 48 complex floats; setup scratch may be larger
    W = 32 * 64 * 48 * 8
    assert int(on[2]) >= W + 2 * 64 * 1024


_KEY_SCRIPT = r"""
import ctypes as C, sys
sys.path.insert(0, %r)
from paper_2512_08555_amd import _capi as capi
from paper_2512_08555_amd.solver import make_problem
L = capi.lib()
out = []
for shape, pad in (((512, 512, 512), None), ((512, 16, 16), (1024, 32, 32))):
    p = make_problem(shape, 1 / 512, prec="f32", pad=pad)
    h = C.c_void_p()
    assert L.ups_plan_create(C.byref(p), C.byref(h)) == 0
    out.append(L.ups_plan_kernel(h, 2).decode())
    L.ups_plan_destroy(h)
print(" ".join(out))
"""


def test_tuning_cache_key_has_size_class(tmp_path):
    """A cached choice applies to plans of the same pass, precision, padded
    length and size class (floor log2 of the lines of the pass): the 512^3
    z pass has 513 x 1024 lines (class 19); a 16 x 16 x 512 grid padded to
    32 x 32 x 1024 has 17 x 32 (class 9) and keeps the table default."""
    _lib_or_skip()
    from paper_2512_08555_amd.solver import kernel_variants
    names = kernel_variants(2, "f32", 1024)
    # a wave-per-line variant: the 512^3 FP32 plan carries the Nyquist column
    # in column 0 and runs only those in its z pass
    default, other = names[0], [n for n in names if "_w" in n][-1]
    assert default != other
    cache = tmp_path / "tune.json"
    cache.write_text('{"zconv/f32/1024/l19": "%s"}' % other)
    got = _run({"UPS_TUNE_CACHE": str(cache)}, _KEY_SCRIPT % ROOT)
    assert got == [other, default]
    cache.write_text('{"zconv/f32/1024/l9": "%s"}' % other)
    got = _run({"UPS_TUNE_CACHE": str(cache)}, _KEY_SCRIPT % ROOT)
    assert got == [default, other]


def test_kernel_variant_listing():
    _lib_or_skip()
    from paper_2512_08555_amd.solver import kernel_variants
    L = capi.lib()
    for k in range(5):
        for prec in ("f32", "f64"):
            names = kernel_variants(k, prec, 512)
            assert names, (k, prec)
            assert len(set(names)) == len(names)
    z = kernel_variants(2, "f32", 1024)
    assert any(n.startswith("zconv_float_w16") for n in z)
    assert L.ups_kernel_variants(5, capi.UPS_F32, 512, None, 0) == 0
    assert L.ups_kernel_variants(0, 7, 512, None, 0) == 0
    assert L.ups_kernel_variants(0, capi.UPS_F32, 33, None, 0) == 0
    # a plan's default is the first variant listed
    p = make_problem((512, 8, 8), 1 / 512, prec="f32", pad=(1024, 32, 32))
    s, h, _ = _create(p)
    assert s == capi.UPS_OK
    assert L.ups_plan_kernel(h, 2).decode() in z
    assert L.ups_plan_set_slab(h, 7) == capi.UPS_ERR_INVALID_ARG
    assert L.ups_plan_set_slab(h, 16) == capi.UPS_OK
    assert L.ups_plan_slab(h) == 16
    L.ups_plan_destroy(h)
    assert L.ups_plan_slab(None) == -1


def test_default_schedule_pipelines_large_fp64_plans():
    # an FP64 plan with >= 384 x-frequencies starts with 128-column slabs
    # pipelined over two streams; other plans with one slab and the
    # remainder launches on the second stream
    from paper_2512_08555_amd.solver import Plan
    big64 = Plan((8, 8, 300), 1.0 / 300, "f64", pad=(32, 32, 1024), setup=False)
    small64 = Plan((8, 8, 200), 1.0 / 200, "f64", pad=(32, 32, 512), setup=False)
    big32 = Plan((8, 8, 300), 1.0 / 300, "f32", pad=(32, 32, 1024), setup=False)
    assert (big64.slab, big64.side_stream) == (128, True)
    assert (small64.slab, small64.side_stream) == (0, True)
    assert (big32.slab, big32.side_stream) == (0, True)
    big32.set_side_stream(False)
    assert not big32.side_stream
    assert capi.lib().ups_plan_side_stream(None) == -1
