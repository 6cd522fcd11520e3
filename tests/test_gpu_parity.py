"""Parity of the HIP path (through the C ABI) with the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2512_08555_amd import workloads

pytestmark = pytest.mark.gpu


def _plan(shape, h, prec="f64", ncomp=1, pad=None):
    from paper_2512_08555_amd.lengths import auto_pad
    from paper_2512_08555_amd.solver import Plan
    if pad is None:
        pad = auto_pad(shape, prec)
    return Plan(shape, h, prec, ncomp=ncomp, pad=pad)


def _dev(a, prec):
    return torch.from_numpy(np.ascontiguousarray(a)).to(
        device="cuda", dtype=torch.float64 if prec == "f64" else torch.float32)


def _rel_inf(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _announce(msg):
    print("[case]", msg, flush=True)


# ---- A0: Green's spectrum ------------------------------------------------------

@pytest.mark.parametrize("shape,prec", [((16, 16, 16), "f64"), ((12, 20, 28), "f64"),
                                        ((64, 64, 64), "f64"), ((32, 32, 32), "f32")])
def test_green_spectrum_matches_oracle(shape, prec):
    _announce("ghat %s %s" % (shape, prec))
    h = 1.0 / max(shape)
    plan = _plan(shape, h, prec)
    got = plan.ghat().cpu().numpy().astype(np.float64)
    ref = oracle.green_spectrum_scaled(plan.padded, h)
    tol = 1e-13 if prec == "f64" else 2e-7
    assert got.shape == ref.shape
    assert _rel_inf(got, ref) < tol


def test_green_spectrum_513_octant_f64():
    """The FP64 spectrum of the 512^3 solve: the whole 513^3 octant against
    the oracle's DCT-I of its LGF table."""
    _announce("ghat 513^3 octant f64")
    n = 512
    h = 1.0 / n
    plan = _plan((n, n, n), h, "f64")
    got = plan.ghat().cpu().numpy()
    del plan
    torch.cuda.empty_cache()
    ref = oracle.green_spectrum_scaled((2 * n,) * 3, h)
    assert got.shape == ref.shape == (n + 1,) * 3
    err = _rel_inf(got, ref)
    print("ghat 513^3 rel Linf %.3e" % err, flush=True)
    assert err < 1e-13


# ---- single passes against numpy's FFT -----------------------------------------

def test_passes_one_by_one_f64():
    _announce("passes f64 (10, 12, 14)")
    shape = (10, 12, 14)
    nz, ny, nx = shape
    rng = np.random.default_rng(3)
    f = rng.standard_normal(shape)
    plan = _plan(shape, 0.1, "f64")
    mz, my, mx = plan.padded
    kx = mx // 2 + 1
    fd = _dev(f, "f64")
    W = plan.work_complex()
    plan.run_pass(0, f=fd)
    torch.cuda.synchronize()
    ref1 = np.fft.rfft(f, n=mx, axis=2)
    got1 = W[0, :, :ny, :kx].cpu().numpy()
    assert _rel_inf(got1, ref1) < 1e-14
    plan.run_pass(1)
    torch.cuda.synchronize()
    ref2 = np.fft.fft(ref1, n=my, axis=1)
    got2 = W[0, :, :my, :kx].cpu().numpy()
    assert _rel_inf(got2, ref2) < 1e-14
    plan.run_pass(2)
    torch.cuda.synchronize()
    G = plan.ghat().cpu().numpy()
    iz = np.minimum(np.arange(mz), mz - np.arange(mz))
    iy = np.minimum(np.arange(my), my - np.arange(my))
    spec = np.fft.fft(ref2, n=mz, axis=0) * G[np.ix_(iz, iy, np.arange(kx))]
    ref3 = (np.fft.ifft(spec, axis=0) * mz)[:nz]
    got3 = W[0, :, :my, :kx].cpu().numpy()
    assert _rel_inf(got3, ref3) < 1e-13
    plan.run_pass(3)
    torch.cuda.synchronize()
    ref4 = (np.fft.ifft(ref3, axis=1) * my)[:, :ny]
    got4 = W[0, :, :ny, :kx].cpu().numpy()
    assert _rel_inf(got4, ref4) < 1e-13
    u = torch.empty_like(fd)
    plan.run_pass(4, u=u)
    torch.cuda.synchronize()
    ref5 = (np.fft.irfft(ref4, n=mx, axis=2) * mx)[:, :, :nx]
    assert _rel_inf(u.cpu().numpy(), ref5) < 1e-13


# ---- A1-A5: the whole solve ------------------------------------------------------

@pytest.mark.parametrize("shape", [(16, 16, 16), (32, 32, 32), (13, 17, 11), (5, 40, 9), (64, 48, 33)])
def test_solve_f64_matches_oracle(shape):
    _announce("solve f64 %s" % (shape,))
    rng = np.random.default_rng(sum(shape))
    f = rng.standard_normal(shape)
    h = 1.0 / max(shape)
    plan = _plan(shape, h, "f64")
    u = plan.solve(_dev(f, "f64")).cpu().numpy()
    ref = oracle.solve(f, h)
    assert _rel_inf(u, ref) < 1e-12


def test_c1_workload_f64():
    cfg = workloads.config_c1()
    _announce("c1 32^3 f64")
    f, h = cfg["f"], cfg["h"]
    plan = _plan(cfg["shape"], h, "f64")
    assert plan.padded == (64, 64, 64)
    u = plan.solve(_dev(f, "f64")).cpu().numpy()
    ref = oracle.solve(f, h)
    assert _rel_inf(u, ref) < 1e-12
    # and against the brute-force lattice sum on a 12^3 corner of it
    fc = f[:12, :12, :12].copy()
    pc = _plan(fc.shape, h, "f64")
    uc = pc.solve(_dev(fc, "f64")).cpu().numpy()
    assert _rel_inf(uc, oracle.brute_force(fc, h)) < 1e-12


@pytest.mark.parametrize("shape", [(32, 32, 32), (24, 40, 17)])
def test_solve_f32_error_vs_f64_oracle(shape):
    _announce("solve f32 %s" % (shape,))
    rng = np.random.default_rng(7)
    f = rng.standard_normal(shape).astype(np.float32).astype(np.float64)
    h = 1.0 / max(shape)
    plan = _plan(shape, h, "f32")
    u = plan.solve(_dev(f, "f32")).cpu().numpy().astype(np.float64)
    ref = oracle.solve(f, h)
    err = _rel_inf(u, ref)
    print("f32 rel Linf", err)
    assert err < 2e-6


def test_vector_rhs_equals_scalar_solves():
    _announce("vector rhs 3 x 24^3 f64")
    n = 24
    h = 1.0 / n
    f = workloads.curl_source(n, h, seed=9)
    pv = _plan((n, n, n), h, "f64", ncomp=3)
    uv = pv.solve(_dev(f, "f64")).cpu().numpy()
    ps = _plan((n, n, n), h, "f64")
    for c in range(3):
        us = ps.solve(_dev(f[c], "f64")).cpu().numpy()
        assert np.array_equal(us, uv[c])
        assert _rel_inf(uv[c], oracle.solve(f[c], h)) < 1e-12


def test_in_place_and_adjoint_dot_product():
    _announce("in place + adjoint 20x18x22 f64")
    shape = (20, 18, 22)
    rng = np.random.default_rng(21)
    f = rng.standard_normal(shape)
    g = rng.standard_normal(shape)
    h = 0.05
    plan = _plan(shape, h, "f64")
    fd, gd = _dev(f, "f64"), _dev(g, "f64")
    Kf = plan.solve(fd).cpu().numpy()
    Ktg = plan.adjoint(gd).cpu().numpy()
    lhs, rhs = np.vdot(Kf, g), np.vdot(f, Ktg)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    assert _rel_inf(Ktg, oracle.brute_force_adjoint(g, h) if max(shape) <= 12 else oracle.adjoint(g, h)) < 1e-12
    x = fd.clone()
    plan.solve(x, out=x)
    assert np.array_equal(x.cpu().numpy(), Kf)
    # the input of an out-of-place solve is untouched
    assert np.array_equal(fd.cpu().numpy(), f)


def test_repeated_solves_are_deterministic():
    _announce("determinism 32^3 f32")
    rng = np.random.default_rng(5)
    f = _dev(rng.standard_normal((32, 32, 32)), "f32")
    plan = _plan((32, 32, 32), 1 / 32, "f32")
    a = plan.solve(f).clone()
    for _ in range(3):
        assert torch.equal(plan.solve(f), a)
