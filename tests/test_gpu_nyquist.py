"""Plans whose column 0 of W carries the Nyquist column X[mx/2] in its
imaginary part (FP32, mx = 1024, mz = 512 or 1024): the solve against the
oracle, for scalar and vector sources, mixed boundary conditions, the
Mehrstellen kernel and the adjoint (the pair launch of the z pass uses the
Hermitian symmetry of the real kx = 0 and kx = mx/2 columns, Sec. 2.2)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import bc as obc
from paper_2512_08555_amd import workloads
from paper_2512_08555_amd.lengths import auto_pad
from paper_2512_08555_amd.solver import Plan

pytestmark = pytest.mark.gpu
TOL = 2e-6


def _src(shape, seed, ncomp=1):
    h = 1.0 / max(shape)
    fs = [workloads.blob_source(shape, h, seed=seed + c, nblobs=6, sigma=(0.03, 0.1), noise=1e-3)
          for c in range(ncomp)]
    f = fs[0] if ncomp == 1 else np.stack(fs)
    return f.astype(np.float32).astype(np.float64), h


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("shape", [(200, 30, 500), (300, 20, 400), (256, 64, 512), (511, 7, 511)])
def test_packed_solve_matches_oracle(shape):
    f, h = _src(shape, 3)
    pad = auto_pad(shape, "f32")
    plan = Plan(shape, h, "f32", pad=pad)
    print("[case] packed %s pad %s" % (shape, pad), flush=True)
    assert plan.nyquist_packed
    u = plan.solve(torch.from_numpy(f).float().cuda()).double().cpu().numpy()
    err = _rel(u, oracle.solve(f, h, M=pad))
    print("  rel Linf %.2e" % err, flush=True)
    assert err < TOL


def test_packed_vector_source_and_adjoint():
    shape = (200, 30, 500)
    f, h = _src(shape, 7, ncomp=3)
    pad = auto_pad(shape, "f32")
    plan = Plan(shape, h, "f32", ncomp=3, pad=pad)
    print("[case] packed vector %s" % (shape,), flush=True)
    assert plan.nyquist_packed
    fd = torch.from_numpy(f).float().cuda()
    u = plan.solve(fd).double().cpu().numpy()
    g = plan.adjoint(fd).double().cpu().numpy()
    for c in range(3):
        ref = oracle.solve(f[c], h, M=pad)
        assert _rel(u[c], ref) < TOL and _rel(g[c], ref) < TOL


@pytest.mark.parametrize("bc", [("per", "unb", "unb"), ("unb", "odd", "unb"), ("unb", "per", "per"),
                                ("per", "even", "per")])
def test_packed_mixed_boundary_conditions(bc):
    shape = tuple(256 if b != "unb" and i == 0 else 16 if b != "unb" else n
                  for i, (b, n) in enumerate(zip(bc, (300, 20, 500))))
    if bc[2] == "per":
        shape = shape[:2] + (512,)
    f, h = _src(shape, 11)
    ap = auto_pad(shape, "f32")
    pad = tuple(m if b == "unb" else 2 * n for n, b, m in zip(shape, bc, ap))
    plan = Plan(shape, h, "f32", pad=pad, bc=bc)
    print("[case] packed bc %s shape %s pad %s packed %s" % (bc, shape, pad, plan.nyquist_packed), flush=True)
    assert plan.nyquist_packed
    if "unb" not in bc and "odd" not in bc:
        f = f - f.mean()
    u = plan.solve(torch.from_numpy(f).float().cuda()).double().cpu().numpy()
    err = _rel(u, obc.solve_bc(f, h, bc, M=pad))
    print("  rel Linf %.2e" % err, flush=True)
    assert err < TOL


def test_packed_mehrstellen_solve():
    # against the unpacked FP64 plan of the same problem (the oracle's
    # Mehrstellen table for a 513-wide x octant takes minutes on the CPU;
    # the FP64 path is checked against it at smaller sizes)
    shape = (200, 24, 500)
    f, h = _src(shape, 13)
    pad = auto_pad(shape, "f32")
    plan = Plan(shape, h, "f32", pad=pad, green="mehr6")
    print("[case] packed mehr6 %s" % (shape,), flush=True)
    assert plan.nyquist_packed
    u = plan.solve(torch.from_numpy(f).float().cuda()).double().cpu().numpy()
    p64 = Plan(shape, h, "f64", pad=pad, green="mehr6")
    assert not p64.nyquist_packed
    ref = p64.solve(torch.from_numpy(f).cuda()).cpu().numpy()
    err = _rel(u, ref)
    print("  rel Linf %.2e" % err, flush=True)
    assert err < TOL


def test_packed_equals_fp64_unpacked_at_512():
    # the 512^3 headline configuration: the packed FP32 solve against the
    # unpacked FP64 solve of the same (FP32-rounded) input
    n = 512
    f = torch.from_numpy(workloads.config_blobs_noise(n, 2).astype(np.float32)).cuda()
    p32 = Plan((n, n, n), 1.0 / n, "f32")
    print("[case] 512^3 packed FP32 vs FP64", flush=True)
    assert p32.nyquist_packed
    u32 = p32.solve(f)
    del p32
    p64 = Plan((n, n, n), 1.0 / n, "f64")
    assert not p64.nyquist_packed
    u64 = p64.solve(f.double())
    err = float((u32.double() - u64).abs().max() / u64.abs().max())
    print("  rel Linf %.2e" % err, flush=True)
    assert err < 1e-6
