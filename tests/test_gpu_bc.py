"""Periodic, even and odd directions mixed with unbounded ones (Sec. 2.2,
eq. 2unbkernel) through the C ABI, against the oracle's plain per-axis
solve."""
import itertools

import numpy as np
import pytest
import torch

from oracle import bc as obc
from paper_2512_08555_amd import workloads
from paper_2512_08555_amd.lengths import auto_pad
from paper_2512_08555_amd.solver import Batch, Plan

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-6}
PER_UNB = [b for b in itertools.product(("unb", "per"), repeat=3) if "per" in b]


def _rel_inf(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _pads(shape, bc, prec):
    """2 n along periodic, even and odd axes, the smallest supported length
    >= 2 n along unbounded ones."""
    ap = auto_pad(shape, prec)
    return tuple(m if b == "unb" else 2 * n for n, b, m in zip(shape, bc, ap))


def _source(shape, h, seed):
    return workloads.blob_source(shape, h, seed=seed, nblobs=5, sigma=(0.05, 0.12), noise=1e-3)


def _run(shape, bc, prec, seed, ncomp=1):
    h = 1.0 / max(shape)
    pad = _pads(shape, bc, prec)
    print("[case] bc %s %s shape %s pad %s ncomp %d" % (bc, prec, shape, pad, ncomp), flush=True)
    if ncomp == 1:
        f = _source(shape, h, seed)
    else:
        f = np.stack([_source(shape, h, seed + c) for c in range(ncomp)])
    if prec == "f32":
        f = f.astype(np.float32).astype(np.float64)
    plan = Plan(shape, h, prec, ncomp=ncomp, pad=pad, bc=bc)
    dt = torch.float64 if prec == "f64" else torch.float32
    u = plan.solve(torch.from_numpy(f).to("cuda", dt)).double().cpu().numpy()
    comps = [(u, f)] if ncomp == 1 else [(u[c], f[c]) for c in range(ncomp)]
    worst = 0.0
    for uc, fc in comps:
        ref = obc.solve_bc(fc, h, bc, M=pad)
        worst = max(worst, _rel_inf(uc, ref))
    print("  rel Linf %.3e" % worst, flush=True)
    return worst


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("bc", PER_UNB)
def test_periodic_mixes_match_oracle(bc, prec):
    # periodic axes of 16 or 32 points (2 n a compiled length), unbounded
    # axes of uneven sizes padded to the next compiled length
    shape = tuple(32 if b == "per" and i == 0 else 16 if b == "per" else n
                  for i, (b, n) in enumerate(zip(bc, (20, 27, 13))))
    assert _run(shape, bc, prec, seed=len(shape) + hash(bc) % 97) < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_two_unbounded_one_periodic_vector_source(prec):
    assert _run((32, 30, 21), ("per", "unb", "unb"), prec, seed=3, ncomp=3) < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_two_unbounded_one_periodic_128(prec):
    # the configuration of the paper's vortex tube: periodic along z,
    # unbounded in x and y, one wave per line in every pass (pads 256)
    assert _run((128, 128, 128), ("per", "unb", "unb"), prec, seed=21) < TOL[prec]


def test_fully_periodic_mean_free():
    shape, bc = (32, 16, 64), ("per", "per", "per")
    h = 1.0 / 64
    f = _source(shape, h, 5)
    f -= f.mean()
    plan = Plan(shape, h, "f64", bc=bc)
    u = plan.solve(torch.from_numpy(f).cuda()).cpu().numpy()
    ref = obc.solve_bc(f, h, bc)
    assert abs(u.mean()) < 1e-14 * np.abs(u).max()
    assert _rel_inf(u, ref) < 1e-12


def test_batch_with_periodic_directions_equals_single_plans():
    specs = [dict(shape=(32, 20, 27), h=1 / 32, prec="f32", bc=("per", "unb", "unb"), pad=(64, 64, 64)),
             dict(shape=(16, 32, 32), h=1 / 32, prec="f32", bc=("unb", "per", "per"), pad=(32, 64, 64)),
             dict(shape=(20, 20, 20), h=1 / 20, prec="f32", pad=(64, 64, 64)),
             dict(shape=(16, 16, 16), h=1 / 16, prec="f32", bc=("per",) * 3, pad=(32, 32, 32))]
    print("[case] batch of %d problems with periodic directions" % len(specs), flush=True)
    b = Batch(specs)
    fs = [torch.from_numpy(_source(sp["shape"], sp["h"], 40 + i).astype(np.float32)).cuda()
          for i, sp in enumerate(specs)]
    us = b.solve(fs)
    torch.cuda.synchronize()
    for i, sp in enumerate(b.specs):
        p = Plan(sp["shape"], sp["h"], "f32", pad=sp["pad"], bc=sp["bc"])
        assert torch.equal(p.solve(fs[i]), us[i]), i
        ref = obc.solve_bc(fs[i].double().cpu().numpy(), sp["h"], sp["bc"], M=sp["pad"])
        assert _rel_inf(us[i].double().cpu().numpy(), ref) < TOL["f32"], i


# ---- even and odd directions (mirrored fill in the forward passes) ----------------

MIRROR = [("even", "unb", "unb"), ("unb", "odd", "unb"), ("unb", "unb", "even"), ("odd", "odd", "odd"),
          ("even", "even", "even"), ("per", "even", "odd"), ("odd", "unb", "per"), ("even", "odd", "unb")]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("bc", MIRROR)
def test_even_odd_mixes_match_oracle(bc, prec):
    # spectral axes of 16 or 32 points (the mirrored-fill kernels cover
    # padded lengths 32 .. 1024); the x extent of an even or odd direction
    # must be even
    base = (20, 27, 13)
    shape = tuple(n if b == "unb" else (32 if i == 1 else 16) for i, (b, n) in enumerate(zip(bc, base)))
    f_mean_free = "unb" not in bc and "odd" not in bc
    h = 1.0 / max(shape)
    pad = _pads(shape, bc, prec)
    print("[case] bc %s %s shape %s pad %s" % (bc, prec, shape, pad), flush=True)
    f = _source(shape, h, 17 + hash(bc) % 91)
    if f_mean_free:
        f -= f.mean()
    if prec == "f32":
        f = f.astype(np.float32).astype(np.float64)
    plan = Plan(shape, h, prec, pad=pad, bc=bc)
    assert all(plan.kernel(k).endswith("_e") == (bc[2 - k] in ("even", "odd")) for k in range(3))
    dt = torch.float64 if prec == "f64" else torch.float32
    u = plan.solve(torch.from_numpy(f).to("cuda", dt)).double().cpu().numpy()
    ref = obc.solve_bc(f, h, bc, M=pad)
    err = _rel_inf(u, ref)
    print("  rel Linf %.3e" % err, flush=True)
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_even_odd_at_long_lines(prec):
    # mirrored fill at the lengths 512 and 1024 (wave-per-line y and z
    # kernels, the four-step x kernel)
    shape, bc = (64, 16, 512), ("even", "odd", "even")
    h = 1.0 / 512
    pad = _pads(shape, bc, prec)
    print("[case] bc %s %s shape %s pad %s" % (bc, prec, shape, pad), flush=True)
    f = _source(shape, h, 77)
    f -= f.mean()
    if prec == "f32":
        f = f.astype(np.float32).astype(np.float64)
    plan = Plan(shape, h, prec, pad=pad, bc=bc)
    dt = torch.float64 if prec == "f64" else torch.float32
    u = plan.solve(torch.from_numpy(f).to("cuda", dt)).double().cpu().numpy()
    ref = obc.solve_bc(f, h, bc, M=pad)
    assert _rel_inf(u, ref) < TOL[prec]
    shape, bc = (256, 24, 20), ("odd", "unb", "unb")
    h = 1.0 / 256
    pad = _pads(shape, bc, prec)
    print("[case] bc %s %s shape %s pad %s" % (bc, prec, shape, pad), flush=True)
    f = _source(shape, h, 78)
    if prec == "f32":
        f = f.astype(np.float32).astype(np.float64)
    plan = Plan(shape, h, prec, pad=pad, bc=bc)
    u = plan.solve(torch.from_numpy(f).to("cuda", dt)).double().cpu().numpy()
    ref = obc.solve_bc(f, h, bc, M=pad)
    assert _rel_inf(u, ref) < TOL[prec]


def test_batch_with_even_and_odd_directions_equals_single_plans():
    specs = [dict(shape=(32, 20, 16), h=1 / 32, prec="f64", bc=("even", "unb", "odd"), pad=(64, 64, 32)),
             dict(shape=(16, 16, 16), h=1 / 16, prec="f64", bc=("odd",) * 3, pad=(32, 32, 32)),
             dict(shape=(24, 20, 16), h=1 / 24, prec="f64", pad=(64, 64, 32))]
    print("[case] batch of %d problems with even and odd directions" % len(specs), flush=True)
    b = Batch(specs)
    fs = [torch.from_numpy(_source(sp["shape"], sp["h"], 60 + i)).cuda() for i, sp in enumerate(specs)]
    us = b.solve(fs)
    torch.cuda.synchronize()
    for i, sp in enumerate(b.specs):
        p = Plan(sp["shape"], sp["h"], "f64", pad=sp["pad"], bc=sp["bc"])
        assert torch.equal(p.solve(fs[i]), us[i]), i
        ref = obc.solve_bc(fs[i].cpu().numpy(), sp["h"], sp["bc"], M=sp["pad"])
        assert _rel_inf(us[i].cpu().numpy(), ref) < TOL["f64"], i


def test_vortex_tube_velocity_second_order():
    # the paper's Biot-Savart benchmark (Sec. 5): -curl(omega) as a
    # 3-component source, unbounded in x and y, periodic in z; FP64 against
    # the oracle at 32^3 and against the closed-form velocity at second order
    from oracle import analytic
    errs = []
    for n in (32, 64, 128):
        print("[case] vortex tube %d^3 f64" % n, flush=True)
        f = workloads.vortex_tube_source(n)
        plan = Plan((n, n, n), 1.0 / n, "f64", ncomp=3, bc=("per", "unb", "unb"))
        u = plan.solve(torch.from_numpy(f).cuda()).cpu().numpy()
        assert np.abs(u[2]).max() < 1e-12 * np.abs(u[:2]).max()
        ref = analytic.vortex_tube_velocity(n)
        errs.append(np.abs(u[:2] - ref[:2]).max() / np.abs(ref[:2]).max())
        if n == 32:
            for c in range(2):
                assert _rel_inf(u[c], obc.solve_bc(f[c], 1.0 / n, ("per", "unb", "unb"))) < 1e-12
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print("vortex tube rel Linf %s orders %s" % (errs, orders), flush=True)
    assert 1.95 < orders[-1] < 2.2 and errs[-1] < 5e-4
