"""Column-pass schedules (slabs run one after the other or pipelined over two
streams, remainder launches on the side stream) give the oracle's result and
the single-slab values up to the last bit (a slab's last columns may go
through another compiled variant of the same pass)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2512_08555_amd.solver import Plan

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_schedules_match_oracle_and_each_other(prec):
    # nx = 250 pads to 512: 257 x-frequencies; slabs of 16/48/80/128/144 leave
    # ragged ends, some one column and some several columns past the aligned
    # launch width
    shape, pad = (20, 24, 250), (64, 64, 512)
    rng = np.random.default_rng(21)
    f = rng.standard_normal(shape)
    if prec == "f32":
        f = f.astype(np.float32).astype(np.float64)
    h = 1.0 / 250
    plan = Plan(shape, h, prec, pad=pad)
    dt = torch.float64 if prec == "f64" else torch.float32
    fd = torch.from_numpy(f).to("cuda", dt)
    ref = oracle.solve(f, h, M=pad)
    base = None
    for slab in (0, 16, 48, 80, 128, 144):
        for side in (False, True):
            print("[case] %s slab %d side %s" % (prec, slab, side), flush=True)
            plan.slab = slab
            plan.set_side_stream(side)
            u = plan.solve(fd)
            torch.cuda.synchronize()
            un = u.double().cpu().numpy()
            err = float(np.abs(un - ref).max() / np.abs(ref).max())
            assert err < (1e-12 if prec == "f64" else 3e-6), (slab, side, err)
            if base is None:
                base = un
            else:
                rel = float(np.abs(un - base).max() / np.abs(base).max())
                assert rel <= (4e-16 if prec == "f64" else 2e-7), (slab, side, rel)



@pytest.mark.parametrize("side", [False, True])
def test_wide_column_remainder(side):
    # nx = 190 padded to 384 (FP32): 193 x-frequencies, 65 past the aligned
    # 128-column launch, which take a second launch of the pass's own kernel
    shape, pad = (12, 20, 190), (32, 64, 384)
    rng = np.random.default_rng(23)
    f = rng.standard_normal(shape).astype(np.float32).astype(np.float64)
    h = 1.0 / 190
    plan = Plan(shape, h, "f32", pad=pad)
    plan.set_side_stream(side)
    print("[case] f32 pad 384 side %s" % side, flush=True)
    u = plan.solve(torch.from_numpy(f).to("cuda", torch.float32))
    torch.cuda.synchronize()
    ref = oracle.solve(f, h, M=pad)
    err = float(np.abs(u.double().cpu().numpy() - ref).max() / np.abs(ref).max())
    assert err < 3e-6, err


@pytest.mark.parametrize("prec,slab,side", [("f64", 128, True), ("f64", 0, True), ("f32", 0, False),
                                            ("f32", 0, True), ("f32", 128, True)])
def test_solve_captured_in_a_graph(prec, slab, side):
    """A solve captured in a HIP graph (two-stream pipelined schedule included)
    gives the eager result on every replay, with eager work between replays."""
    shape, pad = (16, 20, 300), (32, 64, 1024)
    rng = np.random.default_rng(31)
    dt = torch.float64 if prec == "f64" else torch.float32
    f = torch.from_numpy(rng.standard_normal(shape)).to("cuda", dt)
    plan = Plan(shape, 1.0 / 300, prec, pad=pad)
    plan.slab = slab
    plan.set_side_stream(side)
    print("[case] graph %s slab %d side %s" % (prec, slab, side), flush=True)
    ref = plan.solve(f)
    torch.cuda.synchronize()
    u = torch.empty_like(f)
    cap = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cap):
        plan.solve(f, out=u, stream=cap)
    for rep in range(3):
        u.zero_()
        tmp = plan.solve(f * 2.0)            # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        tol = 1e-15 if prec == "f64" else 1e-7
        assert float((u - ref).abs().max() / ref.abs().max()) <= tol, rep
        assert float((tmp - 2.0 * ref).abs().max() / ref.abs().max()) < (1e-14 if prec == "f64" else 1e-6)
