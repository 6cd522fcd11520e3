"""Every mirrored-fill variant of the forward passes (even and odd
directions, Sec. 2.2) against the oracle's per-axis solve: the wave-per-line
y and z kernels at 512 and 1024 points, the x one at 1024, and the four-step
kernels beside them, on thin grids whose mirrored axis has n = M/2 points."""
import numpy as np
import pytest
import torch

from oracle import bc as obc
from paper_2512_08555_amd import workloads
from paper_2512_08555_amd.solver import Plan, kernel_variants

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-6}
AXIS_OF_PASS = {0: 2, 1: 1, 2: 0}   # forward pass -> array axis (z, y, x) of its line


def _cases():
    out = []
    for prec in ("f64", "f32"):
        for M in (512, 1024):
            for k in (0, 1, 2):
                for name in kernel_variants(k, prec, M, fill=True):
                    out.append((prec, M, k, name))
    return out


try:
    CASES = _cases()
except Exception:  # library not built: collection must still work
    CASES = []


@pytest.mark.parametrize("prec,M,k,name", CASES)
@pytest.mark.parametrize("sym", ["even", "odd"])
def test_fill_variant_matches_oracle(prec, M, k, name, sym):
    ax = AXIS_OF_PASS[k]
    shape = [6, 10, 7]
    pad = [32, 32, 32]
    bc = ["unb", "unb", "unb"]
    shape[ax], pad[ax], bc[ax] = M // 2, M, sym
    shape, pad, bc = tuple(shape), tuple(pad), tuple(bc)
    print("[case] fill variant %s pass %d M %d %s %s shape %s" % (name, k, M, prec, sym, shape), flush=True)
    h = 1.0 / max(shape)
    f = workloads.blob_source(shape, h, seed=M + k, nblobs=3, sigma=(0.05, 0.12), noise=1e-3)
    if prec == "f32":
        f = f.astype(np.float32).astype(np.float64)
    plan = Plan(shape, h, prec, pad=pad, bc=bc)
    assert plan.kernel(k) == kernel_variants(k, prec, M, fill=True)[0]   # the default is the first
    plan.set_kernel(k, name)
    dt = torch.float64 if prec == "f64" else torch.float32
    u = plan.solve(torch.from_numpy(f).to("cuda", dt)).double().cpu().numpy()
    ref = obc.solve_bc(f, h, bc, M=pad)
    err = float(np.abs(u - ref).max() / np.abs(ref).max())
    print("  rel Linf %.3e" % err, flush=True)
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_wave_fill_variants_are_the_defaults_at_long_lines(prec):
    for M in (512, 1024):
        for k in (0, 1, 2):
            if k == 0 and M == 512:
                continue   # a 512-point real line has no wave-per-line x kernel
            names = kernel_variants(k, prec, M, fill=True)
            assert names and "_w" in names[0] and names[0].endswith("_e"), names
