"""Every compiled kernel variant of every pass against the oracle.

Thin grids with one long axis reach the long padded lengths (1024 in FP32,
512 in FP64) while the oracle stays cheap; a short axis with a larger pad
exercises the ragged paths (fewer live rows than half the line)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2512_08555_amd.solver import Plan, kernel_variants

pytestmark = pytest.mark.gpu

AXIS_OF_PASS = {0: 2, 1: 1, 2: 0, 3: 1, 4: 2}   # pass -> array axis (z, y, x) of its line


def _cases():
    out = []
    for prec, lengths in (("f32", (64, 256, 512, 1024, 384)), ("f64", (64, 256, 512, 1024))):
        for M in lengths:
            for k in range(5):
                names = kernel_variants(k, prec, M)
                for nm in names:
                    out.append((prec, M, k, nm))
    return out


def _shape_pad(M, k, ragged):
    """Short axes of 6, 10, 7 points padded to 32; the pass's own axis has
    M/2 points (all live rows) or fewer (ragged), padded to M."""
    ax = AXIS_OF_PASS[k]
    shape = [6, 10, 7]
    pad = [32, 32, 32]
    shape[ax] = M // 2 - (M // 8 if ragged else 0)
    pad[ax] = M
    return tuple(shape), tuple(pad)


try:
    CASES = _cases()
except Exception:  # library not built: collection must still work
    CASES = []


@pytest.mark.parametrize("prec,M,k,name", CASES)
@pytest.mark.parametrize("ragged", [False, True])
def test_variant_matches_oracle(prec, M, k, name, ragged):
    shape, pad = _shape_pad(M, k, ragged)
    print("[case] variant %s pass %d M %d %s shape %s pad %s ragged %s" % (name, k, M, prec, shape, pad, ragged),
          flush=True)
    rng = np.random.default_rng(M + 7 * k)
    f = rng.standard_normal(shape)
    if prec == "f32":
        f = f.astype(np.float32).astype(np.float64)
    h = 1.0 / max(shape)
    plan = Plan(shape, h, prec, pad=pad)
    plan.set_kernel(k, name)
    dt = torch.float64 if prec == "f64" else torch.float32
    u = plan.solve(torch.from_numpy(f).to("cuda", dt)).double().cpu().numpy()
    ref = oracle.solve(f, h, M=pad)
    err = float(np.abs(u - ref).max() / np.abs(ref).max())
    tol = 1e-12 if prec == "f64" else 3e-6
    assert err < tol, (name, err)


def _wave_cases():
    out = []
    for prec, lengths in (("f32", (512, 1024)), ("f64", (512, 1024))):
        for M in lengths:
            for k in (2, 3):
                for nm in kernel_variants(k, prec, M):
                    if "_w" in nm:
                        out.append((k, prec, M, nm))
    return out


try:
    WAVE_CASES = _wave_cases()
except Exception:  # library not built: collection must still work
    WAVE_CASES = []


@pytest.mark.parametrize("k,prec,M,name", WAVE_CASES)
def test_wave_pass_aligned_columns_plus_remainder(k, prec, M, name):
    """257 x-frequencies: a wave-per-line pass runs 256 aligned columns and
    one left over through the narrow kernel of its family."""
    ax = AXIS_OF_PASS[k]
    shape, pad = [6, 6, 140], [32, 32, 512]
    shape[ax], pad[ax] = M // 2 - 3, M
    shape, pad = tuple(shape), tuple(pad)
    print("[case] column split %s pass %d M %d %s" % (name, k, M, prec), flush=True)
    rng = np.random.default_rng(M + k)
    f = rng.standard_normal(shape)
    if prec == "f32":
        f = f.astype(np.float32).astype(np.float64)
    h = 1.0 / 512
    plan = Plan(shape, h, prec, pad=pad)
    plan.set_kernel(k, name)
    dt = torch.float64 if prec == "f64" else torch.float32
    u = plan.solve(torch.from_numpy(f).to("cuda", dt)).double().cpu().numpy()
    ref = oracle.solve(f, h, M=pad)
    err = float(np.abs(u - ref).max() / np.abs(ref).max())
    assert err < (1e-12 if prec == "f64" else 3e-6), (name, err)


def _x_cases():
    out = []
    for prec in ("f32", "f64"):
        for k in (0, 4):
            for nm in kernel_variants(k, prec, 1024):
                out.append((k, prec, nm))
    return out


try:
    X_CASES = _x_cases()
except Exception:  # library not built: collection must still work
    X_CASES = []


@pytest.mark.parametrize("k,prec,name", X_CASES)
@pytest.mark.parametrize("nx", [511, 301])
def test_x_pass_odd_row_length(k, prec, name, nx):
    """Odd nx: the packed row ends in a lone real value (scalar loads and stores)."""
    shape, pad = (6, 10, nx), (32, 32, 1024)
    print("[case] odd nx %d %s pass %d %s" % (nx, name, k, prec), flush=True)
    rng = np.random.default_rng(nx + k)
    f = rng.standard_normal(shape)
    if prec == "f32":
        f = f.astype(np.float32).astype(np.float64)
    h = 1.0 / nx
    plan = Plan(shape, h, prec, pad=pad)
    plan.set_kernel(k, name)
    dt = torch.float64 if prec == "f64" else torch.float32
    u = plan.solve(torch.from_numpy(f).to("cuda", dt)).double().cpu().numpy()
    ref = oracle.solve(f, h, M=pad)
    err = float(np.abs(u - ref).max() / np.abs(ref).max())
    assert err < (1e-12 if prec == "f64" else 3e-6), (name, err)
