"""Mehrstellen kernels (eqs. mehrstellen_discr4/6) on the GPU through the C
ABI: the Green's spectrum and solves against the oracle, and the fourth-
and sixth-order convergence the paper states (Sec. 4) on its bump."""
import numpy as np
import pytest
import torch

from oracle import analytic, mehrstellen as oms
from paper_2512_08555_amd import workloads
from paper_2512_08555_amd.solver import Plan

pytestmark = pytest.mark.gpu


def _rel_inf(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _plan(shape, h, prec, order, pad=None):
    return Plan(shape, h, prec, pad=pad, green="mehr%d" % order)


@pytest.mark.parametrize("order", [4, 6])
@pytest.mark.parametrize("shape,pad", [((16, 16, 16), (32, 32, 32)), ((12, 20, 14), (32, 64, 32))])
def test_green_spectrum_matches_oracle(order, shape, pad):
    print("[case] mehrstellen %d ghat %s pad %s" % (order, shape, pad), flush=True)
    h = 1.0 / max(shape)
    plan = _plan(shape, h, "f64", order, pad=pad)
    got = plan.ghat().cpu().numpy()
    ref = oms.green_spectrum_raw(pad, order) * (h * h / float(np.prod(pad)))
    assert got.shape == ref.shape
    err = _rel_inf(got, ref)
    print("  rel Linf %.3e" % err, flush=True)
    assert err < 1e-13


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 2e-6)])
@pytest.mark.parametrize("order", [4, 6])
@pytest.mark.parametrize("shape", [(24, 30, 20), (32, 32, 32)])
def test_solve_matches_oracle(order, prec, tol, shape):
    print("[case] mehrstellen %d %s solve %s" % (order, prec, shape), flush=True)
    h = 1.0 / max(shape)
    f = workloads.blob_source(shape, h, seed=order + shape[0], nblobs=6, sigma=(0.05, 0.12), noise=1e-3)
    if prec == "f32":
        f = f.astype(np.float32).astype(np.float64)
    from paper_2512_08555_amd.lengths import auto_pad
    pad = auto_pad(shape, prec)
    plan = _plan(shape, h, prec, order, pad=pad)
    dt = torch.float64 if prec == "f64" else torch.float32
    u = plan.solve(torch.from_numpy(f).to("cuda", dt)).double().cpu().numpy()
    ref = oms.solve(f, h, order, M=pad)
    err = _rel_inf(u, ref)
    print("  rel Linf %.3e" % err, flush=True)
    assert err < tol


@pytest.mark.parametrize("order,lo,hi", [(4, 3.9, 4.1), (6, 5.8, 6.2)])
def test_convergence_order_on_the_paper_bump(order, lo, hi):
    # E_inf proportional to h^M (Sec. 4) with the kernel R G_L: FP64 solves
    # of the compact manufactured solution at 32^3, 64^3 and 128^3
    errs = []
    for n in (32, 64, 128):
        print("[case] mehrstellen %d bump %d^3" % (order, n), flush=True)
        h = 1.0 / n
        x = (np.arange(n) + 0.5) * h
        plan = _plan((n, n, n), h, "f64", order)
        u = plan.solve(torch.from_numpy(analytic.bump_source(x, x, x)).cuda()).cpu().numpy()
        errs.append(np.abs(u - analytic.bump_solution(x, x, x)).max())
    p = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print("mehrstellen %d E_inf %s orders %s" % (order, errs, p), flush=True)
    assert lo < p[-1] < hi, (errs, p)
