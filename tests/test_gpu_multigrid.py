"""The multigrid V-cycle around the solve (Sec. 3.1, Alg. amg_vcycle) through
the C ABI, against the oracle's cycle (oracle/multigrid.py) from the same
start, and against the composite equations its fixed point satisfies."""
import numpy as np
import pytest
import torch

from oracle import multigrid as omg
from paper_2512_08555_amd.lengths import auto_pad
from paper_2512_08555_amd.solver import Multigrid, Plan

pytestmark = pytest.mark.gpu

H0 = 0.1
# (level-0 nodes (z, y, x), boxes [(origin, cells), ...] in (z, y, x))
SMALL = [((12, 11, 13), [((3, 2, 4), (4, 5, 4))]),
         ((13, 12, 14), [((3, 3, 3), (6, 5, 7)), ((2, 2, 3), (6, 6, 5))]),
         ((9, 9, 9), [((1, 1, 1), (6, 6, 6))]),
         ((10, 12, 9), [])]
# level arrays spanning several 64-wide tiles with ragged tails, three levels
LARGE = ((64, 56, 72), [((10, 12, 14), (40, 30, 50)), ((6, 5, 7), (60, 40, 70))])
TOL = {"f64": 1e-12, "f32": 2e-5}


def _setup(n0, patches, prec, seed):
    rng = np.random.default_rng(seed)
    shapes = omg.level_shapes(n0, patches)
    fs = [rng.standard_normal(s) for s in shapes]
    u0 = [0.01 * rng.standard_normal(s) for s in shapes]
    if prec == "f32":
        fs = [f.astype(np.float32).astype(np.float64) for f in fs]
        u0 = [u.astype(np.float32).astype(np.float64) for u in u0]
    plan = Plan(n0, H0, prec, pad=auto_pad(n0, prec))
    mg = Multigrid(plan, patches)
    assert mg.shapes == [tuple(s) for s in shapes]
    dt = plan.dtype
    fd = [torch.from_numpy(f).to("cuda", dt) for f in fs]
    ud = [torch.from_numpy(u).to("cuda", dt) for u in u0]
    return mg, fs, u0, fd, ud


def _compare(ud, us):
    scale = max(np.abs(u).max() for u in us)
    return max(float(np.abs(a.double().cpu().numpy() - b).max()) for a, b in zip(ud, us)) / scale


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("case", range(len(SMALL)))
def test_cycles_match_the_oracle(case, prec):
    n0, patches = SMALL[case]
    print("[case] multigrid %s %s %s" % (prec, n0, patches), flush=True)
    mg, fs, u0, fd, ud = _setup(n0, patches, prec, 10 + case)
    us = [u.copy() for u in u0]
    # odd and even counts on both legs: the pre-smoothed values end in u or
    # in the level's scratch array, and the prolongation writes into either
    for cyc, nu in enumerate([(2, 2), (1, 0), (0, 3), (3, 1), (1, 2)]):
        mg.cycle(fd, ud, *nu)
        omg.vcycle(us, fs, patches, H0, *nu)
        err = _compare(ud, us)
        print("  cycle %d V%s rel err %.2e" % (cyc, nu, err), flush=True)
        assert err < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_large_hierarchy_matches_the_oracle(prec):
    n0, patches = LARGE
    print("[case] multigrid %s %s %s" % (prec, n0, patches), flush=True)
    mg, fs, u0, fd, ud = _setup(n0, patches, prec, 20)
    us = [u.copy() for u in u0]
    for _ in range(2):
        mg.cycle(fd, ud, 2, 2)
        omg.vcycle(us, fs, patches, H0, 2, 2)
    err = _compare(ud, us)
    print("  rel err %.2e" % err, flush=True)
    assert err < TOL[prec]
    res = mg.residuals(fd, ud)
    ref = omg.composite_residuals(us, fs, patches, H0)
    scale = max(np.abs(f).max() for f in fs)
    assert max(abs(a - b) for a, b in zip(res, ref)) < (1e-9 if prec == "f64" else 1e-3) * scale


def test_residual_norms_match_the_oracle():
    n0, patches = SMALL[1]
    mg, fs, u0, fd, ud = _setup(n0, patches, "f64", 30)
    us = [u.copy() for u in u0]
    mg.cycle(fd, ud, 1, 1)
    omg.vcycle(us, fs, patches, H0, 1, 1)
    res = mg.residuals(fd, ud)
    ref = omg.composite_residuals(us, fs, patches, H0)
    print("[case] residual norms gpu %s oracle %s" % (res, ref), flush=True)
    assert all(abs(a - b) <= 1e-10 * max(np.abs(f).max() for f in fs) for a, b in zip(res, ref))
    assert res[0] < 1e-12 and min(res[1:]) > 1e-6


def test_fixed_point_is_the_composite_solution():
    # 14 cycles from zero reach the dense solve of the composite equations
    n0, patches = SMALL[0]
    mg, fs, _, fd, _ = _setup(n0, patches, "f64", 40)
    ud = mg.zeros()
    hist = []
    for _ in range(14):
        mg.cycle(fd, ud, 2, 2)
        hist.append(max(mg.residuals(fd, ud)))
    u0, u1 = omg.composite_dense(fs, patches[0], H0)
    scale = np.abs(u1).max()
    e0 = np.abs(ud[0].cpu().numpy() - u0).max() / scale
    e1 = np.abs(ud[1].cpu().numpy() - u1).max() / scale
    print("[case] composite fixed point: %.2e %.2e, residuals %s" % (e0, e1, ["%.1e" % h for h in hist]), flush=True)
    assert e0 < 1e-11 and e1 < 1e-11
    rates = np.array(hist[1:6]) / np.array(hist[:5])
    assert rates.max() < 0.1


def test_three_levels_converge_on_the_paper_bump():
    # level 0 on [0, 1]^3 (65^3 nodes), boxes on [1/4, 3/4]^3 and
    # [3/8, 5/8]^3: the composite residual falls by more than 10 per cycle
    # and the solution reaches the manufactured one to second-order accuracy
    from oracle import analytic
    n = 64
    h0 = 1.0 / n
    patches = [((16, 16, 16), (32, 32, 32)), ((16, 16, 16), (32, 32, 32))]
    axes = [np.arange(n + 1) * h0, 0.25 + np.arange(n + 1) * h0 / 2, 0.375 + np.arange(n + 1) * h0 / 4]
    plan = Plan((n + 1,) * 3, h0, "f64", pad=auto_pad((n + 1,) * 3, "f64"))
    mg = Multigrid(plan, patches)
    fd = [torch.from_numpy(analytic.bump_source(a, a, a)).cuda() for a in axes]
    ud = mg.zeros()
    hist = []
    for _ in range(10):
        mg.cycle(fd, ud, 2, 2)
        hist.append(max(mg.residuals(fd, ud)))
    errs = [float(np.abs(u.cpu().numpy() - analytic.bump_solution(a, a, a)).max()) for u, a in zip(ud, axes)]
    print("[case] bump, 3 levels: residuals %s errors %s" % (["%.1e" % h for h in hist], errs), flush=True)
    assert hist[-1] < 1e-9 * max(float(f.abs().max()) for f in fd)
    assert max(np.array(hist[1:5]) / np.array(hist[:4])) < 0.1
    assert max(errs) < 6e-4


def test_second_order_on_a_gaussian_with_two_boxes():
    # nested boxes on [1/4, 3/4]^3 and [3/8, 5/8]^3 around a Gaussian charge:
    # the composite error against the erf potential falls as h0^2 from
    # 65^3 to 129^3 level-0 nodes
    from oracle import analytic
    errs = []
    for n in (64, 128):
        h0 = 1.0 / n
        patches = [((n // 4,) * 3, (n // 2,) * 3)] * 2
        plan = Plan((n + 1,) * 3, h0, "f64", pad=auto_pad((n + 1,) * 3, "f64"))
        mg = Multigrid(plan, patches)
        fd, ref = [], []
        o, h = 0.0, h0
        for s in mg.shapes:
            a = o + np.arange(s[0]) * h
            Z, Y, X = np.meshgrid(a, a, a, indexing="ij")
            fd.append(torch.from_numpy(analytic.gaussian_source(X, Y, Z, (0.5, 0.5, 0.5), 0.1, 1.0)).cuda())
            ref.append(analytic.gaussian_potential(X, Y, Z, (0.5, 0.5, 0.5), 0.1, 1.0))
            o, h = o + (n // 4) * h, h / 2
        ud = mg.zeros()
        for _ in range(10):
            mg.cycle(fd, ud, 2, 2)
        res = mg.residuals(fd, ud)
        errs.append(max(float(np.abs(u.cpu().numpy() - r).max()) for u, r in zip(ud, ref)) / np.abs(ref[0]).max())
        print("[case] gaussian, n0 %d: rel err %.3e residuals %s" % (n, errs[-1], res), flush=True)
        assert max(res) < 1e-9 * float(fd[0].abs().max())
    p = np.log2(errs[0] / errs[1])
    assert 1.85 < p < 2.3, (errs, p)


def test_cycle_with_a_periodic_coarse_plan():
    # level 0 periodic along z and unbounded in x and y (eq. 2unbkernel):
    # the boxes sit strictly inside level 0, so the cycle is unchanged and
    # only the direct solve on level 0 differs
    from oracle import bc as obc
    n0, patches = (16, 13, 14), [((4, 3, 3), (6, 5, 6))]
    bc = ("per", "unb", "unb")
    rng = np.random.default_rng(50)
    shapes = omg.level_shapes(n0, patches)
    fs = [rng.standard_normal(s) for s in shapes]
    pad = (32,) + tuple(auto_pad(n0, "f64")[1:])
    plan = Plan(n0, H0, "f64", pad=pad, bc=bc)
    mg = Multigrid(plan, patches)
    print("[case] multigrid, periodic z coarse plan %s pad %s" % (n0, pad), flush=True)
    fd = [torch.from_numpy(f).cuda() for f in fs]
    ud = mg.zeros()
    us = [np.zeros(s) for s in shapes]
    coarse = lambda f, h: obc.solve_bc(f, h, bc, M=pad)
    for _ in range(3):
        mg.cycle(fd, ud, 2, 2)
        omg.vcycle(us, fs, patches, H0, 2, 2, coarse_solve=coarse)
    err = _compare(ud, us)
    print("  rel err %.2e" % err, flush=True)
    assert err < 1e-12


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_wide_level_matches_the_oracle(prec):
    # a refined level 257 nodes wide along x: the fused smoother's widest
    # tiles (256 x 8 in FP32, 128 x 16 in FP64) and a 33 x 41 ragged y-z section
    n0 = (30, 24, 140)
    patches = [((4, 4, 5), (20, 16, 128))]
    print("[case] multigrid wide level %s %s %s" % (prec, n0, patches), flush=True)
    mg, fs, u0, fd, ud = _setup(n0, patches, prec, 60)
    assert mg.shapes[1] == (41, 33, 257)
    us = [u.copy() for u in u0]
    for nu in [(2, 2), (1, 1)]:
        mg.cycle(fd, ud, *nu)
        omg.vcycle(us, fs, patches, H0, *nu)
    err = _compare(ud, us)
    print("  rel err %.2e" % err, flush=True)
    assert err < TOL[prec]
