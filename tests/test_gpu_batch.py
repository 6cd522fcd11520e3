"""Batched solves (one hipGraph of grouped pass kernels), mixed-radix padded
lengths and the autotuner, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_2512_08555_amd import workloads

pytestmark = pytest.mark.gpu


def _announce(msg):
    print("[case]", msg, flush=True)


def _dev(a, prec):
    return torch.from_numpy(np.ascontiguousarray(a)).to(
        device="cuda", dtype=torch.float64 if prec == "f64" else torch.float32)


def _rel_inf(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("n", [40, 48, 72, 80, 96, 144, 160, 192])
def test_mixed_radix_lengths_f32(n):
    from paper_2512_08555_amd.lengths import auto_pad
    from paper_2512_08555_amd.solver import Plan
    shape = (n, max(2, n - 7), n // 2 + 3)
    pad = auto_pad(shape, "f32")
    _announce("mixed radix f32 %s pad %s" % (shape, pad))
    rng = np.random.default_rng(n)
    f = rng.standard_normal(shape).astype(np.float32).astype(np.float64)
    h = 1.0 / max(shape)
    plan = Plan(shape, h, "f32", pad=pad)
    u = plan.solve(_dev(f, "f32")).cpu().numpy().astype(np.float64)
    ref = oracle.solve(f, h, M=pad)
    assert _rel_inf(u, ref) < 3e-6


def _small_batch_specs():
    shapes = [(20, 33, 47), (40, 40, 40), (17, 64, 30), (33, 21, 20), (48, 12, 96), (40, 40, 40)]
    specs = [dict(shape=s, h=1.0 / max(s), prec="f32") for s in shapes]
    specs.append(dict(shape=(24, 24, 24), h=1.0 / 24, prec="f32", ncomp=3))
    specs.append(dict(shape=(16, 18, 20), h=0.05, prec="f64"))
    return specs


def test_batch_equals_single_plans_and_oracle():
    from paper_2512_08555_amd.solver import Batch, Plan
    specs = _small_batch_specs()
    _announce("batch of %d" % len(specs))
    b = Batch(specs)
    assert all(n >= 1 for n in b.launches())
    rng = np.random.default_rng(1)
    fs_host, fs = [], []
    for sp in b.specs:
        shape = sp["shape"] if sp["ncomp"] == 1 else (sp["ncomp"],) + sp["shape"]
        a = rng.standard_normal(shape)
        if sp["prec"] == "f32":
            a = a.astype(np.float32).astype(np.float64)
        fs_host.append(a)
        fs.append(_dev(a, sp["prec"]))
    us = b.solve(fs)
    torch.cuda.synchronize()
    first = [u.clone() for u in us]
    for i, sp in enumerate(b.specs):
        p = Plan(sp["shape"], sp["h"], sp["prec"], ncomp=sp["ncomp"], pad=sp["pad"])
        ref_gpu = p.solve(fs[i]).cpu().numpy()
        got = us[i].cpu().numpy()
        assert np.array_equal(got, ref_gpu), "batch differs from single plan for problem %d" % i
        tol = 1e-12 if sp["prec"] == "f64" else 3e-6
        fh = fs_host[i] if sp["ncomp"] == 1 else fs_host[i]
        if sp["ncomp"] == 1:
            assert _rel_inf(got.astype(np.float64), oracle.solve(fh, sp["h"], M=sp["pad"])) < tol
        else:
            for c in range(sp["ncomp"]):
                assert _rel_inf(got[c].astype(np.float64), oracle.solve(fh[c], sp["h"], M=sp["pad"])) < tol
    # graph replays with eager work in between give the same result every time
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda") * 2.0
        junk.sum().item()
        us2 = b.solve(fs)
        torch.cuda.synchronize()
        for a, c in zip(us2, first):
            assert torch.equal(a, c), "replay %d differs" % rep


def test_batch_c4_workload_smoke():
    """The uneven-size workload (48 solves of 32..192 points per axis plus a
    3-component 128^3 curl source): every problem against the FP64 oracle
    (every component of the vector source), and a sample bitwise against
    single-plan solves."""
    from paper_2512_08555_amd.solver import Batch, Plan
    cfg = workloads.config_c4()
    specs = [dict(shape=p["shape"], h=p["h"], prec="f32") for p in cfg["scalar"]]
    specs.append(dict(shape=cfg["vector"]["shape"], h=cfg["vector"]["h"], prec="f32", ncomp=3))
    _announce("c4 batch %d problems" % len(specs))
    b = Batch(specs)
    fs = [_dev(p["f"], "f32") for p in cfg["scalar"]] + [_dev(cfg["vector"]["f"], "f32")]
    us = b.solve(fs)
    torch.cuda.synchronize()
    for i in (0, 7, 23, 47, 48):
        sp = b.specs[i]
        p = Plan(sp["shape"], sp["h"], "f32", ncomp=sp["ncomp"], pad=sp["pad"])
        assert torch.equal(p.solve(fs[i]), us[i])
    worst = 0.0
    for i, sp in enumerate(b.specs):
        f = fs[i].double().cpu().numpy()
        got = us[i].double().cpu().numpy()
        comps = [(got, f)] if sp["ncomp"] == 1 else [(got[c], f[c]) for c in range(sp["ncomp"])]
        for g, fc in comps:
            err = _rel_inf(g, oracle.solve(fc, sp["h"], M=sp["pad"]))
            worst = max(worst, err)
            assert err < 3e-6, "problem %d %s: rel Linf %.3e" % (i, sp["shape"], err)
    print("c4: worst rel Linf over 49 problems %.3e" % worst, flush=True)


def test_autotune_keeps_results_correct(tmp_path, monkeypatch):
    from paper_2512_08555_amd.solver import Plan
    _announce("autotune 64^3 f32")
    rng = np.random.default_rng(2)
    f = rng.standard_normal((64, 64, 64)).astype(np.float32).astype(np.float64)
    plan = Plan((64, 64, 64), 1 / 64, "f32")
    names = plan.autotune(budget_ms=50.0)
    assert all(isinstance(n, str) for n in names)
    u = plan.solve(_dev(f, "f32")).cpu().numpy().astype(np.float64)
    assert _rel_inf(u, oracle.solve(f, 1 / 64)) < 3e-6


def test_autotune_pipelined_fp64_plan():
    # an FP64 plan with 513 x-frequencies runs the two-stream slab schedule;
    # tuning times whole solves in that schedule and keeps results correct
    from paper_2512_08555_amd.solver import Plan
    _announce("autotune 24x24x300 f64 pipelined")
    rng = np.random.default_rng(3)
    shape, pad = (24, 24, 300), (64, 64, 1024)
    f = rng.standard_normal(shape)
    plan = Plan(shape, 1 / 300, "f64", pad=pad)
    assert plan.slab == 128
    names = plan.autotune(budget_ms=200.0)
    assert len(names) == 5 and all(isinstance(n, str) for n in names)
    u = plan.solve(_dev(f, "f64")).cpu().numpy()
    assert _rel_inf(u, oracle.solve(f, 1 / 300, M=pad)) < 1e-12
