"""Benchmark of the free-space Poisson solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 512] [--no-cpu] [--no-f64]

One step = one forward solve u = h^2 G1 * f on the 512^3 grid in FP32 (the
five passes: x-forward, y-forward, z-convolution, y-inverse, x-inverse),
with f already resident in HBM.  G_hat is built once before timing (setup,
reported separately).  Prints ONE JSON line.

ms_per_step is K whole solves (the plan's own schedule) between two HIP events
on torch's current stream.  The per-pass durations come from a separate run of
K steps with HIP events recorded between the passes (each pass enqueued
alone); the roofline object uses the dominant pass.  The FP32 result is compared with the
FP64 GPU path on the same input (which the test suite pins to the CPU oracle
at <= 1e-12), and the CPU oracle is timed on a bounded sample on the host.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
VALU_FP32_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12   # 78.6, FP32 vector without packed math
PASS_NAMES = ("xfwd", "yfwd", "zconv", "yinv", "xinv")
KERNEL_SOURCES = ("paper_2512_08555_amd/csrc/passes_impl.hpp", "paper_2512_08555_amd/csrc/passes_f32.hip",
                  "paper_2512_08555_amd/csrc/passes_f32m.hip", "paper_2512_08555_amd/csrc/passes_f64.hip",
                  "paper_2512_08555_amd/csrc/zwave.hpp", "paper_2512_08555_amd/csrc/ywave.hpp",
                  "paper_2512_08555_amd/csrc/xwave.hpp", "paper_2512_08555_amd/csrc/ztab.hpp",
                  "paper_2512_08555_amd/csrc/dft.hpp",
                  "paper_2512_08555_amd/csrc/cplx.hpp")


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_name, model_bytes, share=1.0):
    """HBM bytes per main launch measured by rocprofv3 counters (FETCH_SIZE +
    WRITE_SIZE, scaled by the copy-kernel calibration), if the committed
    profile matches the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = rec.get("kernels", {}).get(kernel_name)
    if not ent or rec.get("source_hash") != kernel_source_hash():
        return None
    if "main_launch_bytes" in ent:
        return float(ent["main_launch_bytes"])
    return float(ent["bytes_per_launch"]) * share


def time_passes(plan, f, u, steps, warmup):
    import torch
    for _ in range(warmup):
        plan.solve(f, out=u)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)]
    t0 = time.perf_counter()
    for s in range(steps):
        e = ev[s]
        e[0].record(stream)
        plan.run_pass(0, f=f)
        e[1].record(stream)
        plan.run_pass(1)
        e[2].record(stream)
        plan.run_pass(2)
        e[3].record(stream)
        plan.run_pass(3)
        e[4].record(stream)
        plan.run_pass(4, u=u)
        e[5].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_pass = np.zeros(5)
    total = 0.0
    for s in range(steps):
        for k in range(5):
            per_pass[k] += ev[s][k].elapsed_time(ev[s][k + 1])
        total += ev[s][0].elapsed_time(ev[s][5])
    return per_pass / steps, total / steps, wall


def time_solve(plan, f, u, steps, warmup):
    """Whole solves (ups_solve, the plan's own schedule) timed with HIP events
    on torch's current stream: ms per solve over `steps` solves."""
    import torch
    for _ in range(warmup):
        plan.solve(f, out=u)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan.solve(f, out=u)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def cpu_baseline(n_sample=512, budget_s=10.0, max_reps=8):
    """The CPU oracle (scipy.fft, FP64) on a bounded sample of the headline
    workload: whole n_sample^3 solves of the same source recipe, repeated
    until about `budget_s` of CPU work (G_hat precomputed, outside the timed
    region).  Threads: the host's CPUs available to this process, at most 16
    (the CPU share of one GPU on the measurement hosts)."""
    import oracle
    from paper_2512_08555_amd import workloads
    visible = len(os.sched_getaffinity(0))
    workers = min(visible, 16)
    h = 1.0 / n_sample
    f = workloads.config_blobs_noise(n_sample, 2)
    M = (2 * n_sample,) * 3
    G = oracle.green_spectrum_raw(M)
    reps, dt = 0, 0.0
    while reps < max_reps and (dt < budget_s or reps < 1):
        t0 = time.perf_counter()
        oracle.solve(f, h, G_hat_raw=G, workers=workers)
        dt += time.perf_counter() - t0
        reps += 1
    return {"value": reps * n_sample ** 3 / dt, "unit": "grid points/s", "cores": workers,
            "host_cpus_visible": visible, "kind": "oracle",
            "sample": "%d whole solves of the %d^3 FP64 blob-plus-noise source by oracle.solve (pruned "
                      "scipy.fft, %d threads), G_hat precomputed; %.1f s" % (reps, n_sample, workers, dt)}


def batch_leg(reps=10):
    """The uneven batch (48 solves of 32..192 points per axis + a 3-component
    128^3 curl source, FP32): one graph launch vs a loop of per-problem
    plans running the same kernels eagerly."""
    import torch
    from paper_2512_08555_amd import workloads
    from paper_2512_08555_amd.solver import Batch, Plan
    cfg = workloads.config_c4()
    specs = [dict(shape=p["shape"], h=p["h"], prec="f32") for p in cfg["scalar"]]
    specs.append(dict(shape=cfg["vector"]["shape"], h=cfg["vector"]["h"], prec="f32", ncomp=3))
    fs = [torch.from_numpy(p["f"].astype(np.float32)).cuda() for p in cfg["scalar"]]
    fs.append(torch.from_numpy(cfg["vector"]["f"].astype(np.float32)).cuda())
    t0 = time.perf_counter()
    b = Batch(specs)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    us = b.empty_outputs()
    plans = [Plan(sp["shape"], sp["h"], "f32", ncomp=sp["ncomp"], pad=sp["pad"]) for sp in b.specs]
    pts = sum(int(np.prod(sp["shape"])) * sp["ncomp"] for sp in b.specs)
    stream = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    graph_ms = timed(lambda: b.solve(fs, us))
    loop_ms = timed(lambda: [p.solve(f, out=u) for p, f, u in zip(plans, fs, us)])
    # algorithmic HBM bytes of the whole batch: each problem's five-pass model
    # at its own padded lengths
    model = float(sum(p.model_bytes(-1) for p in plans))
    del plans
    torch.cuda.empty_cache()
    # the plain FP64 GPU path on the same problems: one FP64 plan per problem
    # (lengths padded to the FP64 kernels' sizes), solved one after another
    from paper_2512_08555_amd.lengths import auto_pad
    p64 = [Plan(sp["shape"], sp["h"], "f64", ncomp=sp["ncomp"], pad=auto_pad(sp["shape"], "f64"))
           for sp in b.specs]
    f64s = [f.double() for f in fs]
    u64s = [torch.empty_like(f) for f in f64s]
    loop64_ms = timed(lambda: [p.solve(f, out=u) for p, f, u in zip(p64, f64s, u64s)])
    worst = max(float((u.double() - r).abs().max() / r.abs().max()) for u, r in zip(us, u64s))
    gbs = model / (graph_ms * 1e-3) / 1e9
    return {"problems": len(specs), "points": pts, "graph_ms": graph_ms, "loop_ms": loop_ms,
            "graph_pts_per_s": pts / (graph_ms * 1e-3), "batched_speedup_over_loop": loop_ms / graph_ms,
            "f64_loop_ms": loop64_ms, "batched_speedup_over_f64_loop": loop64_ms / graph_ms,
            "rel_linf_vs_f64_worst": worst,
            "model_bytes": model, "hbm_gbs_model": gbs, "frac": gbs / HBM_PEAK_GBS,
            "launches_per_pass": b.launches(), "setup_ms": setup_ms}


def c2_leg(n=256, reps=10):
    """The plain FP64 GPU path on the 256^3 blob-plus-noise source (padded
    512^3): ms per whole solve, and its grid points per second."""
    import torch
    from paper_2512_08555_amd import workloads
    from paper_2512_08555_amd.solver import Plan
    f = torch.from_numpy(workloads.config_blobs_noise(n, 2)).cuda()
    plan = Plan((n, n, n), 1.0 / n, "f64")
    u = torch.empty_like(f)
    ms = time_solve(plan, f, u, reps, 3)
    return {"n": n, "precision": "f64", "ms_per_solve": ms, "pts_per_s": n ** 3 / (ms * 1e-3),
            "hbm_gbs_model": plan.model_bytes(-1) / (ms * 1e-3) / 1e9}


def variants_leg(n=512, reps=10):
    """The NEXT-row problem classes at the headline size (512^3 FP32, the
    headline source): the sixth-order Mehrstellen kernel (all unbounded),
    periodic z with unbounded x and y (the vortex-tube configuration), and
    an even z direction.  Setup (G_hat build) and whole-solve times beside
    the plain 7-point unbounded solve."""
    import torch
    from paper_2512_08555_amd import workloads
    from paper_2512_08555_amd.solver import Plan
    h = 1.0 / n
    f = torch.from_numpy(workloads.config_blobs_noise(n, 2).astype(np.float32)).cuda()
    u = torch.empty_like(f)
    out = {}
    cases = (("lgf2_unbounded", dict()),
             ("mehr6_unbounded", dict(green="mehr6")),
             ("per_z_unb_xy", dict(bc=("per", "unb", "unb"), pad=(2 * n, 2 * n, 2 * n))),
             ("even_z_unb_xy", dict(bc=("even", "unb", "unb"), pad=(2 * n, 2 * n, 2 * n))))
    for name, kw in cases:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = Plan((n, n, n), h, "f32", **kw)
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
        ms = time_solve(plan, f, u, reps, 3)
        out[name] = {"setup_ms": setup_ms, "ms_per_solve": ms, "pts_per_s": n ** 3 / (ms * 1e-3),
                     "kernels": [plan.kernel(k) for k in range(5)]}
        del plan
        torch.cuda.empty_cache()
    return out


def grad_leg(n=256, reps=5):
    """Differentiable workload: 256^3 FP32 forward solve + loss + backward
    through the hand-written adjoint (torch.autograd)."""
    import torch
    from paper_2512_08555_amd import workloads
    from paper_2512_08555_amd.autograd import poisson_solve
    from paper_2512_08555_amd.solver import Plan
    h = 1.0 / n
    f = torch.from_numpy(workloads.config_blobs_noise(n, 5).astype(np.float32)).cuda()
    w = torch.from_numpy(workloads.weight_field(n, h, seed=55).astype(np.float32)).cuda()
    plan = Plan((n, n, n), h, "f32")
    inv = 1.0 / (2.0 * h)

    def step():
        fr = f.detach().requires_grad_(True)
        u = poisson_solve(fr, plan)
        dx = (u[1:-1, 1:-1, 2:] - u[1:-1, 1:-1, :-2]) * inv
        dy = (u[1:-1, 2:, 1:-1] - u[1:-1, :-2, 1:-1]) * inv
        dz = (u[2:, 1:-1, 1:-1] - u[:-2, 1:-1, 1:-1]) * inv
        L = h ** 3 * (w[1:-1, 1:-1, 1:-1] * (dx * dx + dy * dy + dz * dz)).sum()
        L.backward()
        return fr.grad

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    return {"n": n, "fwd_bwd_ms": ms, "solves_per_step": 2}


def calibrate_copy(nbytes=2 << 30, reps=3):
    """A plain copy of known size (reads and writes nbytes each) whose
    FETCH_SIZE / WRITE_SIZE readings calibrate the HBM counters."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        torch.add(a, 0.0, out=b)
    torch.cuda.synchronize()
    return {"bytes": nbytes, "reps": reps, "grid_elements": a.numel()}


def mg_leg(n=512, prec="f32", reps=5):
    """The multigrid V(2, 2) cycle (Sec. 3.1) around the solve: level 0 the
    n^3 grid solved by the FFT plan, level 1 a (n + 1)^3 box over the
    central half at spacing h / 2, each level with its own seeded
    blob-plus-noise source (a timing workload: the values do not change the
    work).
    ms per cycle (HIP events on the caller's stream), and the composite
    residual's reduction per cycle from zero."""
    import torch
    from paper_2512_08555_amd import workloads
    from paper_2512_08555_amd.solver import Multigrid, Plan
    h0 = 1.0 / n
    dt = torch.float64 if prec == "f64" else torch.float32
    plan = Plan((n, n, n), h0, prec)
    mg = Multigrid(plan, [((n // 4,) * 3, (n // 2,) * 3)])
    f0 = torch.from_numpy(workloads.config_blobs_noise(n, 2)).to("cuda", dt)
    f1 = torch.from_numpy(workloads.config_blobs_noise(n + 1, 3)).to("cuda", dt) * 0.25
    fs = [f0, f1]
    us = mg.zeros()
    res = [max(mg.residuals(fs, us))]
    for _ in range(3):
        mg.cycle(fs, us, 2, 2)
        res.append(max(mg.residuals(fs, us)))
    stream = torch.cuda.current_stream()
    out = {"levels": [list(s) for s in mg.shapes], "precision": prec,
           "residual_per_cycle": [float(r) for r in res],
           "rate": float((res[-1] / res[1]) ** 0.5) if res[1] > 0 else None}
    for nu in ((2, 2), (1, 1)):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            mg.cycle(fs, us, *nu)
        e1.record(stream)
        torch.cuda.synchronize()
        out["ms_per_cycle_V%d%d" % nu] = e0.elapsed_time(e1) / reps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    u0 = torch.empty_like(f0)
    e0.record(stream)
    for _ in range(reps):
        plan.solve(f0, out=u0)
    e1.record(stream)
    torch.cuda.synchronize()
    out["level0_solve_ms"] = e0.elapsed_time(e1) / reps
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--seed", type=int, default=2, help="seed of the headline source (blobs plus noise)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-mg", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the Mehrstellen / periodic / even leg")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 2 GiB copy kernel (for counter calibration runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (--gpus must be 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2512_08555_amd import workloads
    from paper_2512_08555_amd.solver import Plan

    n = args.n
    h = 1.0 / n
    f64 = workloads.config_blobs_noise(n, args.seed)
    f32_host = f64.astype(np.float32)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    t0 = time.perf_counter()
    plan = Plan((n, n, n), h, "f32")
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    f = torch.from_numpy(f32_host).to(dev)
    u = torch.empty_like(f)
    step_ms = time_solve(plan, f, u, args.steps, args.warmup)
    per_pass, _, _ = time_passes(plan, f, u, args.steps, 2)
    value = n ** 3 / (step_ms * 1e-3)
    dom = int(np.argmax(per_pass))
    dom_name = plan.kernel(dom)
    # With column 0 carrying the Nyquist column (ups_plan_nyquist_packed, the
    # 512^3 FP32 plan), each column pass runs one launch over its kx - 1
    # columns, the z pass with its pair launch for column 0 beside it, joined
    # before the pass ends: the events around the pass time all of it, and
    # its algorithmic bytes are the whole pass's (all kx x-frequencies).
    # Otherwise a column pass (1-3) runs one main launch over the first kmain
    # of the kx columns (a multiple of 8 XCDs x the columns of one 128-byte
    # line) and a narrow launch over the rest on the plan's second stream,
    # alongside it; the events then time the main launch.  Every term of a
    # column pass's byte model is linear in the number of columns, so the
    # main launch's algorithmic bytes are the pass's times kmain / kx.
    packed = plan.nyquist_packed
    m = 2 * n
    kx = m // 2 + 1
    align = 8 * (128 // 8)   # 8 XCDs x 16 complex floats per 128-byte line
    kzm = kx if packed else kx // align * align
    kmain = kzm if dom in (1, 2, 3) else kx
    dom_bytes = plan.model_bytes(dom) * kmain / kx
    achieved = dom_bytes / (per_pass[dom] * 1e-3) / 1e9
    # The z pass is bound by vector-ALU issue rather than by HBM: its roofline
    # against the FP32 vector peak without packed math.  Flops per line of the
    # main launch (kmain * m lines), radix-2 count of the pruned transforms:
    # forward 5 m log2 m - 2 m (the first layer's partners are the zero
    # padding: one complex product per pair instead of a butterfly), inverse
    # 5 m log2 m - m (the last layer keeps half its outputs), plus 2 m for
    # the real G_hat scaling.
    z_flops = kzm * m * ((5.0 * m * np.log2(m) - 2.0 * m) + (5.0 * m * np.log2(m) - m) + 2.0 * m)
    z_tflops = z_flops / (per_pass[2] * 1e-3) / 1e12
    traffic = load_traffic(dom_name, dom_bytes, kmain / kx)
    total_bytes = plan.model_bytes(-1)
    kernels = [plan.kernel(k) for k in range(5)]

    extra = {}
    if not args.no_f64:
        u32 = plan.solve(f).double()
        del plan
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
        p64 = Plan((n, n, n), h, "f64")
        torch.cuda.synchronize()
        setup64 = (time.perf_counter() - t0) * 1e3
        fd = f.double()   # the same (FP32-rounded) input
        ud = torch.empty_like(fd)
        step64 = time_solve(p64, fd, ud, max(3, args.steps // 2), 2)
        pp64, _, _ = time_passes(p64, fd, ud, max(3, args.steps // 2), 2)
        ref = ud
        d = (u32 - ref)
        extra = {
            "f64_pts_per_s": n ** 3 / (step64 * 1e-3),
            "f64_ms_per_step": step64,
            "f64_setup_ms": setup64,
            "f32_speedup_over_f64": step64 / step_ms,
            "f32_rel_linf_vs_f64": float(d.abs().max() / ref.abs().max()),
            "f32_rel_l2_vs_f64": float(d.norm() / ref.norm()),
            "f64_pass_ms": dict(zip(PASS_NAMES, [round(float(x), 4) for x in pp64])),
        }
        del p64

    if not args.no_f64:
        extra["c2_f64_256"] = c2_leg()
        torch.cuda.empty_cache()
    if not args.no_batch:
        extra["batch"] = batch_leg()
        torch.cuda.empty_cache()
    if not args.no_grad:
        extra["grad_256"] = grad_leg()
        torch.cuda.empty_cache()
    if not args.no_mg:
        extra["multigrid"] = mg_leg(n)
        torch.cuda.empty_cache()
    if not args.no_variants:
        extra["problem_classes"] = variants_leg(n)
        torch.cuda.empty_cache()
    if args.calibrate_copy:
        extra["copy_calibration"] = calibrate_copy()

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(n)

    out = {
        "metric": "grid points/s (512^3 unbounded Poisson solve, FP32)",
        "value": value,
        "unit": "grid points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (16 seeded Gaussian blobs + 1e-3 zero-mean noise)",
        "config": {"workload": "free-space Poisson solve, %d^3 cell-centred grid, FP32, "
                               "padded %d^3 FFT convolution with the 7-point LGF" % (n, 2 * n),
                   "n": n, "padded": 2 * n, "precision": "f32"},
        "hbm_gbs_model": total_bytes / (step_ms * 1e-3) / 1e9,
        "model_bytes_per_step": total_bytes,
        "pass_ms": dict(zip(PASS_NAMES, [round(float(x), 4) for x in per_pass])),
        "kernels": kernels,
        "setup_ms": setup_ms,
        "roofline_alu_zconv": {"bound": "alu", "achieved": z_tflops, "peak": VALU_FP32_PEAK_TFLOPS,
                               "unit": "TFLOP/s", "frac": z_tflops / VALU_FP32_PEAK_TFLOPS,
                               "flops_per_launch": z_flops,
                               "peak_basis": "256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz, FP32 without packed math"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom_name,
                     "launch_ms": round(float(per_pass[dom]), 4),
                     "algorithmic_bytes_per_launch": dom_bytes,
                     "columns_per_launch": ("all %d (column 0 carries the Nyquist column)" % kx if packed
                                            else "%d of %d" % (kmain, kx))},
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
