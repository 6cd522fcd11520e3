"""The opt-in checks of the C ABI on the GPU: the non-finite input check and
the guard mode (canary bands around W, NaN poison of unwritten W)."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2512_08555_amd import workloads

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _announce(msg):
    print("[case]", msg, flush=True)


def test_nonfinite_input_is_refused():
    from paper_2512_08555_amd._capi import UPS_ERR_NONFINITE, UpsError
    from paper_2512_08555_amd.solver import Plan
    _announce("non-finite check 32^3 f32")
    cfg = workloads.config_c1()
    plan = Plan(cfg["shape"], cfg["h"], "f32")
    f = torch.from_numpy(cfg["f"].astype(np.float32)).cuda()
    ref = plan.solve(f)
    plan.set_check_finite(True)
    assert torch.equal(plan.solve(f), ref)          # finite input: same result
    for bad in (float("nan"), float("inf"), -float("inf")):
        g = f.clone()
        g[3, 17, 30] = bad
        u = torch.full_like(f, 7.0)
        with pytest.raises(UpsError) as ei:
            plan.solve(g, out=u)
        assert ei.value.status == UPS_ERR_NONFINITE
        assert torch.all(u == 7.0)                  # nothing was solved
    plan.set_check_finite(False)
    g = f.clone()
    g[0, 0, 0] = float("nan")
    plan.solve(g)                                   # unchecked: no error


_GUARD_CHILD = r"""
import sys
sys.path.insert(0, %(root)r)
import numpy as np, torch
import oracle
from paper_2512_08555_amd import workloads
from paper_2512_08555_amd._capi import UpsError, UPS_ERR_INTERNAL
from paper_2512_08555_amd.solver import Plan
cfg = workloads.config_c1()
for prec, tol in (("f64", 1e-12), ("f32", 2e-6)):
    plan = Plan(cfg["shape"], cfg["h"], prec)
    assert plan.guard_mode
    dt = torch.float64 if prec == "f64" else torch.float32
    fin = cfg["f"].astype(np.float32).astype(np.float64) if prec == "f32" else cfg["f"]
    f = torch.from_numpy(fin).to("cuda", dt)
    for rep in range(2):
        u = plan.solve(f).double().cpu().numpy()
        ref = oracle.solve(fin, cfg["h"])
        err = float(np.abs(u - ref).max() / np.abs(ref).max())
        assert err < tol, (prec, err)
    # a host write into the canary band above W is reported after the first pass
    lay = plan.layout()
    esz = 16 if prec == "f64" else 8
    wbytes = plan.ncomp * lay["comp_stride"] * esz
    wbytes = (wbytes + 255) // 256 * 256
    from paper_2512_08555_amd import _capi as capi
    woff = capi.lib().ups_plan_work_offset(plan._h)
    plan.work[woff + wbytes + 100] = 0
    try:
        plan.solve(f)
        raise SystemExit("canary damage not reported")
    except UpsError as e:
        assert e.status == UPS_ERR_INTERNAL and "above" in str(e), str(e)
print("GUARD_OK")
"""


def test_guard_mode_c1():
    """A C1-size plan created with UPS_DEBUG_GUARDS=1 (in a child process,
    the switch is read at plan creation) solves to the oracle's result with
    intact canary bands and no NaN poison in the output, twice; a byte of the
    upper band overwritten from the host is reported."""
    _announce("guard mode c1 (child process)")
    env = dict(os.environ)
    env["UPS_DEBUG_GUARDS"] = "1"
    r = subprocess.run([sys.executable, "-c", _GUARD_CHILD % {"root": ROOT}], env=env, capture_output=True,
                       text=True, timeout=110)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0 and "GUARD_OK" in r.stdout
