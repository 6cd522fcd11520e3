"""Host-side observability: roctx ranges are linked in, and UPS_LOG_LEVEL
controls the stderr log (errors at 1, plan, batch and cycle decisions at 2).
Each level runs in its own process, since the library reads the variable
once."""
import os
import subprocess
import sys

import pytest

PAD = None
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2512_08555_amd", "libups.so")

SCRIPT = r"""
import sys
sys.path.insert(0, %r)
from paper_2512_08555_amd.solver import Plan, Batch, Multigrid
from paper_2512_08555_amd.lengths import auto_pad
p = Plan((32, 36, 40), 0.05, "f32", pad=auto_pad((32, 36, 40), "f32"), setup=False)
print("pad", *auto_pad((32, 36, 40), "f32"))
Batch([dict(shape=(20, 30, 40), h=0.05), dict(shape=(16, 16, 16), h=1 / 16, prec="f64")], setup=False)
c = Plan((33, 33, 33), 1 / 32, "f64", pad=auto_pad((33, 33, 33), "f64"), setup=False)
Multigrid(c, [((8, 8, 8), (16, 16, 16))], setup=False)
try:
    Plan((40, 36, 1), 0.05, "f32", setup=False)   # fewer than 2 points: INVALID_ARG
except Exception as e:
    print("raised", type(e).__name__)
""" % ROOT


def _lib_or_skip():
    if not os.path.exists(LIB):
        pytest.skip("libups.so not built")


def _run(level):
    env = dict(os.environ)
    env.pop("UPS_LOG_LEVEL", None)
    if level is not None:
        env["UPS_LOG_LEVEL"] = str(level)
    r = subprocess.run([sys.executable, "-c", SCRIPT], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr
    assert "raised" in r.stdout
    global PAD
    PAD = [int(v) for v in r.stdout.split("pad", 1)[1].split()[:3]]   # (z, y, x)
    return [l for l in r.stderr.splitlines() if l.startswith("[ups] ")]


def test_library_calls_roctx():
    _lib_or_skip()
    out = subprocess.run(["readelf", "-d", "--dyn-syms", LIB], capture_output=True, text=True).stdout
    assert "librocprofiler-sdk-roctx.so" in out
    assert "roctxRangePushA" in out and "roctxRangePop" in out


def test_silent_by_default():
    _lib_or_skip()
    assert _run(None) == []
    assert _run(0) == []


def test_level_1_logs_failures_only():
    _lib_or_skip()
    lines = _run(1)
    assert lines and all(l.startswith("[ups] error 1: ") for l in lines)
    assert any("2" in l and "point" in l for l in lines), lines


def test_level_2_logs_plans_batches_and_cycles():
    _lib_or_skip()
    lines = _run(2)
    plans = [l for l in lines if l.startswith("[ups] plan ")]
    assert len(plans) == 2, lines
    assert "40 x 36 x 32" in plans[0] and "FP32" in plans[0]
    assert "padded %d x %d x %d" % (PAD[2], PAD[1], PAD[0]) in plans[0]
    for k in ("xfwd_float", "yfwd_float", "zconv_float", "yinv_float", "xinv_float"):
        assert k in plans[0]
    assert any(l.startswith("[ups] batch ") and "2 problems" in l for l in lines)
    assert sum(1 for l in lines if " pass " in l and l.startswith("[ups] batch ")) >= 5
    assert any(l.startswith("[ups] cycle ") and "1 refined level(s)" in l for l in lines)
    assert any("level 1: 33 x 33 x 33 nodes" in l for l in lines)
    assert any(l.startswith("[ups] error 1: ") for l in lines)
    assert not any(l.startswith("[ups] solve") for l in lines)   # level 3 only
