"""The bench script's command line on a machine without a GPU: it measures
one GPU only and says so for any other count.  No GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_committed_traffic_record_is_well_formed():
    # per-launch HBM bytes of the dominant kernel, from the counter runs
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        rec = json.load(fh)
    assert isinstance(rec.get("source_hash"), str) and rec["source_hash"]
    assert rec["kernels"]
    for name, ent in rec["kernels"].items():
        # bytes of the main launch of a column pass, or of every launch
        b = ent.get("main_launch_bytes", ent.get("bytes_per_launch"))
        assert b is not None and float(b) > 0, name
