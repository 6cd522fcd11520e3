"""The C-ABI host code under AddressSanitizer and UndefinedBehaviorSanitizer.

`python -m paper_2512_08555_amd.build --sanitize` builds libups_san.so: the
plan, validation, batch, autotuner and multigrid sources (capi.cpp,
batch.cpp, autotune.cpp, mg_capi.cpp) instrumented on the host pass only,
linked with the regular kernel objects.  This test runs the CPU tests of the
C ABI (test_capi_cpu.py, test_lane_offsets.py, test_mg_cpu.py,
test_nyquist_cpu.py) against that library in a child process with the
sanitizer runtime preloaded; any report aborts the child.
Skipped when the sanitized library has not been built."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_LIB = os.path.join(ROOT, "paper_2512_08555_amd", "libups_san.so")


def _asan_runtime():
    r = subprocess.run(["/opt/rocm/llvm/bin/clang", "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_capi_cpu_tests_under_asan_ubsan():
    if not os.path.exists(SAN_LIB):
        pytest.skip("libups_san.so not built (python -m paper_2512_08555_amd.build --sanitize)")
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no ASan runtime found")
    env = dict(os.environ)
    env.update({
        "UPS_LIB": "libups_san.so",
        "LD_PRELOAD": rt,
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_capi_cpu.py"), os.path.join(ROOT, "tests", "test_lane_offsets.py"),
           os.path.join(ROOT, "tests", "test_mg_cpu.py"), os.path.join(ROOT, "tests", "test_nyquist_cpu.py")]
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=600, cwd=ROOT)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
