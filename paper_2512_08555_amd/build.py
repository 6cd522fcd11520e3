"""Build libups.so (HIP, gfx950 only) in-tree.

    python -m paper_2512_08555_amd.build [-v] [--incremental] [--sanitize]

Each source is compiled to an object with hipcc in parallel, then linked into
paper_2512_08555_amd/libups.so.  Packed-FP32 instructions are disabled for
all device code.

--incremental recompiles only sources older than their object or than any
header; the default (and build()) compiles everything.

--sanitize builds libups_san.so instead: the host-side sources of the C ABI
(capi.cpp, batch.cpp, autotune.cpp) compiled with AddressSanitizer and
UndefinedBehaviorSanitizer on the host pass only (-Xarch_host before each
-fsanitize=), linked with the regular objects of the kernel sources.  It is
loaded by tests/test_capi_sanitized.py with the sanitizer runtime preloaded.
"""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libups.so")
OUT_SAN = os.path.join(PKG, "libups_san.so")
OBJ = os.path.join(PKG, "_build")
OBJ_SAN = os.path.join(OBJ, "san")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["passes_f32.hip", "passes_f32m.hip", "passes_f64.hip", "passes.cpp", "green.hip", "debug.hip",
           "multigrid.hip", "capi.cpp", "batch.cpp", "autotune.cpp", "mg_capi.cpp", "trace.cpp"]
HOST_SOURCES = ["capi.cpp", "batch.cpp", "autotune.cpp", "mg_capi.cpp", "trace.cpp"]
# roctx ranges (trace.hpp); the library's run path already holds the ROCm lib directory
LINK_LIBS = ["-L" + os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib"), "-lrocprofiler-sdk-roctx"]
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def _obj_path(src, objdir):
    return os.path.join(objdir, os.path.splitext(src)[0] + ".o")


def _stale(src, objdir):
    obj = _obj_path(src, objdir)
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, src), os.path.join(ROOT, "include", "ups.h")]
    deps += glob.glob(os.path.join(CSRC, "*.hpp"))
    return any(os.path.getmtime(d) > t for d in deps)


def _compile(src, verbose, objdir=OBJ, extra=()):
    obj = _obj_path(src, objdir)
    cmd = [HIPCC] + FLAGS + list(extra) + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s%s" % (src, r.stdout, r.stderr))
    if verbose and r.stderr.strip():
        sys.stderr.write(r.stderr)
    return obj


def _link(objs, out, extra=(), verbose=False):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + list(extra) + ["-o", tmp] + objs + LINK_LIBS
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s%s" % (r.stdout, r.stderr))
    os.replace(tmp, out)
    return out


def build(verbose=False, incremental=False):
    os.makedirs(OBJ, exist_ok=True)
    todo = [s for s in SOURCES if not incremental or _stale(s, OBJ)]
    if todo:
        with ThreadPoolExecutor(max_workers=len(todo)) as ex:
            list(ex.map(lambda s: _compile(s, verbose), todo))
    objs = [_obj_path(s, OBJ) for s in SOURCES]
    if not incremental or todo or not os.path.exists(OUT):
        _link(objs, OUT, verbose=verbose)
    return OUT


def build_sanitized(verbose=False):
    """libups_san.so: the C-ABI host sources under ASan + UBSan (host pass
    only), the kernel sources as in the regular build."""
    build(verbose=verbose, incremental=True)
    os.makedirs(OBJ_SAN, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(HOST_SOURCES)) as ex:
        list(ex.map(lambda s: _compile(s, verbose, OBJ_SAN, SAN_FLAGS), HOST_SOURCES))
    objs = [_obj_path(s, OBJ_SAN) if s in HOST_SOURCES else _obj_path(s, OBJ) for s in SOURCES]
    return _link(objs, OUT_SAN, extra=["-fsanitize=address", "-fsanitize=undefined", "-shared-libsan"],
                 verbose=verbose)


if __name__ == "__main__":
    v = "-v" in sys.argv
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose=v))
    else:
        print(build(verbose=v, incremental="--incremental" in sys.argv))
