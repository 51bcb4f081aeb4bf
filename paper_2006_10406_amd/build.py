"""Build libeed4.so for gfx950 with hipcc (in-tree, no JIT).

Every ``csrc/*.hip`` file is compiled to an object under ``_build/`` and the
objects are linked into ``paper_2006_10406_amd/lib/libeed4.so``.  Packed FP32
instructions are disabled for all device code.

``build_sentinel()`` builds the same sources with ``EED4_LDS_SENTINEL=1`` into
``lib/libeed4_sentinel.so``: a debug library whose stencil kernels fill their
LDS with NaN before each stage, for the halo-coverage tests only.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libeed4.so")
SENTINEL_LIB = os.path.join(LIBDIR, "libeed4_sentinel.so")
# roctx ranges and marks of the host code (rocprofiler-sdk)
LINK_LIBS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def compile_flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-parameter",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _compile(src: str, verbose: bool, objdir: str = BUILD, defines=()) -> str:
    obj = os.path.join(objdir, os.path.basename(src) + ".o")
    cmd = [hipcc()] + compile_flags() + [f"-D{d}" for d in defines] + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the packed-fp32 feature and says so; that is harmless
    msg = "\n".join(l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{msg}")
    if verbose and msg.strip():
        print(msg, flush=True)
    return obj


def _build_lib(out: str, objdir: str, defines, verbose: bool, jobs: int) -> str:
    os.makedirs(objdir, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, objdir, defines), srcs))
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + LINK_LIBS
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False, jobs: int = 4) -> str:
    return _build_lib(LIB, BUILD, (), verbose, jobs)


def build_sentinel(verbose: bool = False, jobs: int = 4) -> str:
    return _build_lib(SENTINEL_LIB, os.path.join(BUILD, "sentinel"), ("EED4_LDS_SENTINEL=1",),
                      verbose, jobs)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
    if "--sentinel" in sys.argv:
        build_sentinel(verbose="-v" in sys.argv)
        print(SENTINEL_LIB)
