"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only).

eed4_api.hip and eed4_adjoint.hip hold the argument checks, the workspace
sizing and the host side of every entry point but the batched ones.  They are
compiled with host-side ASan and UBSan (device code as in the library) and
linked with the library's other objects from its build.  The CPU ABI tests then
run against that build in a child process with clang's ASan runtime preloaded,
through the binding's EED4_LIBRARY override; a finding aborts the run.  A canary
library with a planted heap overflow, built and loaded the same way, shows that
the sanitizers are live.
"""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2006_10406_amd")
HIPCC = "/opt/rocm/bin/hipcc"
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")


def _asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        pytest.skip("clang ASan runtime not available")
    return found[-1]


def _env(lib):
    env = dict(os.environ)
    env["LD_PRELOAD"] = _asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["EED4_LIBRARY"] = lib
    env["PYTHONPATH"] = ROOT
    return env


def test_sanitizers_are_live(tmp_path):
    src = tmp_path / "canary.cpp"
    src.write_text('#include <cstdlib>\nextern "C" int canary(int n) { int *a = (int *)malloc(4 * n);'
                   " a[n] = 1; int r = a[0]; free(a); return r; }\n")
    lib = tmp_path / "libcanary.so"
    subprocess.run([HIPCC, "-O1", "-g", "-shared", "-fPIC"] + SANITIZE + ["-o", str(lib), str(src)],
                   check=True, capture_output=True)
    code = f"import ctypes; ctypes.CDLL({str(lib)!r}).canary(4)"
    r = subprocess.run([sys.executable, "-c", code], env=_env(str(lib)), capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr


def test_abi_checks_under_asan_and_ubsan(tmp_path):
    others = [os.path.join(PKG, "_build", f + ".hip.o") for f in ("eed4_batched", "eed4_forward")]
    if not all(os.path.exists(o) for o in others):
        pytest.skip("the library's objects are missing: run __graft_entry__.build()")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]

    def compile_one(name):
        obj = str(tmp_path / (name + ".o"))
        cmd = ([HIPCC, "--offload-arch=gfx950", "-O3", "-Xarch_host", "-O1", "-g", "-std=c++17",
                "-fPIC", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + SANITIZE
               + inc + ["-c", os.path.join(PKG, "csrc", name + ".hip"), "-o", obj])
        subprocess.run(cmd, check=True, capture_output=True)
        return obj

    with cf.ThreadPoolExecutor(max_workers=2) as ex:
        objs = list(ex.map(compile_one, ("eed4_api", "eed4_adjoint")))
    lib = str(tmp_path / "libeed4_san.so")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + SANITIZE
                   + ["-o", lib] + objs + others + ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"],
                   check=True, capture_output=True)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", os.path.join(ROOT, "tests", "test_abi.py")],
                       env=_env(lib), capture_output=True, text=True, timeout=600, cwd=ROOT)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "failed" not in r.stdout, tail
