"""The oracle pins under AddressSanitizer and UndefinedBehaviorSanitizer.

The FP64 oracle (plain C) is rebuilt with -fsanitize=address,undefined and
the pin tests run against that build in a child process with the ASan runtime
preloaded; any out-of-bounds access, use after free or undefined behaviour in
the oracle aborts the run.  A canary library with a deliberate out-of-bounds
write, loaded the same way, shows that the sanitizers are live in this setup.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")


def _asan_runtime():
    out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = out.stdout.strip()
    if not path or not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip("libasan not available")
    return path


def _env(lib):
    env = dict(os.environ)
    env["LD_PRELOAD"] = _asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["EED4_ORACLE_LIB"] = lib
    env["PYTHONPATH"] = ROOT
    return env


def test_sanitizers_are_live(tmp_path):
    src = tmp_path / "canary.c"
    src.write_text("#include <stdlib.h>\n"
                   "int canary(int n) { int *a = malloc(4 * n); a[n] = 1; int r = a[0]; free(a); "
                   "return r; }\n")
    lib = tmp_path / "libcanary.so"
    subprocess.run(["gcc", "-O1", "-g", "-shared", "-fPIC", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-o", str(lib), str(src)], check=True)
    code = f"import ctypes; ctypes.CDLL({str(lib)!r}).canary(4)"
    r = subprocess.run([sys.executable, "-c", code], env=_env(str(lib)), capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    from oracle import build
    lib = build.build_sanitized(str(tmp_path / "liboracle_san.so"))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_variants.py")],
                       env=_env(lib), capture_output=True, text=True, timeout=600, cwd=ROOT)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "failed" not in r.stdout, tail
