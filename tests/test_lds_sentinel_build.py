"""The LDS-sentinel debug build really fills LDS with NaN, and the library
build does not (CPU only: hipcc cross-compiles a strip step and a tile step of
the library's headers both ways and reads the gfx950 assembly)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2006_10406_amd", "csrc")
NAN = "0x7fc00000"          # the quiet NaN that the fills store

PROBE = r"""
#include "eed4_strip.h"
#include "eed4_tile.h"
using namespace eed4;
__global__ void strip_probe(StripArgs s, StepArgs a)
{
    __shared__ float lds[StripGeo<3, 8>::LDS];
    strip_step<3, false, 8>(lds, s, a.w, nullptr);
}
__global__ void tile_probe(const float *u, float *o, const uint8_t *m, StepArgs a)
{
    __shared__ float smem[TileGeo<3, 32, 16>::SMEM];
    step_tile<3, 32, 16>(smem, u, u, o, nullptr, m, 64, 64, 0, 0, a.w, a.tau, a.alpha, 0.1f,
                         nullptr);
}
"""


def _kernels_with_nan(tmp_path, sentinel):
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not hipcc:
        pytest.skip("hipcc not available")
    src = tmp_path / "probe.hip"
    src.write_text(PROBE)
    out = tmp_path / ("s.s" if sentinel else "l.s")
    cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-S", "--cuda-device-only",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, str(src), "-o", str(out)]
    if sentinel:
        cmd.insert(1, "-DEED4_LDS_SENTINEL=1")
    subprocess.run(cmd, check=True, capture_output=True)
    found, cur = {}, None
    for line in out.read_text().splitlines():
        m = re.match(r"^(_Z\w+):", line)
        if m:
            cur = m.group(1)
            found[cur] = False
        elif cur and NAN in line:
            found[cur] = True
    return found


def test_sentinel_build_fills_lds_and_library_build_does_not(tmp_path):
    lib = _kernels_with_nan(tmp_path, False)
    dbg = _kernels_with_nan(tmp_path, True)
    assert len(lib) == len(dbg) == 2
    assert not any(lib.values()), lib
    assert all(dbg.values()), dbg
