"""Structure of the batched queue kernels in the gfx950 assembly (CPU only:
hipcc cross-compiles).

Each batched kernel walks the work queue in one loop (a static stride over
the queue); the workgroup-tile kernels meet their other waves at barriers
inside it.  The item fetch must sit in the header block of that one loop, and
no loop nested inside it may contain a barrier: a nested barrier loop that
skips the fetch makes the waves spin on a stale item index forever (the
pattern the compiler produced for an earlier atomic-counter version; kept as
a regression test).
"""
import os
import re
import shutil
import subprocess
from collections import defaultdict

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2006_10406_amd", "csrc", "eed4_batched.hip")


def _assembly(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not hipcc:
        pytest.skip("hipcc not available")
    out = tmp_path / "b.s"
    cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-S", "--cuda-device-only",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.dirname(SRC), SRC, "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text()


def _loops(asm, kernel):
    """Blocks of a kernel with their innermost loop header and depth, from the
    compiler's block annotations (labelled .LBB blocks and '; %bb.N:' ones)."""
    i = asm.index(kernel + ":")
    j = asm.index(".Lfunc_end", i)
    blocks, cur = [], None
    for line in asm[i:j].splitlines():
        m = re.match(r"^\.(LBB\w+):\s*(.*)$", line) or re.match(r"^; %bb\.(\d+):\s*(.*)$", line)
        if m:
            name = m.group(1)[1:] if m.group(1).startswith("LBB") else "bb." + m.group(1)
            cur = {"name": name, "note": m.group(2), "hdr": None, "depth": 0, "bar": 0, "atom": 0}
            blocks.append(cur)
        elif cur is not None and re.match(r"^\s*;", line) and not re.match(r"^; %bb", line):
            cur["note"] += " " + line
            continue
        elif cur is None:
            continue
        else:
            cur["bar"] += "s_barrier" in line
            cur["atom"] += "global_atomic" in line
            continue
    for b in blocks:
        h = re.search(r"This (?:Inner )?Loop Header: Depth=(\d)", b["note"])
        if h:
            b["hdr"], b["depth"] = b["name"], int(h.group(1))
            continue
        h = re.search(r"in Loop: Header=(\w+) Depth=(\d)", b["note"])
        if h:
            b["hdr"], b["depth"] = h.group(1), int(h.group(2))
    loops = defaultdict(lambda: {"bar": 0, "depth": 0})
    for b in blocks:
        if b["hdr"]:
            loops[b["hdr"]]["bar"] += b["bar"]
            loops[b["hdr"]]["depth"] = max(loops[b["hdr"]]["depth"], b["depth"])
    atom_blocks = [(b["name"], b["hdr"]) for b in blocks if b["atom"]]
    return loops, atom_blocks


def test_tile_queue_loops(tmp_path):
    # one queue loop per tile kernel, no atomics, and no loop nested in it
    # that holds a barrier (such a loop is how a lane-dependent branch near the
    # loop head once left waves spinning on a stale work index)
    asm = _assembly(tmp_path)
    kernels = [k for k in re.findall(r"^(_ZN4eed412btile_kernel\w+):", asm, re.M)]
    assert kernels
    for k in kernels:
        loops, atom_blocks = _loops(asm, k)
        outer = [h for h, L in loops.items() if L["depth"] == 1]
        assert len(outer) == 1, (k, dict(loops))
        assert not atom_blocks, (k, atom_blocks)
        nested_with_barrier = [h for h, L in loops.items() if L["depth"] > 1 and L["bar"]]
        assert not nested_with_barrier, (k, nested_with_barrier)


def test_queue_loops_exit_uniformly(tmp_path):
    # A queue loop must leave through a uniform (SGPR/VCC) branch: an
    # exec-mask exit (s_cbranch_execz to the kernel end) means lanes took
    # different paths around the loop, i.e. a partial wave would keep pulling.
    asm = _assembly(tmp_path)
    kernels = re.findall(r"^(_ZN4eed4\w*(?:bstrip|btile)_kernel\w+):", asm, re.M)
    assert len(kernels) >= 10
    for k in kernels:
        i = asm.index(k + ":")
        j = asm.index(".Lfunc_end", i)
        raw = asm[i:j].splitlines()
        end = None
        for n, line in enumerate(raw):
            m = re.match(r"^(\.LBB\w+):", line)
            if m and any("s_endpgm" in x for x in raw[n + 1:n + 3]):
                end = m.group(1)
        assert end, k
        bad = [x for x in raw if re.search(r"s_cbranch_execz\s+" + re.escape(end) + r"\b", x)]
        assert not bad, (k, bad)


def test_no_scalar_stores_or_atomics(tmp_path):
    # device code writes only through vector memory instructions
    asm = _assembly(tmp_path)
    hits = re.findall(r"^\s*(s_store\w*|s_buffer_store\w*|s_atomic\w*|s_buffer_atomic\w*|"
                      r"s_dcache_wb\w*|s_scratch_store\w*)", asm, re.M)
    assert not hits, hits[:5]
