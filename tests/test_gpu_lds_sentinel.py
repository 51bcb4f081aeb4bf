"""Halo coverage of every stencil kernel: the LDS-sentinel debug build against
the library.

``lib/libeed4_sentinel.so`` is the library's sources compiled with
EED4_LDS_SENTINEL=1: each stencil kernel (forward strips and tiles, their
batched queue versions, both reverse steps, the presmoothing kernel) fills its
LDS with NaN before each stage that writes it.  A slot that a stage reads
without having written it (an undersized halo, a missing barrier) then feeds NaN
into the outputs that depend on it, or changes them.  Every result of the debug
build must be finite and bitwise equal to the library's, for every kernel shape
at several radii on ragged sizes.
"""
import os

import numpy as np
import pytest

from synth import make_problem
from tests.helpers import announce, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
import paper_2006_10406_amd as eed4  # noqa: E402
from paper_2006_10406_amd import _lib  # noqa: E402

SENTINEL_PATH = os.path.join(os.path.dirname(_lib.LIB_PATH), "libeed4_sentinel.so")

# (H, W, sigma): radii 0, 2, 3, 6 and 8, with tails in both directions
SIZES = [(37, 130, 1.0), (130, 37, 2.0), (5, 300, 0.5), (70, 66, 2.6), (200, 9, 0.0)]


@pytest.fixture(scope="module")
def sentinel():
    if not os.path.exists(SENTINEL_PATH):
        pytest.fail(f"{SENTINEL_PATH} is missing: run __graft_entry__.build()")
    return _lib.load_library(SENTINEL_PATH)


def with_library(handle, fn):
    """fn() with the binding pointed at handle (the sentinel build), then back."""
    saved = _lib._L
    _lib._L = handle
    try:
        out = fn()
        torch.cuda.synchronize()
        return out
    finally:
        _lib._L = saved


def problem(H, W, B, seed):
    prs = [make_problem(H, W, 4, True, 0.01, 0.08, seed + i) for i in range(B)]
    return {k: np.stack([p[k] for p in prs]) for k in ("u_init", "mask", "known")}


def same(a, b, what):
    assert bool(torch.isfinite(b).all()), f"{what}: the sentinel build produced non-finite values"
    assert torch.equal(a, b), f"{what}: the sentinel build differs from the library"


@pytest.mark.parametrize("shape", range(len(eed4.SHAPE_NAMES)))
@pytest.mark.parametrize("H,W,sigma", SIZES)
def test_forward_cycle_every_shape(sentinel, shape, H, W, sigma):
    announce(f"sentinel forward {eed4.SHAPE_NAMES[shape]} {H}x{W} sigma={sigma}")
    b = problem(H, W, 2, 300 + H)
    mask, known = to_dev(b["mask"]), to_dev(b["known"])
    p = eed4.params(0.04, sigma, 0.05, 3, 1, flags=eed4.EED4_FORCE_SHAPE(shape))
    outs = []
    for handle in (None, sentinel):
        u = to_dev(b["u_init"])
        sums = torch.zeros((2, 2), dtype=torch.float64, device="cuda")
        run = lambda: eed4.eed4_fsi_cycle(u, mask, known, p, sums)  # noqa: E731
        if handle is None:
            run()
            torch.cuda.synchronize()
        else:
            with_library(handle, run)
        outs.append((u, sums))
    same(outs[0][0], outs[1][0], "cycle state")
    same(outs[0][1], outs[1][1], "cycle residual sums")


@pytest.mark.parametrize("shape", range(len(eed4.SHAPE_NAMES)))
def test_batched_every_shape(sentinel, shape):
    sizes = [(37, 130), (130, 37), (5, 300), (70, 66)]
    announce(f"sentinel batched {eed4.SHAPE_NAMES[shape]} {sizes}")
    probs = [make_problem(H, W, 4, True, 0.01, 0.08, 500 + i) for i, (H, W) in enumerate(sizes)]
    p = eed4.params(0.04, 1.5, 0.05, 3, 2, flags=eed4.EED4_FORCE_SHAPE(shape))
    outs = []
    for handle in (None, sentinel):
        imgs = [(to_dev(pr["u_init"]), to_dev(pr["mask"]), to_dev(pr["known"]), 0.04)
                for pr in probs]
        run = lambda: eed4.eed4_inpaint_batched(imgs, p)  # noqa: E731
        if handle is None:
            run()
            torch.cuda.synchronize()
        else:
            with_library(handle, run)
        outs.append([im[0] for im in imgs])
    for i, (a, c) in enumerate(zip(*outs)):
        same(a, c, f"batched image {i}")


@pytest.mark.parametrize("flags", [0, eed4.EED4_DIFFUSIVITY(eed4.EED4_PERONA_MALIK_EXP)
                                   | eed4.EED4_MU3(eed4.EED4_MU3_ARITHMETIC)],
                         ids=["foeed", "variant"])
@pytest.mark.parametrize("shape", range(len(eed4.SHAPE_NAMES)))
@pytest.mark.parametrize("H,W,sigma", [(37, 130, 1.0), (70, 66, 2.0), (5, 300, 2.6)])
def test_backward_every_shape(sentinel, shape, H, W, sigma, flags):
    if flags and shape != 5:
        pytest.skip("tensor variants run one kernel shape (strip_short)")
    announce(f"sentinel backward {eed4.SHAPE_NAMES[shape]} {H}x{W} sigma={sigma} flags={flags}")
    b = problem(H, W, 2, 700 + W)
    mask, known = to_dev(b["mask"]), to_dev(b["known"])
    n, M = 3, 2
    p = eed4.params(0.04, sigma, 0.05, n, M, flags=flags | eed4.EED4_FORCE_SHAPE(shape))
    u = to_dev(b["u_init"])
    ck = torch.empty((M, 2, H, W), dtype=torch.float32, device="cuda")
    eed4.eed4_inpaint(u, mask, known, p, ckpt=ck)
    gu = to_dev((np.random.default_rng(H + W).normal(size=(2, H, W)) * 1e-2).astype(np.float32))
    outs = []
    for handle in (None, sentinel):
        gk, gi = torch.empty_like(gu), torch.empty_like(gu)
        gl = torch.empty(2, device="cuda")
        run = lambda: eed4.eed4_backward(ck, mask, known, p, M, gu, gk, gi, gl)  # noqa: E731
        if handle is None:
            run()
            torch.cuda.synchronize()
        else:
            with_library(handle, run)
        outs.append((gk, gi, gl))
    for name, a, c in zip(("dL/df", "dL/du_init", "dL/dlambda"), outs[0], outs[1]):
        same(a, c, name)
