"""Batched uneven-size inpainting (eed4_inpaint_batched): one launch per inner
step over a work queue spanning all images, cycle replayed as a hipGraph,
per-image stop, autotuned kernel shape.

Every kernel shape must give, for each image, exactly (bitwise) what
eed4_inpaint gives for that image alone, whatever shape that call uses (all
shapes form every value the same way); sampled images are also checked
against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
from synth import WORKLOADS, make_problem, make_uneven_batch
from tests.helpers import REL_L2_PER_CYCLE, announce, assert_steady_parity, rel_l2, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
import paper_2006_10406_amd as eed4  # noqa: E402

SHAPES = range(len(eed4.SHAPE_NAMES))
SIZES = [(1, 1), (3, 200), (130, 70), (256, 300), (64, 64), (17, 33), (200, 9), (95, 181)]
LAMS = [0.05, 0.03, 0.02, 0.04, 0.05, 0.1, 0.03, 0.06]


def make_images(sizes=SIZES, seed=50):
    out = []
    for i, (H, W) in enumerate(sizes):
        pr = make_problem(H, W, 4, True, 0.01, 0.06, seed + i)
        out.append(pr)
    return out


def run_batched(probs, lams, p):
    us = [to_dev(pr["u_init"]) for pr in probs]
    imgs = [(u, to_dev(pr["mask"]), to_dev(pr["known"]), lam) for u, pr, lam in zip(us, probs, lams)]
    st = eed4.eed4_inpaint_batched(imgs, p)
    torch.cuda.synchronize()
    return [u.cpu().numpy() for u in us], st


def run_single(pr, lam, sigma, tau, n, M, tol=0.0, flags=0):
    u = to_dev(pr["u_init"])
    st, _ = eed4.eed4_inpaint(u, to_dev(pr["mask"]), to_dev(pr["known"]),
                              eed4.params(lam, sigma, tau, n, M, tol=tol, flags=flags))
    torch.cuda.synchronize()
    return u.cpu().numpy(), st


@pytest.mark.parametrize("shape", SHAPES)
def test_each_shape_equals_single_image_runs(shape):
    announce(f"batched shape {eed4.SHAPE_NAMES[shape]} vs per-image eed4_inpaint")
    probs = make_images()
    sigma, tau, n, M = 1.5, 0.05, 7, 3
    p = eed4.params(1.0, sigma, tau, n, M, flags=eed4.EED4_FORCE_SHAPE(shape))
    outs, st = run_batched(probs, LAMS, p)
    for i, pr in enumerate(probs):
        ref, _ = run_single(pr, LAMS[i], sigma, tau, n, M)          # the single-image default
        assert st[i].cycles == M
        assert np.array_equal(outs[i], ref), f"image {i} {pr['u_init'].shape}"


@pytest.mark.parametrize("n", [1, 2])
def test_short_cycles_batched(n):
    announce(f"batched n={n}")
    probs = make_images(SIZES[:4], seed=70)
    p = eed4.params(1.0, 1.0, 0.05, n, 2, flags=eed4.EED4_FORCE_SHAPE(3))
    outs, _ = run_batched(probs, LAMS[:4], p)
    for i, pr in enumerate(probs):
        ref, _ = run_single(pr, LAMS[i], 1.0, 0.05, n, 2, flags=eed4.EED4_FORCE_SHAPE(3))
        assert np.array_equal(outs[i], ref)


def test_per_image_stop_matches_single_runs():
    announce("batched per-image stop (tol 1e-3)")
    probs = make_images(SIZES[1:6], seed=90)
    lams = LAMS[1:6]
    sigma, tau, n, M, tol = 1.0, 0.05, 10, 60, 1e-3
    p = eed4.params(1.0, sigma, tau, n, M, tol=tol, flags=eed4.EED4_FORCE_SHAPE(3))
    outs, st = run_batched(probs, lams, p)
    cyc = []
    for i, pr in enumerate(probs):
        ref, s1 = run_single(pr, lams[i], sigma, tau, n, M, tol=tol,
                             flags=eed4.EED4_FORCE_SHAPE(5))
        cyc.append((st[i].cycles, s1.cycles))
        assert st[i].cycles == s1.cycles
        assert np.array_equal(outs[i], ref)
    print(f"cycles per image (batched, single): {cyc}")
    assert len(set(c[0] for c in cyc)) > 1, "images should stop at different cycles"


def test_autotune_and_default_path():
    announce("autotuner picks a shape; default call uses it")
    probs = make_images(seed=110)
    p = eed4.params(1.0, 1.5, 0.05, 8, 2)
    imgs = [(to_dev(pr["u_init"]), to_dev(pr["mask"]), to_dev(pr["known"]), lam)
            for pr, lam in zip(probs, LAMS)]
    before = [t[0].clone() for t in imgs]
    shape = eed4.eed4_autotune_batched(imgs, p)
    print(f"autotuned shape: {eed4.SHAPE_NAMES[shape]}")
    assert 0 <= shape < len(eed4.SHAPE_NAMES)
    for t, b0 in zip(imgs, before):        # the tuner leaves u untouched
        assert torch.equal(t[0], b0)
    outs, _ = run_batched(probs, LAMS, p)
    forced, _ = run_batched(probs, LAMS, eed4.params(1.0, 1.5, 0.05, 8, 2,
                                                     flags=eed4.EED4_FORCE_SHAPE(shape)))
    for a, b in zip(outs, forced):
        assert np.array_equal(a, b)


def test_batched_against_oracle():
    announce("batched vs FP64 oracle on sampled images")
    probs = make_images(seed=130)
    sigma, tau, n, M = 1.5, 0.05, 8, 3
    outs, _ = run_batched(probs, LAMS, eed4.params(1.0, sigma, tau, n, M))
    for i in (1, 2, 5, 7):
        pr = probs[i]
        ref, _, _ = oracle.inpaint(pr["u_init"], pr["mask"], pr["known"], LAMS[i], sigma, tau, n, M)
        assert_steady_parity(outs[i], ref, f"image {i} {pr['u_init'].shape}")
        assert rel_l2(outs[i], ref) <= REL_L2_PER_CYCLE


def test_batch64_workload_equals_per_image_runs():
    wl = WORKLOADS["batch64"]
    announce("batch64 workload: 64 uneven images, batched vs per-image (2 cycles)")
    probs = make_uneven_batch(wl)
    M = 2
    p = eed4.params(1.0, wl.sigma, wl.tau, wl.n, M, flags=eed4.EED4_FORCE_SHAPE(3))
    lams = [wl.lam] * len(probs)
    outs, st = run_batched(probs, lams, p)
    for i in range(0, len(probs), 7):
        ref, _ = run_single(probs[i], wl.lam, wl.sigma, wl.tau, wl.n, M,
                            flags=eed4.EED4_FORCE_SHAPE(4))
        assert np.array_equal(outs[i], ref)
    pr = probs[3]
    ref, _, _ = oracle.inpaint(pr["u_init"], pr["mask"], pr["known"], wl.lam, wl.sigma, wl.tau,
                               wl.n, M)
    assert_steady_parity(outs[3], ref, f"batch64 image 3 {pr['u_init'].shape}")
    assert rel_l2(outs[3], ref) <= REL_L2_PER_CYCLE


@pytest.mark.parametrize("d,r", [(1, 0), (2, 1), (3, 2)])
def test_tensor_variant_batched_equals_single_images(d, r):
    # a tensor variant (Table 7 diffusivity, Sec. 3.1 mu3 choice) through the batched queue:
    # each image equals eed4_inpaint of it alone with the same variant, and one against the oracle
    fl = eed4.EED4_DIFFUSIVITY(d) | eed4.EED4_MU3(r)
    announce(f"batched tensor variant {eed4.DIFFUSIVITY_NAMES[d]}/{eed4.MU3_NAMES[r]}")
    probs = make_images()
    sigma, tau, n, M = 1.5, 0.05, 7, 3
    outs, st = run_batched(probs, LAMS, eed4.params(1.0, sigma, tau, n, M, flags=fl))
    for i, pr in enumerate(probs):
        ref, _ = run_single(pr, LAMS[i], sigma, tau, n, M, flags=fl)
        assert st[i].cycles == M
        assert np.array_equal(outs[i], ref), f"image {i} {pr['u_init'].shape}"
    i = 7
    oref, _, _ = oracle.inpaint(probs[i]["u_init"], probs[i]["mask"], probs[i]["known"], LAMS[i],
                                sigma, tau, n, M, diff=d, mu3=r)
    assert_steady_parity(outs[i], oref, f"batched variant image {i}")
