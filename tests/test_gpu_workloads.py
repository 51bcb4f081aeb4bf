"""Colour (channel-wise) and scratch-removal inpainting on the GPU against the
FP64 oracle, through the C ABI.

The paper inpaints RGB images channel-wise (Sec. 4.1) and removes thin (6 %)
and thick (18 %) scratches (Sec. 4.2).  Here a colour image is an equal-size
batch of three planes sharing one mask, and a scratch mask is a structured
mask with most pixels known.  Both also go through the uneven-batch call
beside images of other sizes.  Bar: relative L2 <= 1e-5 and every element
within 1e-5 per cycle from the oracle's state; RMSE <= 1e-4 and every element
within 1e-4 at equal cycle counts.
"""
import numpy as np
import pytest

import oracle
from synth import WORKLOADS, make_rgb_problem, make_scratch_problem, make_workload_problem
from tests.helpers import (announce, assert_cycle_parity, assert_steady_parity, rmse,
                           to_dev)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
import paper_2006_10406_amd as eed4  # noqa: E402


def test_rgb_channelwise_run_and_single_channels():
    wl = WORKLOADS["rgb512"]
    H, W, M = 160, 200, 6
    announce(f"rgb channel-wise {H}x{W}x3, {M} cycles of {wl.n}")
    pr = make_rgb_problem(H, W, 12, True, 0.01, wl.density, 6100)
    ref, cyc, rh = oracle.inpaint(pr["u_init"], pr["mask"], pr["known"], wl.lam, wl.sigma,
                                  wl.tau, wl.n, M)
    u = to_dev(pr["u_init"])
    p = eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, M)
    st, hist = eed4.eed4_inpaint(u, to_dev(pr["mask"]), to_dev(pr["known"]), p, history=True)
    got = u.cpu().numpy()
    print(f"rgb {H}x{W}: RMSE vs ground truth {rmse(got, pr['image']):.4f} "
          f"(oracle {rmse(ref, pr['image']):.4f})")
    assert st.cycles == cyc == M
    for c in range(3):
        assert_steady_parity(got[c], ref[c], f"rgb {H}x{W} channel {c}")
    assert np.allclose(hist[:, :, 1], rh[:, :, 1], rtol=1e-5)
    kn = pr["mask"] != 0
    assert np.array_equal(got[kn], pr["known"][kn])
    # channel-wise: each plane equals a single-channel run with the same kernel shape
    shape = eed4.eed4_step_shape(3, H, W, p)
    for c in range(3):
        uc = to_dev(pr["u_init"][c])
        pc = eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, M, flags=eed4.EED4_FORCE_SHAPE(shape))
        eed4.eed4_inpaint(uc, to_dev(pr["mask"][c]), to_dev(pr["known"][c]), pc)
        assert np.array_equal(uc.cpu().numpy(), got[c])


def test_rgb512_per_cycle_parity():
    wl = WORKLOADS["rgb512"]
    M = 2
    announce(f"rgb512 full size, per-cycle parity of {M} cycles")
    pr = make_workload_problem(wl)
    _, _, _, ck = oracle.inpaint(pr["u_init"], pr["mask"], pr["known"], wl.lam, wl.sigma, wl.tau,
                                 wl.n, M, checkpoints=True)
    states = ck.reshape(M * 3, wl.H, wl.W).astype(np.float32)
    masks = np.tile(pr["mask"], (M, 1, 1))
    knowns = np.tile(pr["known"], (M, 1, 1))
    u = to_dev(states)
    sums = torch.zeros((M * 3, 2), dtype=torch.float64, device="cuda")
    eed4.eed4_fsi_cycle(u, to_dev(masks), to_dev(knowns), eed4.params(wl.lam, wl.sigma, wl.tau,
                                                                      wl.n, 1), sums)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    ref, _, _ = oracle.inpaint(states.astype(np.float64), masks, knowns, wl.lam, wl.sigma,
                               wl.tau, wl.n, 1)
    for i in range(M * 3):
        assert_cycle_parity(got[i], ref[i], f"rgb512 cycle {i // 3} channel {i % 3}")


@pytest.mark.parametrize("name", ["scratch512_thin", "scratch512_thick"])
def test_scratch_removal_full_size(name):
    wl = WORKLOADS[name]
    M = 10
    announce(f"{name}: {wl.H}x{wl.W}, {100 * wl.density:.0f}% scratched, {M} cycles of {wl.n}")
    pr = make_workload_problem(wl)
    ref, cyc, rh = oracle.inpaint(pr["u_init"], pr["mask"], pr["known"], wl.lam, wl.sigma,
                                  wl.tau, wl.n, M)
    u = to_dev(pr["u_init"])
    st, hist = eed4.eed4_inpaint(u, to_dev(pr["mask"]), to_dev(pr["known"]),
                                 eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, M), history=True)
    got = u.cpu().numpy()
    unk = pr["mask"] == 0
    print(f"{name}: on the scratches vs ground truth "
          f"{rmse(got[unk], pr['image'][unk]):.4f} (oracle {rmse(ref[unk], pr['image'][unk]):.4f}, "
          f"initial {rmse(pr['u_init'][unk], pr['image'][unk]):.4f})")
    assert st.cycles == cyc == M
    assert_steady_parity(got, ref, f"{name} after {M} cycles")
    assert np.allclose(hist[:, 0, 1], rh[:, 1], rtol=1e-5)
    assert np.array_equal(got[~unk], pr["known"][~unk])


@pytest.mark.parametrize("shape", [2, 5, 10])
def test_colour_and_scratch_images_in_one_uneven_batch(shape):
    # three colour planes sharing one mask, a thin and a thick scratch image of other sizes, in
    # one eed4_inpaint_batched call: each equals its own eed4_inpaint run in the same kernel
    # shape bitwise, and one plane meets the oracle bar
    sigma, tau, n, M = 1.5, 0.05, 8, 4
    announce(f"colour + scratch uneven batch, shape {eed4.SHAPE_NAMES[shape]}, {M} cycles of {n}")
    rgb = make_rgb_problem(120, 150, 10, True, 0.01, 0.05, 6200)
    thin = make_scratch_problem(130, 97, 10, True, 0.005, 0.06, 2, 6201)
    thick = make_scratch_problem(88, 170, 10, True, 0.005, 0.18, 6, 6202)
    probs = [{k: rgb[k][c] for k in ("mask", "known", "u_init")} for c in range(3)]
    probs += [thin, thick]
    lams = [0.03, 0.03, 0.03, 0.02, 0.04]
    flags = eed4.EED4_FORCE_SHAPE(shape)
    us = [to_dev(pr["u_init"]) for pr in probs]
    st = eed4.eed4_inpaint_batched([(u, to_dev(pr["mask"]), to_dev(pr["known"]), lam)
                                    for u, pr, lam in zip(us, probs, lams)],
                                   eed4.params(1.0, sigma, tau, n, M, flags=flags))
    torch.cuda.synchronize()
    for i, (u, pr, lam) in enumerate(zip(us, probs, lams)):
        v = to_dev(pr["u_init"])
        eed4.eed4_inpaint(v, to_dev(pr["mask"]), to_dev(pr["known"]),
                          eed4.params(lam, sigma, tau, n, M, flags=flags))
        assert st[i].cycles == M
        assert torch.equal(u, v), f"image {i} {tuple(u.shape)}"
    ref, _, _ = oracle.inpaint(probs[4]["u_init"], probs[4]["mask"], probs[4]["known"], lams[4],
                               sigma, tau, n, M)
    assert_steady_parity(us[4].cpu().numpy(), ref, f"thick scratch {eed4.SHAPE_NAMES[shape]}")
