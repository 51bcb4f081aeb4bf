"""Parity of the HIP adjoint (eed4_backward) with the FP64 oracle adjoint, a
directional finite-difference check, and tonal optimisation through the
torch.autograd wrapper.

Both adjoints differentiate the same trajectory: the oracle recomputes each
cycle in FP64 from the checkpoints the GPU forward wrote.  Bar: relative L2
<= 1e-4 and every element within 1e-4 of the largest oracle value, for dL/df
on the mask, dL/du_init off the mask, and dL/dlambda.
"""
import numpy as np
import pytest

import oracle
from synth import WORKLOADS, make_batch, make_problem
from tests.helpers import announce, assert_grad_parity, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
import paper_2006_10406_amd as eed4  # noqa: E402
from paper_2006_10406_amd import autograd as ea  # noqa: E402


def gpu_forward_backward(b, lam, sigma, tau, n, M, gu, flags=0):
    u = to_dev(b["u_init"])
    mask, known = to_dev(b["mask"]), to_dev(b["known"])
    B, H, W = u.shape
    p = eed4.params(lam, sigma, tau, n, M, flags=flags)
    ck = torch.empty((M, B, H, W), dtype=torch.float32, device="cuda")
    eed4.eed4_inpaint(u, mask, known, p, ckpt=ck)
    g = to_dev(gu.astype(np.float32))
    gk, gi = torch.empty_like(g), torch.empty_like(g)
    gl = torch.empty(B, device="cuda")
    eed4.eed4_backward(ck, mask, known, p, M, g, gk, gi, gl)
    torch.cuda.synchronize()
    return (u.cpu().numpy(), ck.cpu().numpy(), gk.cpu().numpy(), gi.cpu().numpy(),
            gl.cpu().numpy())


def compare(b, ck, gk, gi, gl, lam, sigma, tau, n, gu, label):
    ogk, ogi, ogl = oracle.backward(ck.astype(np.float64), b["mask"], b["known"], lam, sigma, tau,
                                    n, gu)
    m = b["mask"] != 0
    print(f"{label}: dL/dlambda gpu {gl[:2]}, oracle {np.atleast_1d(ogl)[:2]}")
    assert np.all(gk[~m] == 0) and np.all(gi[m] == 0)
    assert_grad_parity(gk[m], ogk[m], f"{label} dL/df")
    assert_grad_parity(gi[~m], ogi[~m], f"{label} dL/du_init")
    assert_grad_parity(gl, ogl, f"{label} dL/dlambda")


@pytest.mark.parametrize("H,W,sigma,lam,n,M", [
    (40, 52, 1.0, 0.05, 5, 3), (67, 45, 1.5, 0.03, 4, 2), (33, 70, 2.0, 0.02, 3, 2),
    (20, 17, 0.0, 0.1, 6, 2), (9, 130, 2.6, 0.05, 2, 2), (70, 66, 0.5, 0.04, 1, 3),
    # many cycles: the recompute alternates its two buffer sets across odd and even counts
    (30, 41, 1.0, 0.05, 3, 19), (26, 33, 1.5, 0.03, 2, 8)])
def test_adjoint_matches_oracle(H, W, sigma, lam, n, M):
    announce(f"adjoint {H}x{W} sigma={sigma} n={n} M={M}")
    b = {k: np.stack([make_problem(H, W, 4, True, 0.01, 0.08, 900 + i + H)[k] for i in range(2)])
         for k in ("image", "mask", "known", "u_init")}
    gu = np.random.default_rng(H * W).normal(size=b["u_init"].shape) * 1e-2
    _, ck, gk, gi, gl = gpu_forward_backward(b, lam, sigma, 0.05, n, M, gu)
    compare(b, ck, gk, gi, gl, lam, sigma, 0.05, n, gu, f"{H}x{W} s{sigma} n{n}")


@pytest.mark.parametrize("shape", range(len(eed4.SHAPE_NAMES)))
@pytest.mark.parametrize("H,W,sigma,n", [(75, 140, 1.0, 4), (131, 62, 2.0, 3), (7, 200, 0.5, 2)])
def test_each_reverse_step_kernel_matches_oracle(shape, H, W, sigma, n):
    # tile shapes select the two-pass tile adjoint, strip shapes the fused
    # strip adjoint of that segment height (and the same forward shape)
    announce(f"reverse step {eed4.SHAPE_NAMES[shape]} {H}x{W} sigma={sigma} n={n}")
    b = {k: np.stack([make_problem(H, W, 5, True, 0.01, 0.06, 700 + i + W)[k] for i in range(2)])
         for k in ("image", "mask", "known", "u_init")}
    gu = np.random.default_rng(H + W).normal(size=b["u_init"].shape) * 1e-2
    _, ck, gk, gi, gl = gpu_forward_backward(b, 0.04, sigma, 0.05, n, 2, gu,
                                             flags=eed4.EED4_FORCE_SHAPE(shape))
    compare(b, ck, gk, gi, gl, 0.04, sigma, 0.05, n, gu,
            f"{eed4.SHAPE_NAMES[shape]} {H}x{W} s{sigma}")


@pytest.mark.parametrize("shape", [0, 3, 6])
@pytest.mark.parametrize("H,W", [(1, 1), (2, 3), (1, 40), (37, 1)])
def test_reverse_step_degenerate_sizes(shape, H, W):
    # one pixel, single rows and columns: every neighbour comes from the
    # mirror (repeated reflection), in both the recompute and the reverse step
    announce(f"reverse step {eed4.SHAPE_NAMES[shape]} degenerate {H}x{W}")
    b = {k: np.stack([make_problem(H, W, 2, True, 0.01, 0.25, 40 + i + 3 * H + W)[k]
                      for i in range(2)]) for k in ("image", "mask", "known", "u_init")}
    gu = np.random.default_rng(7 + H * W).normal(size=b["u_init"].shape) * 1e-2
    _, ck, gk, gi, gl = gpu_forward_backward(b, 0.05, 1.0, 0.05, 4, 2, gu,
                                             flags=eed4.EED4_FORCE_SHAPE(shape))
    compare(b, ck, gk, gi, gl, 0.05, 1.0, 0.05, 4, gu,
            f"{eed4.SHAPE_NAMES[shape]} {H}x{W}")


def test_adjoint_tile_kernel_recompute():
    announce("adjoint with the tile step kernel for the recompute")
    b = {k: v[None] for k, v in make_problem(48, 60, 4, True, 0.01, 0.06, 31).items()
         if k in ("image", "mask", "known", "u_init")}
    gu = np.random.default_rng(3).normal(size=b["u_init"].shape) * 1e-2
    _, ck, gk, gi, gl = gpu_forward_backward(b, 0.05, 1.0, 0.05, 5, 2, gu,
                                             flags=eed4.EED4_TILE_KERNEL)
    compare(b, ck, gk, gi, gl, 0.05, 1.0, 0.05, 5, gu, "tile recompute")


def test_adjoint16_workload_sampled_images():
    wl = WORKLOADS["adjoint16"]
    announce("adjoint16: 16 x 256x256, 30 cycles of 10; oracle on images 0 and 9")
    b = make_batch(wl)
    u_gpu = None
    gu = None
    # loss = MSE against the ground truth, seed 2 (u - gt) / N
    u = to_dev(b["u_init"])
    mask, known = to_dev(b["mask"]), to_dev(b["known"])
    B, H, W = u.shape
    p = eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, wl.M)
    ck = torch.empty((wl.M, B, H, W), dtype=torch.float32, device="cuda")
    eed4.eed4_inpaint(u, mask, known, p, ckpt=ck)
    u_gpu = u.cpu().numpy()
    gu = 2.0 * (u_gpu - b["image"]) / u_gpu.size
    g = to_dev(gu.astype(np.float32))
    gk, gi = torch.empty_like(g), torch.empty_like(g)
    gl = torch.empty(B, device="cuda")
    eed4.eed4_backward(ck, mask, known, p, wl.M, g, gk, gi, gl)
    torch.cuda.synchronize()
    ckn, gkn, gin, gln = ck.cpu().numpy(), gk.cpu().numpy(), gi.cpu().numpy(), gl.cpu().numpy()
    for i in (0, 9):
        sub = {k: b[k][i:i + 1] for k in ("image", "mask", "known", "u_init")}
        compare(sub, ckn[:, i:i + 1], gkn[i:i + 1], gin[i:i + 1], gln[i:i + 1], wl.lam, wl.sigma,
                wl.tau, wl.n, gu[i:i + 1], f"adjoint16 image {i}")


def test_directional_finite_difference_on_gpu():
    announce("directional FD of the GPU forward vs GPU adjoint")
    pr = make_problem(64, 64, 5, True, 0.01, 0.05, 1234)
    image = to_dev(pr["image"])
    mask = to_dev(pr["mask"])
    m = mask.float()
    known = (image * m).contiguous()
    lam, sigma, tau, n, M = 0.05, 1.0, 0.05, 10, 5
    kp = known.clone().requires_grad_(True)
    u = ea.inpaint(kp, lam, mask, sigma, tau, n, M)
    loss = torch.sum((u - image) ** 2)
    loss.backward()
    g = kp.grad.detach()
    v = (torch.randn_like(known) * m).contiguous()
    h = 1e-3

    def L(k):
        with torch.no_grad():
            uu = ea.inpaint(k.contiguous(), lam, mask, sigma, tau, n, M)
            return float(torch.sum((uu.double() - image.double()) ** 2))

    fd = (L(known + h * v) - L(known - h * v)) / (2 * h)
    an = float(torch.sum(g * v))
    print(f"directional FD {fd:.6e} vs adjoint {an:.6e}")
    assert abs(fd - an) <= 1e-2 * abs(an)


def test_tonal_optimisation_decreases_mse():
    wl = WORKLOADS["adjoint16"]
    announce("tonal optimisation: 50 Adam steps on 16 x 256x256")
    b = make_batch(wl)
    image = to_dev(b["image"])
    mask = to_dev(b["mask"])
    out = ea.tonal_optimize(image, mask, wl.lam, wl.sigma, wl.tau, wl.n, wl.M, steps=50,
                            lr=5e-3)
    h = out["loss"]
    print(f"tonal optimisation MSE: {h[0]:.6f} -> {out['final_loss']:.6f}")
    assert out["final_loss"] < 0.9 * h[0]
    assert np.all(np.isfinite(h))
