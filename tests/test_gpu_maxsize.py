"""The largest single image the C ABI accepts (H*W = 2^31 pixels, 8 GiB per
float plane) through the fused step and one FSI cycle, on the GPU.

The oracle cannot run on the whole image, so outputs are compared pixel by
pixel at sampled points: corners, edges, strip and tile seams, and random
interior points.  One step (one cycle of n steps) at a pixel depends only on
the input within R+2 (n(R+2)) pixels of it, and the half-sample mirror only
at the image border, so the oracle run on a crop that reaches that far on
every side (or to the border) gives the exact value at the crop's centre.
The cycle residual, which no crop holds, is checked against a plain FP64 sum
of the difference of the two full-size states.
"""
import numpy as np
import pytest

import oracle
from synth import make_problem_device
from tests.helpers import announce

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
import paper_2006_10406_amd as eed4  # noqa: E402

H, W = 32768, 65536                     # H * W = 2^31
LAM, SIGMA, TAU = 0.02, 2.0, 0.05       # the 4096^2 workload's parameters (R = 6)
PIX_TOL = 1e-5                          # grey values in [0, 1]


def sample_points():
    pts = [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (0, W // 2), (H - 1, 12345),
           (H // 3, 0), (H // 2, W - 1), (1, 1), (H - 2, W - 2), (H - 9, W - 9),
           (7000, 59999), (7000, 60000), (20000, 61999), (20000, 62000), (H - 1, 65471),
           (16383, 16384), (16384, 32767)]
    rng = np.random.default_rng(99)
    pts += [(int(rng.integers(0, H)), int(rng.integers(0, W))) for _ in range(22)]
    return pts


def crop(t, y, x, c):
    y0, y1 = max(0, y - c), min(H, y + c + 1)
    x0, x1 = max(0, x - c), min(W, x + c + 1)
    return t[y0:y1, x0:x1].cpu().numpy(), y - y0, x - x0


@pytest.fixture(scope="module")
def problem():
    free, _ = torch.cuda.mem_get_info()
    if free < 72 * 2 ** 30:
        pytest.skip(f"needs about 72 GiB of free device memory, {free / 2 ** 30:.0f} GiB free")
    announce(f"maximum size {H}x{W}: drawing the problem on the device")
    pr = make_problem_device(H, W, 200, True, 0.005, 0.03, 4242)
    torch.cuda.synchronize()
    yield pr
    del pr
    torch.cuda.empty_cache()


@pytest.mark.parametrize("shape", [None, 5, 7, 0, 10])
def test_one_step_at_maximum_size(problem, shape):
    u, mask = problem["u_init"], problem["mask"]
    flags = 0 if shape is None else eed4.EED4_FORCE_SHAPE(shape)
    p = eed4.params(LAM, SIGMA, TAU, 15, 1, flags=flags)
    used = eed4.eed4_step_shape(1, H, W, p)
    announce(f"maximum size {H}x{W}: one step, shape {eed4.SHAPE_NAMES[used]}")
    out = torch.empty_like(u)
    eed4.eed4_fsi_step(u[None], u[None], out[None], mask[None], p, 0)
    torch.cuda.synchronize()
    R = oracle.radius(SIGMA)
    errs = []
    for (y, x) in sample_points():
        uc, cy, cx = crop(u, y, x, R + 3)
        mc, _, _ = crop(mask, y, x, R + 3)
        ref = oracle.step(uc, uc, mc, uc, LAM, SIGMA, TAU, 0)[cy, cx]
        errs.append(abs(float(out[y, x]) - ref))
    print(f"{eed4.SHAPE_NAMES[used]}: max |GPU - FP64| over {len(errs)} samples {max(errs):.2e}")
    assert max(errs) <= PIX_TOL
    del out
    torch.cuda.empty_cache()


def test_one_cycle_at_maximum_size(problem):
    n = 2
    u0, mask, known = problem["u_init"], problem["mask"], problem["known"]
    p = eed4.params(LAM, SIGMA, TAU, n, 1)
    announce(f"maximum size {H}x{W}: one FSI cycle of {n}, shape "
             f"{eed4.SHAPE_NAMES[eed4.eed4_step_shape(1, H, W, p)]}")
    u = u0.clone()
    sums = torch.zeros((1, 2), dtype=torch.float64, device="cuda")
    eed4.eed4_fsi_cycle(u[None], mask[None], known[None], p, sums)
    torch.cuda.synchronize()
    R = oracle.radius(SIGMA)
    c = n * (R + 2) + 1
    errs = []
    for (y, x) in sample_points():
        uc, cy, cx = crop(u0, y, x, c)
        mc, _, _ = crop(mask, y, x, c)
        kc, _, _ = crop(known, y, x, c)
        ref, _, _ = oracle.inpaint(uc, mc, kc, LAM, SIGMA, TAU, n, 1)
        errs.append(abs(float(u[y, x]) - ref[cy, cx]))
    # residual sums: plain FP64 sums over blocks of rows of the two full-size states
    d2 = n2 = 0.0
    for r0 in range(0, H, 2048):
        a = u[r0:r0 + 2048].double()
        d2 += float(((a - u0[r0:r0 + 2048].double()) ** 2).sum())
        n2 += float((a * a).sum())
    got = sums.cpu().numpy()[0]
    print(f"cycle: max |GPU - FP64| over {len(errs)} samples {max(errs):.2e}; residual "
          f"{np.sqrt(got[0]):.6e} (plain sum {np.sqrt(d2):.6e}), norm {np.sqrt(got[1]):.6e}")
    assert max(errs) <= PIX_TOL
    assert got[0] == pytest.approx(d2, rel=1e-9) and got[1] == pytest.approx(n2, rel=1e-9)
    for r0 in range(0, H, 2048):           # known pixels hold f (by blocks of rows: boolean
        rows = slice(r0, r0 + 2048)        # indexing of 2^31 elements fails in torch itself)
        assert bool(((u[rows] == known[rows]) | (mask[rows] == 0)).all())
    del u
    torch.cuda.empty_cache()
