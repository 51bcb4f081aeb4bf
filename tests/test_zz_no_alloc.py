"""The allocation-free entry point eed4_fsi_cycle_static against eed4_fsi_cycle.

eed4_fsi_cycle_static runs the same cycle with its scratch in the library's
static device array instead of a caller workspace, so on the same inputs its
state and residual sums must equal eed4_fsi_cycle's bitwise.  Two calls in a
row, the second on a smaller batch, check that nothing the first call left in
the shared scratch leaks into the second; one call is also held to the FP64
oracle bar.
"""
import numpy as np
import pytest

import oracle
from synth import make_problem
from tests.helpers import announce, assert_cycle_parity, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
import paper_2006_10406_amd as eed4  # noqa: E402


def batch(B, H, W, seed):
    prs = [make_problem(H, W, 8, True, 0.01, 0.05, seed + i) for i in range(B)]
    return {k: np.stack([pr[k] for pr in prs]) for k in ("mask", "known", "u_init")}


def both(b, p):
    """(u, sums) of eed4_fsi_cycle with a workspace and of eed4_fsi_cycle_static."""
    mask, known = to_dev(b["mask"]), to_dev(b["known"])
    B = b["u_init"].shape[0]
    out = []
    for fn in ("ws", "static"):
        u = to_dev(b["u_init"].astype(np.float32))
        sums = torch.full((B, 2), -1.0, dtype=torch.float64, device="cuda")
        if fn == "ws":
            eed4.eed4_fsi_cycle(u, mask, known, p, sums)
        else:
            eed4.eed4_fsi_cycle_static(u, mask, known, p, sums)
        torch.cuda.synchronize()
        out.append((u.cpu().numpy(), sums.cpu().numpy()))
    return out


def test_static_cycle_equals_workspace_cycle_on_two_calls():
    lam, sigma, tau, n = 0.03, 1.5, 0.05, 15
    p = eed4.params(lam, sigma, tau, n, 1)
    # first call: one 1024 x 1024 image (32 MiB of the 64 MiB scratch)
    announce("eed4_fsi_cycle_static call 1: 1 x 1024x1024, n 15")
    b1 = batch(1, 1024, 1024, 4100)
    (u_ws, s_ws), (u_st, s_st) = both(b1, p)
    assert np.array_equal(u_st, u_ws)
    assert np.array_equal(s_st, s_ws)
    # second call right after, smaller: three 200 x 130 images with a ragged tail
    announce("eed4_fsi_cycle_static call 2: 3 x 200x130, n 15")
    b2 = batch(3, 200, 130, 4200)
    (u_ws2, s_ws2), (u_st2, s_st2) = both(b2, p)
    assert np.array_equal(u_st2, u_ws2)
    assert np.array_equal(s_st2, s_ws2)
    # and the static path meets the oracle bar on its own
    ref, _, hist = oracle.inpaint(np.where(b2["mask"] != 0, b2["known"], b2["u_init"])
                                  .astype(np.float32).astype(np.float64), b2["mask"],
                                  b2["known"].astype(np.float32), lam, sigma, tau, n, 1)
    for i in range(3):
        assert_cycle_parity(u_st2[i], ref[i], f"static cycle image {i}")
    assert np.allclose(np.sqrt(s_st2[:, 1]), hist[0, :, 1], rtol=1e-6)


def test_static_cycle_rejects_problems_beyond_its_scratch():
    # 3000 x 3000 needs 2 x 36 MB of rotation buffers: EED4_ETOOLARGE, before any device work
    announce("eed4_fsi_cycle_static too large: 3000x3000")
    u = torch.zeros((3000, 3000), dtype=torch.float32, device="cuda")
    m = torch.zeros((3000, 3000), dtype=torch.uint8, device="cuda")
    sums = torch.zeros(2, dtype=torch.float64, device="cuda")
    before = u.clone()
    with pytest.raises(eed4.EED4Error) as err:
        eed4.eed4_fsi_cycle_static(u, m, u, eed4.params(0.03, 1.5, 0.05, 10, 1), sums)
    assert err.value.code == eed4._lib.EED4_ETOOLARGE
    torch.cuda.synchronize()
    assert torch.equal(u, before)
