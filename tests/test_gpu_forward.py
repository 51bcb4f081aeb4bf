"""Parity of the fused HIP forward path (eed4_fsi_cycle, eed4_inpaint) with
the FP64 oracle, through the C ABI.

Bar: relative L2 <= 1e-5 and every element within 1e-5 for one FSI cycle
started from the same FP32 state; RMSE <= 1e-4 and every element within 1e-4
for multi-cycle runs at equal cycle counts (grey values in [0, 1]).  The
FP32-vs-FP64 error of every case is printed.  Inputs come from the seeded
generator.
"""
import numpy as np
import pytest

import oracle
from synth import WORKLOADS, make_batch, make_problem
from tests.helpers import announce, assert_cycle_parity, assert_steady_parity, rmse, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
import paper_2006_10406_amd as eed4  # noqa: E402


KERNELS = {"strip": eed4.EED4_FORCE_SHAPE(3), "tile": eed4.EED4_TILE_KERNEL}


def gpu_cycle(states, mask, known, lam, sigma, tau, n, flags=0):
    """One eed4_fsi_cycle over a batch of FP32 start states; returns (u, sums)."""
    u = to_dev(states.astype(np.float32))
    sums = torch.zeros((states.shape[0], 2), dtype=torch.float64, device="cuda")
    p = eed4.params(lam, sigma, tau, n, 1, flags=flags)
    eed4.eed4_fsi_cycle(u, to_dev(mask), to_dev(known.astype(np.float32)), p, sums)
    torch.cuda.synchronize()
    return u.cpu().numpy(), sums.cpu().numpy()


def oracle_cycle(states, mask, known, lam, sigma, tau, n):
    u, _, hist = oracle.inpaint(states.astype(np.float32).astype(np.float64), mask,
                                known.astype(np.float32), lam, sigma, tau, n, 1)
    return u, hist


def test_small64_per_cycle_parity():
    wl = WORKLOADS["small64"]
    announce(f"small64 per-cycle parity, {wl.M} cycles of {wl.n}")
    pr = make_problem(wl.H, wl.W, wl.n_ellipses, wl.ramp, wl.noise_std, wl.density, wl.seed_base)
    _, cyc, hist, ck = oracle.inpaint(pr["u_init"], pr["mask"], pr["known"], wl.lam, wl.sigma,
                                      wl.tau, wl.n, wl.M, checkpoints=True)
    M = ck.shape[0]
    masks = np.repeat(pr["mask"][None], M, 0)
    knowns = np.repeat(pr["known"][None], M, 0)
    got, sums = gpu_cycle(ck, masks, knowns, wl.lam, wl.sigma, wl.tau, wl.n)
    ref, rh = oracle_cycle(ck, masks, knowns, wl.lam, wl.sigma, wl.tau, wl.n)
    for m in range(M):
        assert_cycle_parity(got[m], ref[m], f"small64 cycle {m}")
    # FP64 residual sums against the oracle's cycle residuals
    assert np.allclose(np.sqrt(sums[:, 1]), rh[0, :, 1], rtol=1e-6)
    r_gpu = np.sqrt(sums[:, 0])
    assert np.allclose(r_gpu, rh[0, :, 0], rtol=1e-2, atol=1e-6)


def test_small64_full_run():
    wl = WORKLOADS["small64"]
    announce("small64 full run, eed4_inpaint vs oracle")
    pr = make_problem(wl.H, wl.W, wl.n_ellipses, wl.ramp, wl.noise_std, wl.density, wl.seed_base)
    ref, cyc, rh = oracle.inpaint(pr["u_init"], pr["mask"], pr["known"], wl.lam, wl.sigma,
                                  wl.tau, wl.n, wl.M)
    u = to_dev(pr["u_init"])
    st, hist = eed4.eed4_inpaint(u, to_dev(pr["mask"]), to_dev(pr["known"]),
                                 eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, wl.M), history=True)
    got = u.cpu().numpy()
    print(f"small64 after {st.cycles} cycles: RMSE vs ground truth {rmse(got, pr['image']):.4f} "
          f"(oracle {rmse(ref, pr['image']):.4f})")
    assert st.cycles == wl.M
    assert_steady_parity(got, ref, f"small64 after {st.cycles} cycles")
    assert np.array_equal(got[pr["mask"] != 0], pr["known"][pr["mask"] != 0])
    assert np.allclose(hist[:, 0, 1], rh[:, 1], rtol=1e-5)


@pytest.mark.parametrize("kernel", ["strip", "tile"])
@pytest.mark.parametrize("H,W,sigma,lam", [
    (37, 53, 1.0, 0.05), (1, 1, 1.0, 0.1), (1, 100, 1.5, 0.05), (100, 1, 1.5, 0.05),
    (3, 5, 2.0, 0.03), (65, 33, 0.0, 0.1), (70, 130, 0.5, 0.02), (97, 67, 2.6, 0.05),
    (64, 64, 1.5, 0.03), (33, 129, 2.0, 0.02), (230, 190, 2.0, 0.02), (161, 250, 1.0, 0.05),
    (150, 121, 0.3, 0.04), (140, 200, 2.3, 0.05)])
def test_ragged_shapes_and_radii(H, W, sigma, lam, kernel):
    announce(f"ragged {H}x{W} sigma={sigma} kernel={kernel}")
    pr = make_problem(H, W, 3, True, 0.01, 0.1, 77 + H * 1000 + W)
    n, tau = 7, 0.05
    # two cycles: the second starts from a non-trivial state
    _, _, _, ck = oracle.inpaint(pr["u_init"], pr["mask"], pr["known"], lam, sigma, tau, n, 2,
                                 checkpoints=True)
    masks = np.repeat(pr["mask"][None], 2, 0)
    knowns = np.repeat(pr["known"][None], 2, 0)
    got, _ = gpu_cycle(ck, masks, knowns, lam, sigma, tau, n, KERNELS[kernel])
    ref, _ = oracle_cycle(ck, masks, knowns, lam, sigma, tau, n)
    for m in range(2):
        assert_cycle_parity(got[m], ref[m], f"{H}x{W} sigma {sigma} {kernel} cycle {m}")


@pytest.mark.parametrize("n", [1, 2, 3])
def test_short_cycles(n):
    announce(f"short cycle n={n}")
    pr = make_problem(40, 45, 4, True, 0.01, 0.08, 99 + n)
    st = pr["u_init"][None]
    got, _ = gpu_cycle(st, pr["mask"][None], pr["known"][None], 0.05, 1.0, 0.05, n)
    ref, _ = oracle_cycle(st, pr["mask"][None], pr["known"][None], 0.05, 1.0, 0.05, n)
    assert_cycle_parity(got, ref, f"short cycle n={n}")


def test_constant_image_is_stationary_bitwise():
    announce("constant image")
    H, W, c = 70, 90, np.float32(0.3721)
    u0 = np.full((H, W), c, np.float32)
    mask = np.zeros((H, W), np.uint8)
    mask[5, 7] = 1
    u = to_dev(u0)
    eed4.eed4_inpaint(u, to_dev(mask), to_dev(u0), eed4.params(0.05, 2.0, 0.05, 10, 3))
    assert np.array_equal(u.cpu().numpy(), u0)


def test_deterministic_and_graph_equivalent():
    announce("determinism, graph vs direct launches")
    pr = make_problem(200, 150, 10, True, 0.01, 0.05, 4242)
    outs = []
    for flags in (0, 0, eed4.EED4_NO_GRAPH):
        u = to_dev(pr["u_init"])
        eed4.eed4_inpaint(u, to_dev(pr["mask"]), to_dev(pr["known"]),
                          eed4.params(0.03, 1.5, 0.05, 15, 4, flags=flags))
        outs.append(u.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[2])


def test_equal_size_batch_matches_single_images():
    announce("equal-size batch vs single images")
    wl = WORKLOADS["adjoint16"]
    b = make_batch(wl, B=3, shape=(96, 80))
    p = eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, 3, flags=eed4.EED4_FORCE_SHAPE(3))
    u = to_dev(b["u_init"])
    eed4.eed4_inpaint(u, to_dev(b["mask"]), to_dev(b["known"]), p)
    batch = u.cpu().numpy()
    for i in range(3):
        ui = to_dev(b["u_init"][i])
        eed4.eed4_inpaint(ui, to_dev(b["mask"][i]), to_dev(b["known"][i]), p)
        assert np.array_equal(ui.cpu().numpy(), batch[i])


def test_stop_rule_and_steady_state_512():
    wl = WORKLOADS["single512"]
    announce("single512 to relative residual 1e-4, then oracle at equal cycle count")
    pr = make_problem(wl.H, wl.W, wl.n_ellipses, wl.ramp, wl.noise_std, wl.density, wl.seed_base)
    u = to_dev(pr["u_init"])
    st, hist = eed4.eed4_inpaint(u, to_dev(pr["mask"]), to_dev(pr["known"]),
                                 eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, wl.M, tol=wl.tol),
                                 history=True)
    got = u.cpu().numpy()
    rel = hist[:, 0, 0] / hist[:, 0, 1]
    print(f"single512: {st.cycles} cycles, final relative residual {st.rel_residual:.3e}")
    assert st.cycles < wl.M and st.rel_residual < wl.tol
    assert rel[-1] < wl.tol and np.all(rel[:-1] >= wl.tol)
    ref, cyc, oh = oracle.inpaint(pr["u_init"], pr["mask"], pr["known"], wl.lam, wl.sigma,
                                  wl.tau, wl.n, st.cycles)
    orel = oh[:, 0] / oh[:, 1]
    gap = float(np.abs(rel / orel - 1).max())
    print(f"single512: RMSE vs ground truth {rmse(got, pr['image']):.4f}; relative residuals "
          f"within {gap:.2e} of FP64; oracle's last two {orel[-2]:.6e} {orel[-1]:.6e}")
    assert_steady_parity(got, ref, f"single512 at {st.cycles} cycles")
    # the FP64 run takes the same stop decision at every cycle: its residual history is
    # within 1e-3 of the GPU's, and no cycle's residual lies that close to tol
    assert gap <= 1e-3
    assert np.all(np.abs(orel / wl.tol - 1) > 5 * gap)
    assert orel[-1] < wl.tol and np.all(orel[:-1] >= wl.tol)


def test_abs_tol_stop_rule_matches_oracle():
    # plain residual ||u^{m,n} - u^{m,0}||_2 < tol (EED4_ABS_TOL), as Sec. 3.3 states it
    pr = make_problem(96, 80, 8, True, 0.01, 0.05, 808)
    lam, sigma, tau, n, M = 0.04, 1.5, 0.05, 10, 150
    # tol goes halfway (geometrically) between the FP64 residual of the first cycle below
    # 1e-2 and the smallest one before it (consecutive cycles are about 3 % apart), so the
    # FP32 path, whose residuals are within 2e-3 of FP64 (asserted), must stop at the same
    # cycle as the oracle
    _, _, oh = oracle.inpaint(pr["u_init"], pr["mask"], pr["known"], lam, sigma, tau, n, M)
    ores = oh[:, 0]
    c = int(np.argmax(ores < 1e-2))
    assert 0 < c < M - 1 and ores[c] < ores[:c].min()
    tol = float(np.sqrt(ores[c] * ores[:c].min()))
    announce(f"absolute stop rule, 96x80, tol {tol:.6e} (oracle stops after cycle {c + 1})")
    u = to_dev(pr["u_init"])
    st, hist = eed4.eed4_inpaint(u, to_dev(pr["mask"]), to_dev(pr["known"]),
                                 eed4.params(lam, sigma, tau, n, M, tol=tol,
                                             flags=eed4.EED4_ABS_TOL), history=True)
    got = u.cpu().numpy()
    res = hist[:, 0, 0]
    gap = float(np.abs(res / ores[:len(res)] - 1).max())
    print(f"absolute stop: GPU {st.cycles} cycles (residual {st.residual:.4e}), oracle {c + 1}; "
          f"residuals within {gap:.2e} of FP64")
    assert gap <= 2e-3
    assert st.cycles == c + 1
    assert res[-1] < tol and np.all(res[:-1] >= tol)
    assert st.residual == pytest.approx(res[-1], rel=1e-6)
    _, ocyc, _ = oracle.inpaint(pr["u_init"], pr["mask"], pr["known"], lam, sigma, tau, n, M,
                                tol=tol, abs_tol=True)
    assert ocyc == c + 1
    ref, _, _ = oracle.inpaint(pr["u_init"], pr["mask"], pr["known"], lam, sigma, tau, n,
                               st.cycles)
    assert_steady_parity(got, ref, f"absolute stop at {st.cycles} cycles")


@pytest.mark.parametrize("tol", [0.0, 1e-4])
def test_divergence_is_reported(tol):
    # tau = 0.4 is far beyond the bound 1/16 (allowed by flag): the state
    # overflows FP32 within about 45 steps, and the call must say so
    announce(f"divergence at tau 0.4, tol {tol}")
    pr = make_problem(64, 64, 5, False, 0.01, 0.05, 77)
    u = to_dev(pr["u_init"])
    with pytest.raises(eed4.EED4Error) as err:
        eed4.eed4_inpaint(u, to_dev(pr["mask"]), to_dev(pr["known"]),
                          eed4.params(0.05, 1.0, 0.4, 10, 8, tol=tol,
                                      flags=eed4.EED4_ALLOW_LARGE_TAU))
    assert err.value.code == eed4._lib.EED4_EDIVERGED


def test_concurrent_host_threads():
    # two host threads in eed4_inpaint at once (ctypes drops the GIL), each on
    # its own stream: graph capture is shared per process and must not clash
    import threading
    announce("two host threads calling eed4_inpaint concurrently")
    probs = [make_problem(160, 200, 6, True, 0.01, 0.05, 900 + i) for i in range(2)]
    p = eed4.params(0.04, 1.5, 0.05, 10, 6)

    def run(pr, stream=None):
        u = to_dev(pr["u_init"])
        eed4.eed4_inpaint(u, to_dev(pr["mask"]), to_dev(pr["known"]), p, stream=stream)
        return u

    ref = [run(pr).cpu().numpy() for pr in probs]
    torch.cuda.synchronize()
    for _ in range(3):
        streams = [torch.cuda.Stream() for _ in probs]
        outs, errs = [None, None], []

        def work(i):
            try:
                with torch.cuda.stream(streams[i]):
                    outs[i] = run(probs[i], streams[i])
                streams[i].synchronize()
            except Exception as exc:        # reported below, on the main thread
                errs.append(exc)

        ts = [threading.Thread(target=work, args=(i,)) for i in range(2)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        assert not errs, errs
        for i in range(2):
            assert np.array_equal(outs[i].cpu().numpy(), ref[i])


def test_strip_and_tile_kernels_agree_bitwise():
    # both kernel families form every value with the same operations in the same order, so
    # the result does not depend on which shape the autotuner picks
    announce("strip vs tile kernel, 300x260, 3 cycles")
    pr = make_problem(300, 260, 12, True, 0.01, 0.04, 555)
    outs = []
    for f in (eed4.EED4_FORCE_SHAPE(3), eed4.EED4_TILE_KERNEL):
        u = to_dev(pr["u_init"])
        eed4.eed4_inpaint(u, to_dev(pr["mask"]), to_dev(pr["known"]),
                          eed4.params(0.03, 1.5, 0.05, 15, 3, flags=f))
        outs.append(u.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("H,W,sigma", [(148, 61, 2.0), (150, 70, 2.0), (160, 130, 1.0),
                                         (200, 66, 0.0), (300, 40, 2.6), (170, 50, 0.3),
                                         (190, 90, 1.3), (260, 45, 2.3)])
def test_strips_streaming_up_agree_bitwise(H, W, sigma):
    # strips of >= 64 rows stream their odd segments bottom up (the last one from beyond
    # the bottom edge, mirrored, when the segment count is even); every value must equal
    # the tile kernel's, which does not stream at all
    announce(f"up/down strip segments vs tiles, {H}x{W}, sigma={sigma}")
    pr = make_problem(H, W, 6, True, 0.01, 0.05, 950 + H)
    outs = {}
    for shape in (0, 3, 4, 7):
        u = to_dev(pr["u_init"])
        st, hist = eed4.eed4_inpaint(u, to_dev(pr["mask"]), to_dev(pr["known"]),
                                     eed4.params(0.03, sigma, 0.05, 7, 3,
                                                 flags=eed4.EED4_FORCE_SHAPE(shape)),
                                     history=True)
        outs[shape] = (u.cpu().numpy(), hist)
    for shape in (3, 4, 7):
        assert np.array_equal(outs[shape][0], outs[0][0]), eed4.SHAPE_NAMES[shape]
        # the FP64 residual partials add rows in another order: equal to rounding only
        np.testing.assert_allclose(outs[shape][1], outs[0][1], rtol=1e-12, atol=0)


@pytest.mark.parametrize("H,W,B", [(300, 260, 1), (96, 80, 4)])
def test_every_step_shape_and_the_autotuned_default(H, W, B):
    announce(f"all step shapes and the autotuned default, {B} x {H}x{W}")
    b = {k: np.stack([make_problem(H, W, 8, True, 0.01, 0.05, 600 + i)[k] for i in range(B)])
         for k in ("mask", "known", "u_init")}
    outs = {}
    for shape in list(range(len(eed4.SHAPE_NAMES))) + [None]:
        flags = 0 if shape is None else eed4.EED4_FORCE_SHAPE(shape)
        u = to_dev(b["u_init"])
        eed4.eed4_inpaint(u, to_dev(b["mask"]), to_dev(b["known"]),
                          eed4.params(0.03, 1.5, 0.05, 9, 2, flags=flags))
        outs[shape] = u.cpu().numpy()
    for sh in range(len(eed4.SHAPE_NAMES)):
        assert np.array_equal(outs[sh], outs[0]), eed4.SHAPE_NAMES[sh]   # same arithmetic
    assert np.array_equal(outs[None], outs[0])


@pytest.mark.parametrize("shape", [2, 3, 5, 7])
@pytest.mark.parametrize("H,W", [(1, 70000), (50000, 3)])
def test_long_thin_images_one_cycle(shape, H, W):
    # the most strips (or segments) per image along one axis, the fewest along
    # the other: strip and row offsets at their largest for the image size
    announce(f"long thin {H}x{W}, shape {eed4.SHAPE_NAMES[shape]}")
    pr = make_problem(H, W, 6, True, 0.01, 0.05, 321 + H)
    u0 = np.where(pr["mask"] != 0, pr["known"], pr["u_init"]).astype(np.float32)
    got, sums = gpu_cycle(u0[None], pr["mask"][None], pr["known"][None], 0.04, 1.5, 0.05, 6,
                          flags=eed4.EED4_FORCE_SHAPE(shape))
    ref, rh = oracle_cycle(u0[None], pr["mask"][None], pr["known"][None], 0.04, 1.5, 0.05, 6)
    assert_cycle_parity(got[0], ref[0], f"{H}x{W} {eed4.SHAPE_NAMES[shape]}")
    assert np.allclose(np.sqrt(sums[0, 1]), rh[0, 0, 1], rtol=1e-6)


def test_large4096_first_cycle_parity():
    # full size, in the kernel shapes the benchmark runs: the autotuner's usual choices
    # (28- and 64-row strips) and the shape eed4_inpaint picks in this process
    wl = WORKLOADS["large4096"]
    announce("large4096 first cycle (bench launch configuration) vs oracle")
    pr = make_problem(wl.H, wl.W, wl.n_ellipses, wl.ramp, wl.noise_std, wl.density, wl.seed_base)
    u0 = np.where(pr["mask"] != 0, pr["known"], pr["u_init"]).astype(np.float32)
    ref, rh = oracle_cycle(u0[None], pr["mask"][None], pr["known"][None], wl.lam, wl.sigma,
                           wl.tau, wl.n)
    u = to_dev(u0)
    eed4.eed4_inpaint(u, to_dev(pr["mask"]), to_dev(pr["known"]),
                      eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, 1))
    tuned = eed4.eed4_step_shape(1, wl.H, wl.W, eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, 1))
    got_tuned = u.cpu().numpy()
    assert_cycle_parity(got_tuned, ref[0], f"large4096 first cycle, autotuned "
                                           f"{eed4.SHAPE_NAMES[tuned]}")
    for shape in (3, 5):
        got, sums = gpu_cycle(u0[None], pr["mask"][None], pr["known"][None], wl.lam, wl.sigma,
                              wl.tau, wl.n, flags=eed4.EED4_FORCE_SHAPE(shape))
        assert_cycle_parity(got[0], ref[0], f"large4096 first cycle {eed4.SHAPE_NAMES[shape]}")
        assert np.allclose(np.sqrt(sums[0, 1]), rh[0, 0, 1], rtol=1e-6)
        if shape == tuned:
            assert np.array_equal(got[0], got_tuned)


def test_empty_mask_smoothing_case():
    # no known pixels: the evolution is the smoothing variant (Sec. 3.3); mean grey value is
    # preserved (P 1 = 0 and P symmetric) and the cycle matches the oracle
    announce("empty mask (smoothing), 90x130, 2 cycles")
    pr = make_problem(90, 130, 6, True, 0.01, 0.05, 4242)
    mask = np.zeros((90, 130), np.uint8)
    st = pr["image"][None].astype(np.float32)
    got, _ = gpu_cycle(st, mask[None], st, 0.05, 1.0, 0.05, 10)
    ref, _ = oracle_cycle(st, mask[None], st, 0.05, 1.0, 0.05, 10)
    assert_cycle_parity(got, ref, "empty mask")
    assert abs(float(got.astype(np.float64).mean()) - float(st.astype(np.float64).mean())) < 1e-6


def test_all_known_mask_is_held():
    announce("all-known mask, 50x70")
    pr = make_problem(50, 70, 4, True, 0.01, 0.05, 4343)
    mask = np.ones((50, 70), np.uint8)
    u = to_dev(np.full((50, 70), 0.5, np.float32))
    st = eed4.eed4_inpaint(u, to_dev(mask), to_dev(pr["image"]), eed4.params(0.05, 1.0, 0.05, 10, 3))[0]
    assert np.array_equal(u.cpu().numpy(), pr["image"])
    assert st.residual == 0.0


@pytest.mark.parametrize("shape", [2, 5])
def test_resume_from_a_result_is_bitwise_continuation(shape):
    # the whole FSI state between cycles is u^{m,0} (each cycle restarts with
    # u^{m,-1} := u^{m,0}, Sec. 3.3), so a run of a cycles resumed for b more equals a run of
    # a + b cycles bitwise, checkpoints included
    a, b = 3, 4
    announce(f"resume: {a} + {b} cycles vs {a + b}, shape {eed4.SHAPE_NAMES[shape]}")
    pr = make_problem(150, 170, 10, True, 0.01, 0.05, 7070 + shape)
    mask, known = to_dev(pr["mask"]), to_dev(pr["known"])
    fl = eed4.EED4_FORCE_SHAPE(shape)
    u = to_dev(pr["u_init"])
    ck = torch.zeros((a + b, 150, 170), dtype=torch.float32, device="cuda")
    eed4.eed4_inpaint(u, mask, known, eed4.params(0.03, 1.5, 0.05, 10, a + b, flags=fl), ckpt=ck)
    v = to_dev(pr["u_init"])
    ck1 = torch.zeros((a, 150, 170), dtype=torch.float32, device="cuda")
    eed4.eed4_inpaint(v, mask, known, eed4.params(0.03, 1.5, 0.05, 10, a, flags=fl), ckpt=ck1)
    ck2 = torch.zeros((b, 150, 170), dtype=torch.float32, device="cuda")
    eed4.eed4_inpaint(v, mask, known, eed4.params(0.03, 1.5, 0.05, 10, b, flags=fl), ckpt=ck2)
    torch.cuda.synchronize()
    assert torch.equal(u, v)
    assert torch.equal(ck[:a], ck1) and torch.equal(ck[a:], ck2)


@pytest.mark.parametrize("tol", [0.0, 1e-4])
def test_nan_in_known_values_is_reported(tol):
    # a NaN among the stored grey values reaches the cycle residual: the call must return
    # EED4_EDIVERGED (an ordinary kernel exit: the arithmetic just carries the NaN)
    announce(f"NaN in known values, tol {tol}")
    pr = make_problem(64, 80, 5, True, 0.01, 0.05, 99)
    known = pr["known"].copy()
    ky, kx = np.argwhere(pr["mask"] != 0)[len(np.argwhere(pr["mask"] != 0)) // 2]
    known[ky, kx] = np.nan
    u = to_dev(pr["u_init"])
    with pytest.raises(eed4.EED4Error) as err:
        eed4.eed4_inpaint(u, to_dev(pr["mask"]), to_dev(known),
                          eed4.params(0.05, 1.0, 0.05, 10, 3, tol=tol))
    assert err.value.code == eed4._lib.EED4_EDIVERGED
    assert bool(torch.isnan(u[ky, kx]))


def test_run_to_tolerance_equals_fixed_cycle_run():
    # a run to a tolerance queues each next cycle before reading the residual and alternates
    # two state buffers; its state, checkpoints and residual history must equal a run of the
    # same number of fixed cycles bitwise, whichever buffer the last cycle ended in
    pr = make_problem(120, 150, 8, True, 0.01, 0.05, 5150)
    mask, known = to_dev(pr["mask"]), to_dev(pr["known"])
    lam, sigma, tau, n, M = 0.04, 1.5, 0.05, 10, 60
    seen = set()
    for tol in (3e-3, 2e-3, 1.5e-3, 1e-3):
        announce(f"run to tolerance {tol} vs fixed cycles, 120x150")
        u = to_dev(pr["u_init"])
        ck = torch.full((M, 120, 150), -7.0, dtype=torch.float32, device="cuda")
        st, hist = eed4.eed4_inpaint(u, mask, known, eed4.params(lam, sigma, tau, n, M, tol=tol),
                                     ckpt=ck, history=True)
        c = st.cycles
        assert 1 < c < M
        v = to_dev(pr["u_init"])
        ck2 = torch.zeros((c, 120, 150), dtype=torch.float32, device="cuda")
        st2, hist2 = eed4.eed4_inpaint(v, mask, known, eed4.params(lam, sigma, tau, n, c),
                                       ckpt=ck2, history=True)
        torch.cuda.synchronize()
        assert torch.equal(u, v)
        assert torch.equal(ck[:c], ck2)
        assert np.array_equal(hist, hist2)
        assert st.residual == st2.residual and st.rel_residual == st2.rel_residual
        seen.add(c % 2)
    assert seen == {0, 1}, "both buffer parities should be covered"
