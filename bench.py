#!/usr/bin/env python3
"""Throughput of fourth-order EED inpainting with FSI on one MI355X.

A timed "step" is one FSI cycle (n fused inner steps plus the FP64 residual)
over the 4096 x 4096 synthetic workload (200 ellipses + ramp + noise, 3%
mask, sigma 2, lambda 0.02, tau 0.05, n 15), run through eed4_inpaint with
the cycle replayed as a hipGraph.  Inputs are resident in HBM before timing.

The JSON line carries:
  value      pixel-updates/s of the whole timed region (Mpixel-updates/s)
  roofline   the fused step kernel: algorithmic bytes per launch (13 B per
             pixel-update: read u^k, read u^{k-1}, write u^{k+1}, read the
             u8 mask) over its average launch time, measured here with HIP
             events around back-to-back eed4_fsi_step launches on the same
             stream, against the 8 TB/s HBM peak; traffic from the committed
             rocprofv3 counter summary when it matches the current kernel
  roofline.out_of_cache  the same fused step on an 8192 x 8192 image, whose
             832 MiB working set cannot stay in the 256 MB Infinity Cache
  cpu_baseline  the FP64 oracle on the host cores, one cycle of the same image;
             beside it a single-thread sample and the oracle rate on the
             other workloads (64^2, 512^2, 16 x 256^2, part of the uneven batch)
  fp64_error  the FP32 GPU result against the FP64 oracle for every reported
             result (relative L2, largest elementwise error, RMSE): the first
             cycle of the timed image here, and one object inside each of the
             objects below
  adjoint_forward_ratio  backward/forward time on 16 x 256 x 256 (30 cycles of 10)
  batched    64 uneven images: one batched call vs 64 single-image calls
  variants   fused step time of each tensor variant (Table 7 diffusivities,
             Sec. 3.1 mu3 choices) on the workload image
  workloads  colour (channel-wise RGB) and scratch-removal inpainting, 512x512,
             and the 512x512 single image run to its relative-residual tolerance
The oracle runs behind every fp64_error object are done after all GPU
timing, so the host work does not let the GPU clock drop between timings.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_UPDATE = 13          # 4 (u^k) + 4 (u^{k-1}) + 4 (u^{k+1}) + 1 (mask)
HBM_PEAK_GBS = 8000.0          # MI355X published HBM3E bandwidth
# MI355X FP32 vector peak: 256 CUs x 4 SIMDs x 32 FP32 lanes x 2 flop (FMA) x 2.4 GHz
# = 157.3 TFLOP/s.  Plain (non-packed) v_fma_f32 issues at that rate on gfx950: a
# wave64 FMA retires every ~2 SIMD cycles (measured; transcendentals ~8.8 cycles).
ALU_PEAK_TFLOPS = 256 * 4 * 32 * 2 * 2.4e9 / 1e12


def flops_per_update(R):
    """Algorithmic FP32 flops of one pixel-update (FMA = 2): separable blur
    4(2R+1), gradient 2, tensor 15, Hessian 11, contraction 24, outer
    differences 13, FSI update and hold 5."""
    return 4 * (2 * R + 1) + 70
# kernel behind each fused-step shape (template arguments: radius, residual
# variant, least segment rows, columns per lane; or tile width and height)
STRIP_GEOMETRY = {"strip": (64, 1), "strip_tall": (136, 1), "strip_short": (28, 1),
                  "strip_tiny": (8, 1), "strip_wide": (64, 2), "strip_wide_short": (28, 2)}
TILE_GEOMETRY = {"tile64x32": (64, 32), "tile64x16": (64, 16), "tile32x32": (32, 32),
                 "tile32x16": (32, 16), "tile16x16": (16, 16)}


def kernel_name(shape_name, R):
    if shape_name in STRIP_GEOMETRY:
        rows, cpl = STRIP_GEOMETRY[shape_name]
        return f"strip_kernel<{R}, false, {rows}, {cpl}>"
    tw, th = TILE_GEOMETRY[shape_name]
    return f"step_kernel<{R}, {tw}, {th}>"


KERNEL_SOURCES = ("paper_2006_10406_amd/csrc/eed4_strip.h",
                  "paper_2006_10406_amd/csrc/eed4_forward.hip",
                  "paper_2006_10406_amd/csrc/eed4_tile.h",
                  "paper_2006_10406_amd/csrc/eed4_pointwise.h",
                  "paper_2006_10406_amd/csrc/eed4_internal.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_large4096_traffic.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_sha():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kname):
    """HBM bytes per launch of kernel kname from the committed counter summary,
    or None when it is missing or was taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != kernel_source_sha():
        return None
    return t.get("kernels", {}).get(kname, {}).get("bytes_per_launch")


def fp64_error(got, ref):
    """FP32 result against the FP64 oracle: relative L2, largest elementwise error, RMSE."""
    import numpy as np
    a = np.asarray(got, np.float64)
    b = np.asarray(ref, np.float64)
    d = a - b
    return {"rel_l2": float(np.linalg.norm(d) / max(np.linalg.norm(b), 1e-300)),
            "max_abs": float(np.abs(d).max()) if d.size else 0.0,
            "rmse": float(np.sqrt(np.mean(d * d))) if d.size else 0.0}


def quality(got, truth):
    """Reconstruction against the synthetic ground truth: MSE and AAE (mean absolute error),
    the error measures of the paper's experiments (Sec. 4), for grey values in [0, 1] and
    scaled to the 0..255 grey range the paper's tables use."""
    import numpy as np
    d = np.asarray(got, np.float64) - np.asarray(truth, np.float64)
    mse, aae = float(np.mean(d * d)), float(np.mean(np.abs(d)))
    return {"mse": mse, "aae": aae, "mse_255": mse * 255.0 ** 2, "aae_255": aae * 255.0,
            "against": "the synthetic ground-truth image"}


def grad_error(got, ref):
    """A gradient against the oracle adjoint: relative L2 and the largest elementwise error
    relative to the largest oracle value."""
    import numpy as np
    a = np.asarray(got, np.float64)
    b = np.asarray(ref, np.float64)
    scale = float(np.abs(b).max()) if b.size else 0.0
    return {"rel_l2": float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)),
            "max_abs_rel": float(np.abs(a - b).max() / scale) if scale > 0 else 0.0}


def timed_oracle(fn, updates):
    """Runs fn() once; returns (Mpixel-updates/s, seconds, result)."""
    t0 = time.perf_counter()
    res = fn()
    dt = time.perf_counter() - t0
    return updates / dt / 1e6, dt, res


def cpu_baseline(pr, wl):
    """The FP64 oracle on the host: one cycle of the timed image on every core (the
    reported value), a single-thread sample of it, and the rate on the other workloads.
    Returns (cpu_baseline object, the oracle's first cycle of the timed image)."""
    import oracle
    from synth import WORKLOADS, make_batch, make_problem, make_uneven_batch
    n = wl.n
    cores = oracle.num_threads()
    one_cycle = lambda p, w, M=1: (lambda: oracle.inpaint(p["u_init"], p["mask"], p["known"],
                                                          w.lam, w.sigma, w.tau, w.n, M)[0])
    val, dt, first = timed_oracle(one_cycle(pr, wl), pr["u_init"].size * n)
    out = {"value": val, "unit": "Mpixel-updates/s", "cores": cores, "kind": "oracle",
           "cpu": cpu_model(),
           "sample": f"one FSI cycle ({n} steps) of the full {wl.H}x{wl.W} workload image, "
                     f"FP64, {dt:.1f} s"}
    # single thread: rows 0..511 of the same image, one cycle (a cycle of a row band costs
    # what the same rows cost inside the full image, up to the mirrored border rows)
    band = {k: pr[k][:512] for k in ("u_init", "mask", "known")}
    oracle.set_num_threads(1)
    try:
        v1, d1, _ = timed_oracle(one_cycle(band, wl), band["u_init"].size * n)
        per = {}
        # the other workloads, each at 1 thread and on every core: 64^2 whole (20 cycles of
        # 10), 512^2 one cycle of 40, 16 x 256^2 one cycle of 10, and 4 images of the uneven
        # batch (one cycle of 15)
        w1 = WORKLOADS["small64"]
        p1 = make_problem(w1.H, w1.W, w1.n_ellipses, w1.ramp, w1.noise_std, w1.density,
                          w1.seed_base)
        w2 = WORKLOADS["single512"]
        p2 = make_problem(w2.H, w2.W, w2.n_ellipses, w2.ramp, w2.noise_std, w2.density,
                          w2.seed_base)
        w5 = WORKLOADS["adjoint16"]
        p5 = make_batch(w5)
        w4 = WORKLOADS["batch64"]
        p4 = make_uneven_batch(w4)[:4]
        cases = [("small64", w1, [p1], w1.M, f"{w1.M} cycles of {w1.n}, 64x64"),
                 ("single512", w2, [p2], 1, f"one cycle of {w2.n}, 512x512"),
                 ("adjoint16", w5, [p5], 1, f"one cycle of {w5.n}, 16 x 256x256"),
                 ("batch64", w4, p4, 1, "one cycle of 15 on images 0-3 of the uneven batch")]
        for name, w, probs, M, what in cases:
            upd = sum(q["u_init"].size for q in probs) * w.n * M
            rates = {}
            for nt in (1, cores):
                oracle.set_num_threads(nt)
                t0 = time.perf_counter()
                for q in probs:
                    one_cycle(q, w, M)()
                rates[nt] = upd / (time.perf_counter() - t0) / 1e6
            per[name] = {"single_thread": round(rates[1], 2), "all_cores": round(rates[cores], 2),
                         "sample": what}
    finally:
        oracle.set_num_threads(cores)
    out["single_thread"] = {"value": round(v1, 2), "cores": 1,
                            "sample": f"one FSI cycle of rows 0-511 of the {wl.H}x{wl.W} image, "
                                      f"{d1:.1f} s"}
    out["per_workload"] = per
    return out, first


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def copy_bandwidth(torch):
    """Achieved GB/s (read + write bytes) of a plain device-to-device copy:
    1 GiB (beyond the 256 MB Infinity Cache) and 64 MiB (one image plane)."""
    out = {}
    for label, nbytes in (("copy_1GiB", 1 << 30), ("copy_64MiB", 64 << 20)):
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        out[label] = round(2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
        del a, b
    out["unit"] = "GB/s"
    return out


def aligned_workspace(torch, nbytes, dev):
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    return buf[(-buf.data_ptr()) % 256:]


def seeded_direction(torch, shape, seed, dev):
    """dL/du^M for the adjoint timings: seeded N(0, 1e-6) values, the same every run."""
    import numpy as np
    g = np.random.default_rng(seed + 7919).standard_normal(shape).astype(np.float32) * 1e-3
    return torch.from_numpy(g).to(dev)


def adjoint_ratio(eed4, torch, args):
    """Forward (with per-cycle checkpoints) vs backward time on 16 x 256 x 256."""
    from synth import WORKLOADS, make_batch
    wl = WORKLOADS["adjoint16"]
    b = make_batch(wl)
    dev = "cuda"
    u0 = torch.from_numpy(b["u_init"]).to(dev)
    mask = torch.from_numpy(b["mask"]).to(dev)
    known = torch.from_numpy(b["known"]).to(dev)
    B, H, W = u0.shape
    p = eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, wl.M)
    ck = torch.empty((wl.M, B, H, W), dtype=torch.float32, device=dev)
    gu = seeded_direction(torch, (B, H, W), wl.seed_base, dev)
    gk = torch.empty_like(gu)
    gi = torch.empty_like(gu)
    gl = torch.empty(B, device=dev)
    wsf = aligned_workspace(torch, eed4.eed4_workspace_size(eed4.EED4_OP_INPAINT, B, H, W, p), dev)
    wsb = aligned_workspace(torch, eed4.eed4_workspace_size(eed4.EED4_OP_BACKWARD, B, H, W, p),
                            dev)
    u = u0.clone()

    def fwd():
        u.copy_(u0)
        eed4.eed4_inpaint(u, mask, known, p, ckpt=ck, ws=wsf)

    def bwd():
        eed4.eed4_backward(ck, mask, known, p, wl.M, gu, gk, gi, gl, ws=wsb)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    tf = timed(fwd, 3)
    tb = timed(bwd, 3)
    upd = B * H * W * wl.n * wl.M
    res = {"forward_ms": tf, "backward_ms": tb, "ratio": tb / tf,
           "forward_mpix_updates_s": upd / (tf * 1e-3) / 1e6,
           "workload": f"adjoint16: {B} x {H}x{W}, {wl.M} cycles of {wl.n}, checkpoint per cycle"}
    # image 0 for the FP64 check: forward state after M cycles and the three gradients
    i0 = {"u": u[0].cpu().numpy(), "ck": ck[:, 0].cpu().numpy(), "gu": gu[0].cpu().numpy(),
          "gk": gk[0].cpu().numpy(), "gi": gi[0].cpu().numpy(), "gl": float(gl[0])}

    def check():
        import numpy as np
        import oracle
        pr = {k: b[k][0] for k in ("u_init", "mask", "known")}
        ref, _, _ = oracle.inpaint(pr["u_init"], pr["mask"], pr["known"], wl.lam, wl.sigma,
                                   wl.tau, wl.n, wl.M)
        ogk, ogi, ogl = oracle.backward(i0["ck"].astype(np.float64), pr["mask"], pr["known"],
                                        wl.lam, wl.sigma, wl.tau, wl.n, i0["gu"])
        m = pr["mask"] != 0
        return {"image": 0, "forward_after_30_cycles": fp64_error(i0["u"], ref),
                "dL_df": grad_error(i0["gk"][m], ogk[m]),
                "dL_du_init": grad_error(i0["gi"][~m], ogi[~m]),
                "dL_dlambda": {"gpu": i0["gl"], "oracle": float(ogl),
                               "rel": abs(i0["gl"] - float(ogl)) / max(abs(float(ogl)), 1e-300)},
                "reference": "FP64 oracle forward from the same input; oracle adjoint on the "
                             "GPU's own checkpoints"}
    return res, check


def probe(eed4, torch, u_init, mask, wl):
    """For every fused-step shape (each is its own kernel), launch the step
    3 x n times; then copy 64 MiB device to device."""
    a, b, c = u_init.clone(), u_init.clone(), u_init.clone()
    roles = lambda k: (a, a, b) if k == 0 else ((b, a, c) if k == 1 else
                                                 ((b, c, c) if k % 2 else (c, b, b)))
    for shape, name in enumerate(eed4.SHAPE_NAMES):
        ps = eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, 1, flags=eed4.EED4_FORCE_SHAPE(shape))
        for _ in range(3):
            for k in range(wl.n):
                cur, prev, out = roles(k)
                eed4.eed4_fsi_step(cur, prev, out, mask, ps, k)
        torch.cuda.synchronize()
        log(f"probe: {name}")
    # the tensor-variant kernel (one kernel serves every variant)
    ps = eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, 1,
                     flags=eed4.EED4_DIFFUSIVITY(eed4.EED4_PERONA_MALIK_EXP)
                     | eed4.EED4_MU3(eed4.EED4_MU3_ARITHMETIC))
    for _ in range(3):
        for k in range(wl.n):
            cur, prev, out = roles(k)
            eed4.eed4_fsi_step(cur, prev, out, mask, ps, k)
    torch.cuda.synchronize()
    log("probe: tensor-variant kernel")
    src = torch.ones(16 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"probe done: {3 * wl.n} step launches per shape, one copy of {src.numel() * 4} bytes")


def variants_timing(eed4, torch, u, mask, wl, stream, reps=2):
    """Fused step of every tensor variant (Table 7 diffusivity x Sec. 3.1 mu3 choice) on
    the workload image, back-to-back launches on one stream, median of three windows.
    The variants run strip_model_kernel<R, false> (60-column strips of >= 28 rows); the
    FOEED default is the tuned kernel of the main measurement."""
    H, W, n = wl.H, wl.W, wl.n
    a, b, c = u.clone(), u.clone(), u.clone()
    roles = lambda k: (a, a, b) if k == 0 else ((b, a, c) if k == 1 else
                                                 ((b, c, c) if k % 2 else (c, b, b)))
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    R = eed4.eed4_radius(wl.sigma)
    res = {"kernel": f"strip_model_kernel<{R}, false>", "unit": "us/launch",
           "bytes_per_launch": BYTES_PER_UPDATE * H * W, "per_variant": {}}
    for d, dn in enumerate(eed4.DIFFUSIVITY_NAMES):
        for r, rn in enumerate(eed4.MU3_NAMES):
            if d == 0 and r == 0:
                continue
            ps = eed4.params(wl.lam, wl.sigma, wl.tau, n, 1,
                             flags=eed4.EED4_DIFFUSIVITY(d) | eed4.EED4_MU3(r))
            for k in range(n):
                cur, prev, out = roles(k)
                eed4.eed4_fsi_step(cur, prev, out, mask, ps, k, stream=stream)
            windows = []
            for _ in range(3):
                e0.record(stream)
                for _ in range(reps):
                    for k in range(n):
                        cur, prev, out = roles(k)
                        eed4.eed4_fsi_step(cur, prev, out, mask, ps, k, stream=stream)
                e1.record(stream)
                torch.cuda.synchronize()
                windows.append(e0.elapsed_time(e1) / (reps * n))
            us = sorted(windows)[1] * 1e3
            gbs = BYTES_PER_UPDATE * H * W / (us * 1e-6) / 1e9
            res["per_variant"][f"{dn}/{rn}"] = {"us": round(us, 1),
                                                "hbm_frac": round(gbs / HBM_PEAK_GBS, 3)}
    return res


def variant_first_cycle(eed4, torch, pr, mask, known, wl, d=2, r=1):
    """One variant's (default: exponential Perona-Malik, arithmetic-mean mu3) first cycle of
    the workload image on the GPU, and the deferred FP64 check of it."""
    u = torch.from_numpy(pr["u_init"]).cuda()
    sums = torch.zeros((1, 2), dtype=torch.float64, device="cuda")
    eed4.eed4_fsi_cycle(u, mask, known, eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, 1,
                                                    flags=eed4.EED4_DIFFUSIVITY(d)
                                                    | eed4.EED4_MU3(r)), sums)
    got = u.cpu().numpy()

    def check():
        import oracle
        ref, _, _ = oracle.inpaint(pr["u_init"], pr["mask"], pr["known"], wl.lam, wl.sigma,
                                   wl.tau, wl.n, 1, diff=d, mu3=r)
        e = fp64_error(got, ref)
        e["variant"] = f"{eed4.DIFFUSIVITY_NAMES[d]}/{eed4.MU3_NAMES[r]}"
        e["sample"] = f"first FSI cycle of the {wl.H}x{wl.W} workload image"
        return e
    return check


def workload_throughput(eed4, torch, names=("rgb512", "scratch512_thin", "scratch512_thick")):
    """Colour (channel-wise, a batch of 3 planes) and scratch-removal workloads through
    eed4_inpaint: wl.M fixed cycles after a tuning call; pixel-updates/s counts every
    channel's pixels."""
    from synth import WORKLOADS, make_problem, make_workload_problem
    res = {}
    checks = []
    for name in names:
        wl = WORKLOADS[name]
        pr = make_workload_problem(wl)
        mask = torch.from_numpy(pr["mask"]).cuda()
        known = torch.from_numpy(pr["known"]).cuda()
        u0 = torch.from_numpy(pr["u_init"]).cuda()
        u = u0.clone()
        eed4.eed4_inpaint(u, mask, known, eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, 2))
        p = eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, wl.M)
        u = u0.clone()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        st, _ = eed4.eed4_inpaint(u, mask, known, p)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        px = u0.numel()
        B = px // (wl.H * wl.W)
        got = u.cpu().numpy()
        res[name] = {"mpix_updates_s": round(px * wl.n * st.cycles / (ms * 1e-3) / 1e6, 1),
                     "ms": round(ms, 3), "cycles": st.cycles, "planes": B,
                     "shape": eed4.SHAPE_NAMES[eed4.eed4_step_shape(B, wl.H, wl.W, p)],
                     "quality": quality(got, pr["image"])}
        # the colour planes are independent: channel 0 stands for the three
        got, q = (got[0], {k: pr[k][0] for k in ("u_init", "mask", "known")}) if B > 1 \
            else (got, pr)
        checks.append((name, deferred_run(got, q, wl, st.cycles,
                                          "channel 0" if B > 1 else "the image")))
    # the 512x512 single image run to the relative-residual tolerance (one host read of the
    # residual per cycle): time to convergence
    wl = WORKLOADS["single512"]
    pr = make_problem(wl.H, wl.W, wl.n_ellipses, wl.ramp, wl.noise_std, wl.density, wl.seed_base)
    mask = torch.from_numpy(pr["mask"]).cuda()
    known = torch.from_numpy(pr["known"]).cuda()
    u0 = torch.from_numpy(pr["u_init"]).cuda()
    p = eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, wl.M, tol=wl.tol)
    # warm-up: the same call (step-shape tuning, cycle graphs, the pinned residual buffer)
    u = u0.clone()
    eed4.eed4_inpaint(u, mask, known, p)
    times = []
    for _ in range(3):
        u = u0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, _ = eed4.eed4_inpaint(u, mask, known, p)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    ms = sorted(times)[1]                   # median of three runs
    res["single512_to_tol"] = {"cycles": st.cycles, "rel_residual": st.rel_residual,
                               "ms": round(ms, 2),
                               "mpix_updates_s": round(wl.H * wl.W * wl.n * st.cycles
                                                       / (ms * 1e-3) / 1e6, 1),
                               "tol": wl.tol, "cycle_len": wl.n,
                               "quality": quality(u.cpu().numpy(), pr["image"])}
    checks.append(("single512_to_tol", deferred_run(u.cpu().numpy(), pr, wl, st.cycles,
                                                    "the image")))
    return res, checks


def deferred_run(got, pr, wl, cycles, what):
    """Deferred FP64 check of a GPU run of `cycles` cycles: the oracle from the same input
    for the same number of cycles (equal cycle counts)."""
    def check():
        import oracle
        ref, _, _ = oracle.inpaint(pr["u_init"], pr["mask"], pr["known"], wl.lam, wl.sigma,
                                   wl.tau, wl.n, cycles)
        e = fp64_error(got, ref)
        e["sample"] = f"{what} after {cycles} cycles of {wl.n}, oracle at the same count"
        return e
    return check


def batched_vs_single(eed4, torch, cycles):
    """64 uneven images (sides U{128..1024}, 2..8% masks, sigma 1.5, lambda 0.03,
    n 15): one eed4_inpaint_batched call (autotuned queue kernels, graph)
    against 64 eed4_inpaint calls, same cycle count; throughput in
    Mpixel-updates/s and the largest RMSE between the two results."""
    from synth import WORKLOADS, make_uneven_batch
    wl = WORKLOADS["batch64"]
    probs = make_uneven_batch(wl)
    dev = "cuda"
    inits = [torch.from_numpy(p["u_init"]).to(dev) for p in probs]
    masks = [torch.from_numpy(p["mask"]).to(dev) for p in probs]
    knowns = [torch.from_numpy(p["known"]).to(dev) for p in probs]
    px = sum(p["u_init"].size for p in probs)
    p = eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, cycles)
    # warm both paths (the first batched call also runs the batched autotuner)
    us = [u.clone() for u in inits]
    eed4.eed4_inpaint_batched([(u, m, k, wl.lam) for u, m, k in zip(us, masks, knowns)],
                              eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, 1))
    # every image size tunes its own step shape on its first call: do that outside the timing
    for u, m, k in zip(inits, masks, knowns):
        eed4.eed4_inpaint(u.clone(), m, k, eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, 1))
    torch.cuda.synchronize()

    ub = [u.clone() for u in inits]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eed4.eed4_inpaint_batched([(u, m, k, wl.lam) for u, m, k in zip(ub, masks, knowns)], p)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    shape = eed4.eed4_autotune_batched([(u, m, k, wl.lam) for u, m, k in zip(ub, masks, knowns)],
                                       p)
    us = [u.clone() for u in inits]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for u, m, k in zip(us, masks, knowns):
        eed4.eed4_inpaint(u, m, k, p)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    diff = max(float(torch.sqrt(torch.mean((a - b) ** 2))) for a, b in zip(ub, us))
    same = all(bool(torch.equal(a, b)) for a, b in zip(ub, us))
    upd = px * wl.n * cycles
    res = {"workload": f"batch64: 64 images, {px} px, {cycles} cycles of {wl.n}",
           "batched_mpix_updates_s": upd / tb / 1e6, "per_image_mpix_updates_s": upd / ts / 1e6,
           "speedup": ts / tb, "batched_ms": tb * 1e3, "per_image_ms": ts * 1e3,
           "autotuned_shape": eed4.SHAPE_NAMES[shape], "max_rmse_between": diff,
           "bitwise_equal_to_per_image": same}
    # FP64 check of two sampled images: the smallest of the batch and one in the middle
    sizes = [q["u_init"].size for q in probs]
    picks = [int(min(range(len(probs)), key=lambda i: sizes[i])), len(probs) // 2]
    kept = [(i, ub[i].cpu().numpy()) for i in picks]

    def check():
        out = {}
        for i, got in kept:
            e = deferred_run(got, probs[i], wl, cycles, f"image {i} {probs[i]['u_init'].shape}")()
            out[f"image_{i}"] = e
        return out
    return res, check


def adjoint_probe(eed4, torch):
    """Backward passes for kernel traces: the 16 x 256x256 workload (30 cycles of 10) and one
    cycle of 15 on the 4096x4096 workload, each after its forward with checkpoints."""
    from synth import WORKLOADS, make_batch, make_problem

    def run(u0, mask, known, wl, M, label):
        B, H, W = u0.shape
        p = eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, M)
        ck = torch.empty((M, B, H, W), dtype=torch.float32, device="cuda")
        u = u0.clone()
        eed4.eed4_inpaint(u, mask, known, p, ckpt=ck)
        gu = seeded_direction(torch, (B, H, W), wl.seed_base, "cuda")
        gk, gi = torch.empty_like(gu), torch.empty_like(gu)
        gl = torch.empty(B, device="cuda")
        for rep in range(2):          # the first call also picks the reverse-step kernel
            torch.cuda.synchronize()
            t = time.perf_counter()
            eed4.eed4_backward(ck, mask, known, p, M, gu, gk, gi, gl)
            torch.cuda.synchronize()
            log(f"{label}: backward {(time.perf_counter() - t) * 1e3:.2f} ms")

    wl = WORKLOADS["adjoint16"]
    b = make_batch(wl)
    dev = lambda a: torch.from_numpy(a).cuda()
    run(dev(b["u_init"]), dev(b["mask"]), dev(b["known"]), wl, wl.M, "adjoint16")
    wl = WORKLOADS["large4096"]
    pr = make_problem(wl.H, wl.W, wl.n_ellipses, wl.ramp, wl.noise_std, wl.density, wl.seed_base)
    one = lambda a: torch.from_numpy(a).cuda()[None].contiguous()
    run(one(pr["u_init"]), one(pr["mask"]), one(pr["known"]), wl, 1, "large4096, one cycle")


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed FSI cycles")
    ap.add_argument("--warmup", type=int, default=300,
                    help="untimed FSI cycles (the GPU clock needs a few hundred ms of sustained work to settle)")
    ap.add_argument("--kernel-reps", type=int, default=20,
                    help="cycles of back-to-back eed4_fsi_step launches for the roofline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-workloads", action="store_true")
    ap.add_argument("--no-out-of-cache", action="store_true")
    ap.add_argument("--no-fp64-check", action="store_true",
                    help="skip the FP64 oracle checks behind the fp64_error objects")
    ap.add_argument("--batched-cycles", type=int, default=40)
    ap.add_argument("--adjoint-probe", action="store_true",
                    help="backward passes only (16 x 256x256 and one 4096x4096 cycle), for "
                         "kernel traces of the reverse-step kernels")
    ap.add_argument("--probe", action="store_true",
                    help="counter probe: 3 cycles of fused step launches on the workload, then "
                         "a plain 64 MiB device copy (calibrates FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path has no multi-GPU decomposition)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2006_10406_amd as eed4
    from synth import WORKLOADS, make_problem

    if args.adjoint_probe:
        adjoint_probe(eed4, torch)
        return

    wl = WORKLOADS["large4096"]
    log(f"generating {wl.name} {wl.H}x{wl.W}")
    pr = make_problem(wl.H, wl.W, wl.n_ellipses, wl.ramp, wl.noise_std, wl.density, wl.seed_base)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    u_init = torch.from_numpy(pr["u_init"]).to(dev)
    mask = torch.from_numpy(pr["mask"]).to(dev)
    known = torch.from_numpy(pr["known"]).to(dev)
    H, W, n = wl.H, wl.W, wl.n
    pw = eed4.params(wl.lam, wl.sigma, wl.tau, n, max(args.warmup, 1))
    pt = eed4.params(wl.lam, wl.sigma, wl.tau, n, args.steps)
    wsv = aligned_workspace(torch, max(eed4.eed4_workspace_size(eed4.EED4_OP_INPAINT, 1, H, W, q)
                                       for q in (pw, pt)), dev)

    if args.probe:
        probe(eed4, torch, u_init, mask, wl)
        return

    # ---- whole-path timing: warmup cycles, then exactly K timed cycles ----
    # Everything the timed call needs is set up before the warmup, so between the
    # warmup's end and the timed call there is only the barrier: the GPU clock drops
    # within a fraction of a millisecond of idling and takes many milliseconds to
    # come back, so host work there would slow the first timed cycles.
    u = u_init.clone()
    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    log(f"warmup {args.warmup} cycles, then {args.steps} timed cycles of {n} steps")
    eed4.eed4_inpaint(u, mask, known, pw, ws=wsv, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    st, _ = eed4.eed4_inpaint(u, mask, known, pt, ws=wsv, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    sec = ms * 1e-3
    updates = H * W * n * args.steps
    value = updates / sec / 1e6
    log(f"{st.cycles} cycles, {ms:.2f} ms (wall {wall * 1e3:.2f} ms), {value:.0f} Mpix-upd/s")

    # ---- kernel timing: back-to-back fused step launches on the same stream ----
    # the shape the library picked for this problem (tuned by the warmup call)
    shape = eed4.eed4_step_shape(1, H, W, pt)
    shape_name = eed4.SHAPE_NAMES[shape]
    ps = eed4.params(wl.lam, wl.sigma, wl.tau, n, 1, flags=eed4.EED4_FORCE_SHAPE(shape))
    windows = step_kernel_windows(eed4, torch, u, mask, ps, n, args.kernel_reps, stream)
    kms = sorted(windows)[2]
    log("fused step windows: " + ", ".join(f"{w * 1e3:.1f}" for w in windows) + " us/launch")
    per_launch_bytes = BYTES_PER_UPDATE * H * W
    achieved = per_launch_bytes / (kms * 1e-3) / 1e9
    R = eed4.eed4_radius(wl.sigma)
    per_launch_flops = flops_per_update(R) * H * W
    tflops = per_launch_flops / (kms * 1e-3) / 1e12
    kname = kernel_name(shape_name, R)
    traffic = measured_traffic(kname)
    log(f"fused step kernel {kname}: {kms * 1e3:.1f} us/launch, {achieved:.0f} GB/s, "
        f"{tflops:.1f} TFLOP/s")
    # the first cycle of the timed image from its initial state, for the FP64 check
    u1 = u_init.clone()
    eed4.eed4_fsi_cycle(u1, mask, known, ps, torch.zeros((1, 2), dtype=torch.float64,
                                                         device=dev))
    first_gpu = u1.cpu().numpy()
    del u1

    out = {
        "metric": "Mpixel-updates/s of fused 4th-order EED FSI step + adjoint/forward time ratio",
        "value": round(value, 1),
        "unit": "Mpixel-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "large4096", "H": H, "W": W, "batch": 1, "sigma": wl.sigma,
                   "lambda": wl.lam, "tau": wl.tau, "cycle_len": n, "mask_density": wl.density,
                   "step": "one FSI cycle (15 fused inner steps + FP64 residual)",
                   "kernel_shape": shape_name, "parallelism": "single GPU"},
        # the nearer roofline is HBM (about 0.5 of 8 TB/s against about 0.25 of the FP32
        # vector peak); the ALU figure is reported beside it
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": f"{kname} (fused FSI step)",
                     "kernel_us": round(kms * 1e3, 2),
                     # the timed region per fused-step launch; beside the step kernels it
                     # holds one residual reduction per cycle, the initial Dirichlet fill and
                     # the gaps between launches
                     "timed_region_us_per_launch": round(ms * 1e3 / (args.steps * n), 2),
                     "algorithmic_bytes_per_launch": per_launch_bytes,
                     "alu": {"achieved": round(tflops, 2), "peak": round(ALU_PEAK_TFLOPS, 1),
                             "unit": "TFLOP/s", "frac": round(tflops / ALU_PEAK_TFLOPS, 4),
                             "algorithmic_flops_per_launch": per_launch_flops},
                     "kernel_source_sha": kernel_source_sha(),
                     "copy_context": copy_bandwidth(torch)},
    }
    if not args.no_out_of_cache:
        log("fused step on 8192x8192 (working set beyond the Infinity Cache)")
        out["roofline"]["out_of_cache"] = out_of_cache_point(eed4, torch, wl, shape,
                                                             max(args.kernel_reps // 4, 2),
                                                             stream)
    checks = []          # (path in out, deferred FP64 check)
    if not args.no_variants:
        log("tensor variants (Table 7 diffusivities x mu3 choices)")
        out["variants"] = variants_timing(eed4, torch, u, mask, wl, stream)
        checks.append((("variants",), variant_first_cycle(eed4, torch, pr, mask, known, wl)))
    if not args.no_workloads:
        log("colour and scratch workloads (512x512)")
        out["workloads"], wchecks = workload_throughput(eed4, torch)
        checks += [(("workloads", name), fn) for name, fn in wchecks]
    if not args.no_adjoint:
        log("adjoint / forward timing (16 x 256x256)")
        out["adjoint_forward_ratio"], fn = adjoint_ratio(eed4, torch, args)
        checks.append((("adjoint_forward_ratio",), fn))
    if not args.no_batched:
        log("batched vs per-image (64 uneven images)")
        out["batched"], fn = batched_vs_single(eed4, torch, args.batched_cycles)
        checks.append((("batched",), fn))
    # ---- host-only work from here on: the FP64 oracle ----
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host (one cycle; single thread; other workloads)")
        out["cpu_baseline"], first_ref = cpu_baseline(pr, wl)
        e = fp64_error(first_gpu, first_ref)
        e["sample"] = (f"first FSI cycle of the {H}x{W} workload image from its initial state, "
                       f"kernel shape {shape_name}")
        out["fp64_error"] = e
    if not args.no_fp64_check:
        log(f"FP64 oracle checks of {len(checks)} results")
        for path, fn in checks:
            node = out
            for key in path:
                node = node[key]
            node["fp64_error"] = fn()
    print(json.dumps(out), flush=True)


def step_kernel_windows(eed4, torch, u, mask, ps, n, reps, stream):
    """Five windows of `reps` cycles of back-to-back eed4_fsi_step launches in the
    buffer rotation of a cycle; returns ms per launch of each window (the first
    launches after a pause run at a lower clock, so callers take the median)."""
    a, b, c = u.clone(), u.clone(), u.clone()

    def roles(k):  # same rotation as a cycle: S=a, X=b, Y=c
        if k == 0:
            return a, a, b
        if k == 1:
            return b, a, c
        return (b, c, c) if k % 2 else (c, b, b)

    e2 = torch.cuda.Event(enable_timing=True)
    e3 = torch.cuda.Event(enable_timing=True)
    eed4.eed4_fsi_step(a, a, b, mask, ps, 0, stream=stream)  # warm
    torch.cuda.synchronize()
    windows = []
    for _ in range(5):
        launches = 0
        e2.record(stream)
        for _ in range(reps):
            for k in range(n):
                cur, prev, nxt = roles(k)
                eed4.eed4_fsi_step(cur, prev, nxt, mask, ps, k, stream=stream)
                launches += 1
        e3.record(stream)
        torch.cuda.synchronize()
        windows.append(e2.elapsed_time(e3) / launches)
    return windows


def out_of_cache_point(eed4, torch, wl, shape, reps, stream):
    """The fused step of the timed kernel shape on an 8192 x 8192 image drawn on the device
    with the same recipe: three state planes and the mask are 832 MiB, beyond the 256 MB
    Infinity Cache, so every launch streams from HBM."""
    from synth import make_problem_device
    H = W = 8192
    pr = make_problem_device(H, W, wl.n_ellipses, wl.ramp, wl.noise_std, wl.density, 8192)
    u, mask = pr["u_init"], pr["mask"]
    del pr["known"]
    ps = eed4.params(wl.lam, wl.sigma, wl.tau, wl.n, 1, flags=eed4.EED4_FORCE_SHAPE(shape))
    windows = step_kernel_windows(eed4, torch, u, mask, ps, wl.n, reps, stream)
    kms = sorted(windows)[2]
    nbytes = BYTES_PER_UPDATE * H * W
    gbs = nbytes / (kms * 1e-3) / 1e9
    log(f"8192x8192 fused step: {kms * 1e3:.1f} us/launch, {gbs:.0f} GB/s")
    del u, mask, pr
    torch.cuda.empty_cache()
    return {"H": H, "W": W, "kernel_us": round(kms * 1e3, 2), "achieved": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_launch": nbytes,
            "working_set_MiB": (3 * 4 + 1) * H * W // (1 << 20),
            "windows_us": [round(w * 1e3, 1) for w in windows]}


if __name__ == "__main__":
    main()
