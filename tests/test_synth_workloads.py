"""Host checks of the colour and scratch workload generators: determinism by
seed, the mask recipes (coverage, shared colour mask) and the initial guess."""
import numpy as np

from synth import (SCRATCH_WIDTH, WORKLOADS, make_problem_device, make_rgb_problem,
                   make_scratch_mask, make_workload_problem)


def test_rgb_problem_channels_share_one_mask():
    p = make_rgb_problem(96, 120, 8, True, 0.01, 0.05, 11)
    assert p["image"].shape == (3, 96, 120) and p["image"].dtype == np.float32
    m = p["mask"]
    assert m.dtype == np.uint8 and np.array_equal(m[0], m[1]) and np.array_equal(m[0], m[2])
    assert int(m[0].sum()) == round(0.05 * 96 * 120)
    for c in range(3):
        kn = m[c] != 0
        assert np.array_equal(p["known"][c][kn], p["image"][c][kn])
        assert np.all(p["known"][c][~kn] == 0)
        fill = p["image"][c][kn].astype(np.float64).mean()
        assert np.allclose(p["u_init"][c][~kn], fill, rtol=1e-6)
    # the channels are different images with coinciding edges, not copies
    assert not np.array_equal(p["image"][0], p["image"][1])
    again = make_rgb_problem(96, 120, 8, True, 0.01, 0.05, 11)
    assert all(np.array_equal(p[k], again[k]) for k in ("image", "mask", "u_init"))


def test_scratch_mask_coverage_and_structure():
    rng = np.random.default_rng(3)
    for cov, width in ((0.06, 2), (0.18, 6)):
        m = make_scratch_mask(300, 400, cov, width, rng)
        frac = 1.0 - m.mean()
        assert cov <= frac <= cov + 0.05
        # scratches are thin: most unknown pixels have a known pixel within the width
        unk = m == 0
        near = np.zeros_like(unk)
        r = width
        padded = np.pad(m != 0, r, constant_values=True)
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                near |= padded[r + dy:r + dy + 300, r + dx:r + dx + 400]
        assert near[unk].mean() > 0.9


def test_workload_problems():
    for name in ("rgb512", "scratch512_thin", "scratch512_thick"):
        wl = WORKLOADS[name]
        p = make_workload_problem(wl)
        if name.startswith("rgb"):
            assert p["image"].shape == (3, wl.H, wl.W)
            assert abs(p["mask"].mean() - wl.density) < 1e-4
        else:
            assert p["image"].shape == (wl.H, wl.W)
            assert wl.density <= 1.0 - p["mask"].mean() <= wl.density + 0.03
            assert SCRATCH_WIDTH[name] in (2, 6)


def test_device_generator_recipe_on_the_cpu_device():
    # the torch-side generator of very large problems, run on the CPU device: seeded, values in
    # [0, 1], Bernoulli mask near its density, known values on the mask and their mean elsewhere
    import torch
    a = make_problem_device(257, 389, 12, True, 0.01, 0.04, 5, device="cpu", chunk_rows=50)
    b = make_problem_device(257, 389, 12, True, 0.01, 0.04, 5, device="cpu", chunk_rows=50)
    assert all(torch.equal(a[k], b[k]) for k in ("u_init", "mask", "known"))
    u, m, f = a["u_init"], a["mask"], a["known"]
    assert u.dtype == torch.float32 and m.dtype == torch.uint8 and u.shape == (257, 389)
    assert abs(float(m.float().mean()) - 0.04) < 0.01
    km = m != 0
    assert torch.equal(u[km], f[km]) and bool((f[~km] == 0).all())
    assert float(u.min()) >= 0.0 and float(u.max()) <= 1.0
    fill = float(f[km].double().mean())
    assert torch.allclose(u[~km].double(), torch.full_like(u[~km].double(), fill), rtol=1e-6)
    assert not torch.equal(make_problem_device(64, 64, 3, False, 0.01, 0.05, 6, device="cpu")["mask"],
                           make_problem_device(64, 64, 3, False, 0.01, 0.05, 7, device="cpu")["mask"])
