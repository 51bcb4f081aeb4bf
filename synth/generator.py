"""Seeded generator of piecewise-smooth test images and random masks.

Recipe (one image):
  1. uniform background grey ~ U[0, 1];
  2. ``n_ellipses`` filled ellipses painted in order: centre uniform over the
     image, semi-axes ~ U[0.05, 0.3] * min(H, W), angle ~ U[0, pi), grey ~ U[0, 1];
  3. optionally ``0.75 * img + 0.25 * ramp`` with a linear ramp of random
     direction rescaled to [0, 1];
  4. additive N(0, noise_std^2) noise, then clipping to [0, 1];
  5. a mask keeping exactly ``max(1, round(density * H * W))`` pixels drawn
     uniformly without replacement.
The unknown pixels of the initial guess hold the mean of the known values.
Everything is drawn from ``numpy.random.default_rng(seed)`` in FP64 and cast
to float32 / uint8 at the end.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    """A named synthetic workload: image shape(s), generator recipe and solver
    parameters (contrast lambda, presmoothing sigma, step tau, FSI cycle
    length n, cycle count M or relative stop tolerance)."""

    name: str
    H: int
    W: int
    n_ellipses: int
    ramp: bool
    noise_std: float
    density: float
    sigma: float
    lam: float
    tau: float
    n: int
    M: int
    tol: float = 0.0
    B: int = 1
    seed_base: int = 0


WORKLOADS = {
    # 64x64, 5 ellipses, 5% mask; the oracle finishes it in seconds.
    "small64": Workload("small64", 64, 64, 5, False, 0.01, 0.05,
                        sigma=1.0, lam=0.05, tau=0.05, n=10, M=20,
                        seed_base=1000),
    # 512x512, 30 ellipses + ramp, 4% mask, run to relative residual < 1e-4.
    "single512": Workload("single512", 512, 512, 30, True, 0.01, 0.04,
                          sigma=1.5, lam=0.03, tau=0.05, n=40, M=400,
                          tol=1e-4, seed_base=2000),
    # 4096x4096, 200 ellipses + ramp, 3% mask, 100 cycles of 15 steps.
    "large4096": Workload("large4096", 4096, 4096, 200, True, 0.005, 0.03,
                          sigma=2.0, lam=0.02, tau=0.05, n=15, M=100,
                          seed_base=3000),
    # 64 images of uneven size (sides U{128..1024}), 2..8% masks.
    "batch64": Workload("batch64", 0, 0, 30, True, 0.005, 0.05,
                        sigma=1.5, lam=0.03, tau=0.05, n=15, M=40, B=64,
                        seed_base=4000),
    # 16 images of 256x256, 4% mask; tonal optimisation through 30 cycles.
    "adjoint16": Workload("adjoint16", 256, 256, 30, True, 0.01, 0.04,
                          sigma=1.0, lam=0.05, tau=0.05, n=10, M=30, B=16,
                          seed_base=5000),
    # colour: 512x512 RGB (3 channels sharing the ellipse geometry), one 5% mask
    # for all channels, inpainted channel-wise as a batch of 3 planes
    "rgb512": Workload("rgb512", 512, 512, 30, True, 0.01, 0.05,
                       sigma=1.5, lam=0.03, tau=0.05, n=15, M=40, B=3,
                       seed_base=6000),
    # scratch removal: 512x512, scratches of width 2 covering 6% of the pixels
    # (density = fraction of unknown pixels)
    "scratch512_thin": Workload("scratch512_thin", 512, 512, 30, True, 0.01, 0.06,
                                sigma=1.5, lam=0.03, tau=0.05, n=15, M=40,
                                seed_base=7000),
    # ... and scratches of width 6 covering 18%
    "scratch512_thick": Workload("scratch512_thick", 512, 512, 30, True, 0.01, 0.18,
                                 sigma=1.5, lam=0.03, tau=0.05, n=15, M=40,
                                 seed_base=8000),
}

#: scratch width in pixels of the scratch workloads
SCRATCH_WIDTH = {"scratch512_thin": 2, "scratch512_thick": 6}


def make_image(H: int, W: int, n_ellipses: int, ramp: bool, noise_std: float,
               rng: np.random.Generator) -> np.ndarray:
    """Draw one piecewise-smooth image in FP64 with values in [0, 1]."""
    img = np.full((H, W), rng.uniform(0.0, 1.0), dtype=np.float64)
    m = float(min(H, W))
    for _ in range(n_ellipses):
        cy = rng.uniform(0.0, H)
        cx = rng.uniform(0.0, W)
        a = rng.uniform(0.05, 0.3) * m
        b = rng.uniform(0.05, 0.3) * m
        th = rng.uniform(0.0, np.pi)
        grey = rng.uniform(0.0, 1.0)
        rad = max(a, b)
        y0, y1 = max(0, int(np.floor(cy - rad))), min(H, int(np.ceil(cy + rad)) + 1)
        x0, x1 = max(0, int(np.floor(cx - rad))), min(W, int(np.ceil(cx + rad)) + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        yy = np.arange(y0, y1, dtype=np.float64)[:, None] - cy
        xx = np.arange(x0, x1, dtype=np.float64)[None, :] - cx
        c, s = np.cos(th), np.sin(th)
        p = (xx * c + yy * s) / a
        q = (-xx * s + yy * c) / b
        inside = p * p + q * q <= 1.0
        img[y0:y1, x0:x1][inside] = grey
    if ramp:
        phi = rng.uniform(0.0, 2.0 * np.pi)
        yy = np.arange(H, dtype=np.float64)[:, None]
        xx = np.arange(W, dtype=np.float64)[None, :]
        r = xx * np.cos(phi) / W + yy * np.sin(phi) / H
        lo, hi = r.min(), r.max()
        r = (r - lo) / (hi - lo) if hi > lo else np.zeros_like(r)
        img = 0.75 * img + 0.25 * r
    if noise_std > 0:
        img = img + rng.normal(0.0, noise_std, size=(H, W))
    return np.clip(img, 0.0, 1.0)


def make_mask(H: int, W: int, density: float, rng: np.random.Generator) -> np.ndarray:
    """Exact-count uniform random mask (uint8, 1 = known)."""
    count = max(1, int(round(density * H * W)))
    count = min(count, H * W)
    idx = rng.choice(H * W, size=count, replace=False)
    mask = np.zeros(H * W, dtype=np.uint8)
    mask[idx] = 1
    return mask.reshape(H, W)


def _initial_guess(img: np.ndarray, mask: np.ndarray) -> np.ndarray:
    known = img[mask != 0]
    fill = float(known.mean()) if known.size else 0.5
    u0 = np.where(mask != 0, img, fill)
    return u0


def make_problem(H: int, W: int, n_ellipses: int, ramp: bool, noise_std: float,
                 density: float, seed: int) -> dict:
    """One inpainting problem: ground truth ``image``, ``mask`` (u8), ``known``
    (image on the mask, 0 elsewhere) and ``u_init`` (known values on the mask,
    mean of the known values elsewhere), all float32 except the mask."""
    rng = np.random.default_rng(seed)
    img = make_image(H, W, n_ellipses, ramp, noise_std, rng)
    mask = make_mask(H, W, density, rng)
    known = np.where(mask != 0, img, 0.0)
    u0 = _initial_guess(img, mask)
    return {
        "image": img.astype(np.float32),
        "mask": mask,
        "known": known.astype(np.float32),
        "u_init": u0.astype(np.float32),
        "seed": seed,
    }


def make_batch(wl: Workload, B: Optional[int] = None,
               shape: Optional[Tuple[int, int]] = None) -> dict:
    """Equal-size batch for workload ``wl`` (arrays shaped [B, H, W]);
    image i uses seed ``wl.seed_base + i``."""
    B = wl.B if B is None else B
    H, W = (wl.H, wl.W) if shape is None else shape
    probs = [make_problem(H, W, wl.n_ellipses, wl.ramp, wl.noise_std,
                          wl.density, wl.seed_base + i) for i in range(B)]
    return {k: np.stack([p[k] for p in probs]) for k in ("image", "mask", "known", "u_init")}


def make_uneven_batch(wl: Workload, B: Optional[int] = None,
                      side_range: Tuple[int, int] = (128, 1024),
                      density_range: Tuple[float, float] = (0.02, 0.08)) -> List[dict]:
    """Uneven batch: image i has H, W ~ U{side_range} independently and mask
    density ~ U[density_range], drawn from ``default_rng(wl.seed_base)``; the
    image itself is drawn from seed ``wl.seed_base + 1 + i``."""
    B = wl.B if B is None else B
    rng = np.random.default_rng(wl.seed_base)
    out = []
    for i in range(B):
        H = int(rng.integers(side_range[0], side_range[1] + 1))
        W = int(rng.integers(side_range[0], side_range[1] + 1))
        dens = float(rng.uniform(*density_range))
        p = make_problem(H, W, wl.n_ellipses, wl.ramp, wl.noise_std, dens,
                         wl.seed_base + 1 + i)
        p["density"] = dens
        out.append(p)
    return out


def make_rgb_image(H: int, W: int, n_ellipses: int, ramp: bool, noise_std: float,
                   rng: np.random.Generator) -> np.ndarray:
    """Colour image [3, H, W] in FP64: the recipe of ``make_image`` with one
    colour (three greys) per ellipse and for the background, so that edges
    coincide across channels; the ramp has one direction and a random
    amplitude per channel; the noise is independent per channel."""
    img = np.empty((3, H, W), dtype=np.float64)
    img[:] = rng.uniform(0.0, 1.0, size=3)[:, None, None]
    m = float(min(H, W))
    for _ in range(n_ellipses):
        cy = rng.uniform(0.0, H)
        cx = rng.uniform(0.0, W)
        a = rng.uniform(0.05, 0.3) * m
        b = rng.uniform(0.05, 0.3) * m
        th = rng.uniform(0.0, np.pi)
        colour = rng.uniform(0.0, 1.0, size=3)
        rad = max(a, b)
        y0, y1 = max(0, int(np.floor(cy - rad))), min(H, int(np.ceil(cy + rad)) + 1)
        x0, x1 = max(0, int(np.floor(cx - rad))), min(W, int(np.ceil(cx + rad)) + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        yy = np.arange(y0, y1, dtype=np.float64)[:, None] - cy
        xx = np.arange(x0, x1, dtype=np.float64)[None, :] - cx
        c, s = np.cos(th), np.sin(th)
        p = (xx * c + yy * s) / a
        q = (-xx * s + yy * c) / b
        inside = p * p + q * q <= 1.0
        for ch in range(3):
            img[ch, y0:y1, x0:x1][inside] = colour[ch]
    if ramp:
        phi = rng.uniform(0.0, 2.0 * np.pi)
        amp = rng.uniform(0.15, 0.35, size=3)
        yy = np.arange(H, dtype=np.float64)[:, None]
        xx = np.arange(W, dtype=np.float64)[None, :]
        r = xx * np.cos(phi) / W + yy * np.sin(phi) / H
        lo, hi = r.min(), r.max()
        r = (r - lo) / (hi - lo) if hi > lo else np.zeros_like(r)
        for ch in range(3):
            img[ch] = (1.0 - amp[ch]) * img[ch] + amp[ch] * r
    if noise_std > 0:
        img = img + rng.normal(0.0, noise_std, size=img.shape)
    return np.clip(img, 0.0, 1.0)


def make_rgb_problem(H: int, W: int, n_ellipses: int, ramp: bool, noise_std: float,
                     density: float, seed: int) -> dict:
    """Channel-wise colour inpainting problem: arrays [3, H, W]; one random mask
    (exact count) shared by the three channels, replicated per channel."""
    rng = np.random.default_rng(seed)
    img = make_rgb_image(H, W, n_ellipses, ramp, noise_std, rng)
    mask = make_mask(H, W, density, rng)
    masks = np.repeat(mask[None], 3, 0)
    known = np.where(masks != 0, img, 0.0)
    u0 = np.stack([_initial_guess(img[c], mask) for c in range(3)])
    return {
        "image": img.astype(np.float32),
        "mask": masks,
        "known": known.astype(np.float32),
        "u_init": u0.astype(np.float32),
        "seed": seed,
    }


def make_scratch_mask(H: int, W: int, coverage: float, width: int,
                      rng: np.random.Generator) -> np.ndarray:
    """Scratch mask (uint8, 1 = known): straight scratches of the given width
    are drawn one at a time (start uniform over the image, angle U[0, pi),
    length U[0.2, 0.8] * min(H, W)) until they cover at least ``coverage`` of
    the pixels; the scratched pixels are the unknown ones."""
    unknown = np.zeros((H, W), dtype=bool)
    target = coverage * H * W
    yy = np.arange(H, dtype=np.float64)[:, None]
    xx = np.arange(W, dtype=np.float64)[None, :]
    half = 0.5 * width
    while unknown.sum() < target:
        y0 = rng.uniform(0.0, H)
        x0 = rng.uniform(0.0, W)
        th = rng.uniform(0.0, np.pi)
        length = rng.uniform(0.2, 0.8) * min(H, W)
        dy, dx = np.sin(th), np.cos(th)
        # distance of every pixel centre to the segment
        t = np.clip((yy - y0) * dy + (xx - x0) * dx, 0.0, length)
        d2 = (yy - (y0 + t * dy)) ** 2 + (xx - (x0 + t * dx)) ** 2
        unknown |= d2 <= half * half
    return (~unknown).astype(np.uint8)


def make_scratch_problem(H: int, W: int, n_ellipses: int, ramp: bool, noise_std: float,
                         coverage: float, width: int, seed: int) -> dict:
    """Scratch-removal problem: the image of ``make_problem`` with a scratch
    mask (``coverage`` of the pixels unknown, scratches ``width`` wide)."""
    rng = np.random.default_rng(seed)
    img = make_image(H, W, n_ellipses, ramp, noise_std, rng)
    mask = make_scratch_mask(H, W, coverage, width, rng)
    known = np.where(mask != 0, img, 0.0)
    u0 = _initial_guess(img, mask)
    return {
        "image": img.astype(np.float32),
        "mask": mask,
        "known": known.astype(np.float32),
        "u_init": u0.astype(np.float32),
        "seed": seed,
    }


def make_workload_problem(wl: Workload) -> dict:
    """The problem of a colour or scratch workload (rgb512, scratch512_*)."""
    if wl.name.startswith("rgb"):
        return make_rgb_problem(wl.H, wl.W, wl.n_ellipses, wl.ramp, wl.noise_std,
                                wl.density, wl.seed_base)
    if wl.name in SCRATCH_WIDTH:
        return make_scratch_problem(wl.H, wl.W, wl.n_ellipses, wl.ramp, wl.noise_std,
                                    wl.density, SCRATCH_WIDTH[wl.name], wl.seed_base)
    raise ValueError(f"{wl.name} is not a colour or scratch workload")


def make_problem_device(H: int, W: int, n_ellipses: int, ramp: bool, noise_std: float,
                        density: float, seed: int, device="cuda", chunk_rows: int = 2048) -> dict:
    """The recipe of ``make_problem`` drawn on a torch device, for images too
    large to draw on the host (up to 2^31 pixels).  Ellipse and ramp
    parameters come from ``numpy.random.default_rng(seed)`` as on the host;
    the per-pixel noise and the mask come from a ``torch.Generator`` on the
    device seeded with ``seed``, in blocks of ``chunk_rows`` rows.  The mask
    keeps each pixel independently with probability ``density`` (a Bernoulli
    mask rather than an exact count).  Returns float32 ``u_init`` and
    ``known`` and a uint8 ``mask`` on the device (no ground-truth copy)."""
    import torch

    rng = np.random.default_rng(seed)
    img = torch.full((H, W), float(rng.uniform(0.0, 1.0)), dtype=torch.float32, device=device)
    m = float(min(H, W))
    for _ in range(n_ellipses):
        cy, cx = rng.uniform(0.0, H), rng.uniform(0.0, W)
        a, b = rng.uniform(0.05, 0.3) * m, rng.uniform(0.05, 0.3) * m
        th, grey = rng.uniform(0.0, np.pi), rng.uniform(0.0, 1.0)
        rad = max(a, b)
        y0, y1 = max(0, int(np.floor(cy - rad))), min(H, int(np.ceil(cy + rad)) + 1)
        x0, x1 = max(0, int(np.floor(cx - rad))), min(W, int(np.ceil(cx + rad)) + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        c, s = float(np.cos(th)), float(np.sin(th))
        xx = torch.arange(x0, x1, dtype=torch.float32, device=device)[None, :] - cx
        for r0 in range(y0, y1, chunk_rows):
            r1 = min(y1, r0 + chunk_rows)
            yy = torch.arange(r0, r1, dtype=torch.float32, device=device)[:, None] - cy
            p = (xx * c + yy * s) / a
            q = (-xx * s + yy * c) / b
            img[r0:r1, x0:x1].masked_fill_(p * p + q * q <= 1.0, grey)
    phi = rng.uniform(0.0, 2.0 * np.pi) if ramp else 0.0
    cu, su = np.cos(phi) / W, np.sin(phi) / H
    corners = [x * cu + y * su for y in (0, H - 1) for x in (0, W - 1)]
    lo, hi = min(corners), max(corners)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    mask = torch.empty((H, W), dtype=torch.uint8, device=device)
    xs = torch.arange(W, dtype=torch.float32, device=device)[None, :] * cu
    for r0 in range(0, H, chunk_rows):
        r1 = min(H, r0 + chunk_rows)
        blk = img[r0:r1]
        if ramp and hi > lo:
            ys = torch.arange(r0, r1, dtype=torch.float32, device=device)[:, None] * su
            blk.mul_(0.75).add_(((xs + ys) - lo) * (0.25 / (hi - lo)))
        if noise_std > 0:
            blk.add_(torch.randn(blk.shape, generator=gen, device=device) * noise_std)
        blk.clamp_(0.0, 1.0)
        mask[r0:r1] = (torch.rand(blk.shape, generator=gen, device=device) < density).to(torch.uint8)
    km = mask != 0
    n_known = int(km.sum())
    fill = float((img * km).sum(dtype=torch.float64) / n_known) if n_known else 0.5
    known = torch.where(km, img, torch.zeros((), device=device))
    img.masked_fill_(~km, fill)            # img becomes u_init
    del km
    return {"u_init": img, "mask": mask, "known": known, "seed": seed}
