"""Seeded synthetic inputs for fourth-order EED inpainting.

This module only draws images and masks; it holds none of the diffusion
arithmetic, so both the HIP path and the FP64 oracle can take their inputs
from it without sharing any part of the method.

Images are piecewise smooth: filled ellipses over a uniform background,
optionally blended with a linear ramp, plus Gaussian noise, clipped to [0, 1].
Masks keep an exact number of uniformly drawn pixels (the device-side
generator for images too large for the host draws a Bernoulli mask).  These
stand in for the
paper's natural and medical test images (Sec. 4), which are not available.
"""
from .generator import (
    Workload,
    make_image,
    make_mask,
    make_problem,
    make_problem_device,
    make_batch,
    make_uneven_batch,
    make_rgb_problem,
    make_scratch_mask,
    make_scratch_problem,
    make_workload_problem,
    SCRATCH_WIDTH,
    WORKLOADS,
)

__all__ = [
    "Workload",
    "make_image",
    "make_mask",
    "make_problem",
    "make_problem_device",
    "make_batch",
    "make_uneven_batch",
    "make_rgb_problem",
    "make_scratch_mask",
    "make_scratch_problem",
    "make_workload_problem",
    "SCRATCH_WIDTH",
    "WORKLOADS",
]
