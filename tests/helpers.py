"""Shared helpers of the GPU tests (device transfer, error metrics, case labels).

The parity bar of the FP32 HIP path against the FP64 oracle, grey values in
[0, 1]:
  one FSI cycle from the same FP32 state   relative L2 <= 1e-5 and every
                                           element within 1e-5
  multi-cycle runs at equal cycle counts   RMSE <= 1e-4 and every element
                                           within 1e-4
  adjoint (dL/df, dL/du_init, dL/dlambda)  relative L2 <= 1e-4 and every
                                           element within 1e-4 * max |oracle|
A whole-image norm alone would let one wrong pixel through at large sizes (at
4096^2 a relative L2 of 1e-5 allows a single pixel off by 0.02), so every
comparison also bounds the largest elementwise error.
"""
import sys

import numpy as np

REL_L2_PER_CYCLE = 1e-5      # one FSI cycle started from the same state
MAX_ABS_PER_CYCLE = 1e-5     # ... and per element
RMSE_STEADY = 1e-4           # grey values in [0, 1], at equal cycle counts
MAX_ABS_STEADY = 1e-4        # ... and per element
ADJ_REL_L2 = 1e-4            # adjoint against the oracle adjoint
ADJ_MAX_REL = 1e-4           # per element, relative to the largest oracle gradient


def announce(msg: str):
    """Print and flush the case about to run on the GPU."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rmse(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.sqrt(np.mean((a - b) ** 2)))


def max_abs(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).max()) if a.size else 0.0


def assert_cycle_parity(got, ref, label=""):
    """One FSI cycle (or several, each started from the oracle's state): relative L2 and
    the largest elementwise error against FP64.  Returns (rel L2, max abs)."""
    e, m = rel_l2(got, ref), max_abs(got, ref)
    print(f"{label}: rel L2 vs FP64 {e:.3e}, max abs {m:.3e}", flush=True)
    assert e <= REL_L2_PER_CYCLE, f"{label}: rel L2 {e:.3e}"
    assert m <= MAX_ABS_PER_CYCLE, f"{label}: max abs {m:.3e}"
    return e, m


def assert_steady_parity(got, ref, label=""):
    """A run of several cycles against the oracle at the same cycle count: RMSE and the
    largest elementwise error.  Returns (RMSE, max abs)."""
    e, m = rmse(got, ref), max_abs(got, ref)
    print(f"{label}: RMSE vs FP64 {e:.3e}, max abs {m:.3e}", flush=True)
    assert e <= RMSE_STEADY, f"{label}: RMSE {e:.3e}"
    assert m <= MAX_ABS_STEADY, f"{label}: max abs {m:.3e}"
    return e, m


def assert_grad_parity(got, ref, label=""):
    """A gradient against the oracle adjoint: relative L2 and the largest elementwise error
    relative to the largest oracle value.  Returns (rel L2, max abs / max |ref|)."""
    e = rel_l2(got, ref)
    scale = float(np.abs(np.asarray(ref, np.float64)).max()) if np.size(ref) else 0.0
    m = max_abs(got, ref) / scale if scale > 0 else max_abs(got, ref)
    print(f"{label}: rel L2 {e:.3e}, max abs / max|oracle| {m:.3e}", flush=True)
    assert e <= ADJ_REL_L2, f"{label}: rel L2 {e:.3e}"
    assert m <= ADJ_MAX_REL, f"{label}: max abs rel {m:.3e}"
    return e, m


def to_dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()
