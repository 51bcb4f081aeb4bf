"""Shared helpers of the GPU tests (device transfer, error metrics, case labels)."""
import sys

import numpy as np

# Tolerances of the parity bar: FP32 HIP path vs FP64 oracle.
REL_L2_PER_CYCLE = 1e-5      # one FSI cycle started from the same state
RMSE_STEADY = 1e-4           # grey values in [0, 1], at equal cycle counts


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


def to_dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()
