"""Fourth-order edge-enhancing diffusion (FOEED) inpainting on MI355X.

Thin Python binding of the C ABI in ``include/eed4.h`` (libeed4.so, HIP for
gfx950).  The functions keep the C names and only marshal arguments: torch
tensors provide device memory and the current HIP stream; every step of the
method runs in the library's kernels.  There is no CPU fallback: importing
the package fails if the library has not been built.

Method: Jumakulyyev & Schultz, "Fourth-Order Anisotropic Diffusion for
Inpainting and Image Compression" (arXiv 2006.10406): the fourth-order
diffusion tensor of Sec. 3.1 driven by the Gaussian-presmoothed gradient,
discretised with the finite differences of Sec. 3.3 and solved to steady
state with FSI cycles (Sec. 3.3).
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib
from ._lib import (EED4_ABS_TOL, EED4_ALLOW_LARGE_TAU, EED4_FORCE_SHAPE, EED4_NO_GRAPH,
                   EED4_OP_BACKWARD, EED4_TILE_KERNEL, SHAPE_NAMES, TILE_SHAPES, STRIP_SHAPES,
                   EED4_OP_CYCLE, EED4_OP_INPAINT, eed4_image, eed4_params, eed4_stats,
                   EED4_CHARBONNIER, EED4_PERONA_MALIK, EED4_PERONA_MALIK_EXP, EED4_GEMAN_REYNOLDS,
                   EED4_MU3_GEOMETRIC, EED4_MU3_ARITHMETIC, EED4_MU3_MAX, EED4_DIFFUSIVITY,
                   EED4_MU3, DIFFUSIVITY_NAMES, MU3_NAMES)

_lib.lib()  # fail loudly at import if libeed4.so is missing

__all__ = [
    "EED4Error", "params", "eed4_radius", "eed4_workspace_size", "eed4_inpaint",
    "eed4_fsi_cycle", "eed4_fsi_cycle_static", "eed4_fsi_step", "eed4_backward", "eed4_batched_workspace_size", "eed4_inpaint_batched",
    "eed4_strerror", "EED4_ABS_TOL", "EED4_ALLOW_LARGE_TAU", "EED4_NO_GRAPH", "EED4_TILE_KERNEL",
    "EED4_OP_INPAINT", "EED4_OP_CYCLE", "EED4_OP_BACKWARD", "EED4_FORCE_SHAPE", "SHAPE_NAMES", "TILE_SHAPES", "STRIP_SHAPES",
    "eed4_autotune_batched", "eed4_step_shape", "library_path",
    "EED4_CHARBONNIER", "EED4_PERONA_MALIK", "EED4_PERONA_MALIK_EXP", "EED4_GEMAN_REYNOLDS",
    "EED4_MU3_GEOMETRIC", "EED4_MU3_ARITHMETIC", "EED4_MU3_MAX", "EED4_DIFFUSIVITY", "EED4_MU3",
    "DIFFUSIVITY_NAMES", "MU3_NAMES",
]


class EED4Error(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {eed4_strerror(code)} (code {code})")


def library_path() -> str:
    return _lib.LIB_PATH


def params(lam: float, sigma: float, tau: float, n: int, M: int, tol: float = 0.0,
           flags: int = 0) -> eed4_params:
    """eed4_params{lambda, sigma, tau, cycle_len, max_cycles, tol, flags}."""
    return eed4_params(float(lam), float(sigma), float(tau), int(n), int(M), float(tol),
                       int(flags))


def eed4_strerror(code: int) -> str:
    return _lib.lib().eed4_strerror(int(code)).decode()


def eed4_radius(sigma: float) -> int:
    return _lib.lib().eed4_radius(float(sigma))


def eed4_workspace_size(op: int, B: int, H: int, W: int, p: eed4_params) -> int:
    return _lib.lib().eed4_workspace_size(int(op), int(B), int(H), int(W), ctypes.byref(p))


# ---------------------------------------------------------------- marshalling helpers
def _check(code: int, where: str):
    if code != 0:
        raise EED4Error(code, where)


def _dev_tensor(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _bhw(t: torch.Tensor, name: str) -> Tuple[int, int, int]:
    if t.dim() == 2:
        return 1, t.shape[0], t.shape[1]
    if t.dim() == 3:
        return t.shape[0], t.shape[1], t.shape[2]
    raise ValueError(f"{name} must be [H,W] or [B,H,W]")


def _stream(t: torch.Tensor, stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream(t.device)
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _workspace(nbytes: int, device, ws: Optional[torch.Tensor]) -> Tuple[int, int, torch.Tensor]:
    """Device workspace (256-byte aligned) of at least nbytes; returns (ptr, size, holder)."""
    if ws is not None:
        _dev_tensor(ws, torch.uint8, "ws")
        return ws.data_ptr(), ws.numel(), ws
    buf = torch.empty(max(nbytes, 1) + 256, dtype=torch.uint8, device=device)
    ptr = buf.data_ptr()
    off = (-ptr) % 256
    return ptr + off, buf.numel() - off, buf


def _mask_known(u, mask, known, B, H, W):
    _dev_tensor(mask, torch.uint8, "mask")
    _dev_tensor(known, torch.float32, "known")
    for t, n in ((mask, "mask"), (known, "known")):
        if _bhw(t, n) != (B, H, W) or t.device != u.device:
            raise ValueError(f"{n} must match u in shape and device")


# ---------------------------------------------------------------- entry points
def eed4_inpaint(u: torch.Tensor, mask: torch.Tensor, known: torch.Tensor, p: eed4_params,
                 ckpt: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
                 stream=None, history: bool = False):
    """In-place inpainting of u ([H,W] or [B,H,W] float32).  Returns
    (eed4_stats, hist) with hist[m, b] = (residual, norm) when history=True."""
    _dev_tensor(u, torch.float32, "u")
    B, H, W = _bhw(u, "u")
    _mask_known(u, mask, known, B, H, W)
    if ckpt is not None:
        _dev_tensor(ckpt, torch.float32, "ckpt")
        if ckpt.numel() < p.max_cycles * B * H * W or ckpt.device != u.device:
            raise ValueError("ckpt must hold max_cycles * B * H * W floats on u's device")
    need = eed4_workspace_size(EED4_OP_INPAINT, B, H, W, p)
    if need == 0:
        _check(-1, "eed4_workspace_size")
    wp, wsz, _hold = _workspace(need, u.device, ws)
    st = eed4_stats()
    hist = np.zeros((p.max_cycles, B, 2)) if history else None
    rc = _lib.lib().eed4_inpaint(
        u.data_ptr(), mask.data_ptr(), known.data_ptr(), B, H, W, ctypes.byref(p),
        ckpt.data_ptr() if ckpt is not None else None, wp, wsz, _stream(u, stream),
        ctypes.byref(st), hist.ctypes.data if hist is not None else None)
    _check(rc, "eed4_inpaint")
    if hist is not None:
        hist = hist[: st.cycles]
    return st, hist


def eed4_fsi_cycle(u: torch.Tensor, mask: torch.Tensor, known: torch.Tensor, p: eed4_params,
                   d_sums: torch.Tensor, ws: Optional[torch.Tensor] = None, stream=None):
    """One FSI cycle in place on u; d_sums (float64 [B,2] on the device) gets
    sum (u^{m,n}-u^{m,0})^2 and sum (u^{m,n})^2 per image."""
    _dev_tensor(u, torch.float32, "u")
    B, H, W = _bhw(u, "u")
    _mask_known(u, mask, known, B, H, W)
    _dev_tensor(d_sums, torch.float64, "d_sums")
    if d_sums.numel() < 2 * B:
        raise ValueError("d_sums must hold 2*B doubles")
    need = eed4_workspace_size(EED4_OP_CYCLE, B, H, W, p)
    if need == 0:
        _check(-1, "eed4_workspace_size")
    wp, wsz, _hold = _workspace(need, u.device, ws)
    rc = _lib.lib().eed4_fsi_cycle(u.data_ptr(), mask.data_ptr(), known.data_ptr(), B, H, W,
                                   ctypes.byref(p), wp, wsz, _stream(u, stream), d_sums.data_ptr())
    _check(rc, "eed4_fsi_cycle")


def eed4_fsi_cycle_static(u: torch.Tensor, mask: torch.Tensor, known: torch.Tensor,
                          p: eed4_params, d_sums: torch.Tensor, stream=None):
    """eed4_fsi_cycle with the library's static device scratch instead of a workspace:
    allocates nothing (not even through torch).  Problems whose cycle workspace exceeds
    EED4_STATIC_SCRATCH_BYTES raise EED4Error(EED4_ETOOLARGE)."""
    _dev_tensor(u, torch.float32, "u")
    B, H, W = _bhw(u, "u")
    _mask_known(u, mask, known, B, H, W)
    _dev_tensor(d_sums, torch.float64, "d_sums")
    if d_sums.numel() < 2 * B:
        raise ValueError("d_sums must hold 2*B doubles")
    rc = _lib.lib().eed4_fsi_cycle_static(u.data_ptr(), mask.data_ptr(), known.data_ptr(), B, H,
                                          W, ctypes.byref(p), _stream(u, stream),
                                          d_sums.data_ptr())
    _check(rc, "eed4_fsi_cycle_static")


def eed4_fsi_step(ucur: torch.Tensor, uprev: torch.Tensor, uout: torch.Tensor,
                  mask: torch.Tensor, p: eed4_params, k: int, stream=None):
    """One FSI inner step: uout = alpha_k (I - tau P(ucur)) ucur + (1-alpha_k) uprev,
    held at ucur on the mask."""
    for t, n in ((ucur, "ucur"), (uprev, "uprev"), (uout, "uout")):
        _dev_tensor(t, torch.float32, n)
    B, H, W = _bhw(ucur, "ucur")
    for t, n in ((uprev, "uprev"), (uout, "uout"), (mask, "mask")):
        if _bhw(t, n) != (B, H, W) or t.device != ucur.device:
            raise ValueError(f"{n} must match ucur in shape and device")
    _dev_tensor(mask, torch.uint8, "mask")
    rc = _lib.lib().eed4_fsi_step(ucur.data_ptr(), uprev.data_ptr(), uout.data_ptr(),
                                  mask.data_ptr(), B, H, W, ctypes.byref(p), int(k),
                                  _stream(ucur, stream))
    _check(rc, "eed4_fsi_step")


def eed4_backward(ckpt: torch.Tensor, mask: torch.Tensor, known: torch.Tensor, p: eed4_params,
                  M: int, grad_u: torch.Tensor, grad_known: torch.Tensor,
                  grad_init: torch.Tensor, grad_lambda: torch.Tensor,
                  ws: Optional[torch.Tensor] = None, stream=None):
    """Adjoint of eed4_inpaint over M fixed cycles (see include/eed4.h)."""
    _dev_tensor(grad_u, torch.float32, "grad_u")
    B, H, W = _bhw(grad_u, "grad_u")
    _mask_known(grad_u, mask, known, B, H, W)
    _dev_tensor(ckpt, torch.float32, "ckpt")
    if ckpt.numel() < M * B * H * W:
        raise ValueError("ckpt must hold M * B * H * W floats")
    for t, n in ((grad_known, "grad_known"), (grad_init, "grad_init")):
        _dev_tensor(t, torch.float32, n)
        if _bhw(t, n) != (B, H, W):
            raise ValueError(f"{n} must be shaped like grad_u")
    _dev_tensor(grad_lambda, torch.float32, "grad_lambda")
    if grad_lambda.numel() < B:
        raise ValueError("grad_lambda must hold B floats")
    need = eed4_workspace_size(EED4_OP_BACKWARD, B, H, W, p)
    if need == 0:
        _check(-1, "eed4_workspace_size")
    wp, wsz, _hold = _workspace(need, grad_u.device, ws)
    rc = _lib.lib().eed4_backward(ckpt.data_ptr(), mask.data_ptr(), known.data_ptr(), B, H, W,
                                  ctypes.byref(p), int(M), grad_u.data_ptr(),
                                  grad_known.data_ptr(), grad_init.data_ptr(),
                                  grad_lambda.data_ptr(), wp, wsz, _stream(grad_u, stream))
    _check(rc, "eed4_backward")


def _image_array(images: Sequence[Tuple[torch.Tensor, torch.Tensor, torch.Tensor, float]]):
    arr = (eed4_image * len(images))()
    dev = None
    for i, (u, m, k, lam) in enumerate(images):
        _dev_tensor(u, torch.float32, "u")
        if u.dim() != 2:
            raise ValueError("batched images must be [H,W]")
        H, W = u.shape
        _mask_known(u, m, k, 1, H, W)
        dev = u.device if dev is None else dev
        if u.device != dev:
            raise ValueError("all images must be on one device")
        arr[i] = eed4_image(u.data_ptr(), m.data_ptr(), k.data_ptr(), H, W, float(lam))
    return arr, dev


def eed4_batched_workspace_size(images, p: eed4_params) -> int:
    arr, _ = _image_array(images)
    return _lib.lib().eed4_batched_workspace_size(arr, len(images), ctypes.byref(p))


def eed4_inpaint_batched(images, p: eed4_params, ws: Optional[torch.Tensor] = None,
                         stream=None) -> List[eed4_stats]:
    """Uneven batch: images is a list of (u, mask, known, lambda); u in place."""
    arr, dev = _image_array(images)
    need = _lib.lib().eed4_batched_workspace_size(arr, len(images), ctypes.byref(p))
    if need == 0:
        _check(-1, "eed4_batched_workspace_size")
    wp, wsz, _hold = _workspace(need, dev, ws)
    st = (eed4_stats * len(images))()
    rc = _lib.lib().eed4_inpaint_batched(arr, len(images), ctypes.byref(p), wp, wsz,
                                         _stream(images[0][0], stream), st)
    _check(rc, "eed4_inpaint_batched")
    return list(st)


def eed4_step_shape(B: int, H: int, W: int, p: eed4_params) -> int:
    """Fused-step shape id the library uses for B x H x W with p (forced, tuned
    in this process, or the size rule); no device work."""
    rc = _lib.lib().eed4_step_shape(B, H, W, ctypes.byref(p))
    if rc < 0:
        _check(rc, "eed4_step_shape")
    return rc


def eed4_autotune_batched(images, p: eed4_params, ws: Optional[torch.Tensor] = None,
                          stream=None) -> int:
    """Run the batched-kernel autotuner on this batch; returns the chosen shape id."""
    arr, dev = _image_array(images)
    need = _lib.lib().eed4_batched_workspace_size(arr, len(images), ctypes.byref(p))
    if need == 0:
        _check(-1, "eed4_batched_workspace_size")
    wp, wsz, _hold = _workspace(need, dev, ws)
    rc = _lib.lib().eed4_autotune_batched(arr, len(images), ctypes.byref(p), wp, wsz,
                                          _stream(images[0][0], stream))
    if rc < 0:
        _check(rc, "eed4_autotune_batched")
    return rc
