"""torch.autograd wrapper of eed4_inpaint / eed4_backward and a tonal
optimisation driver (gradient descent on the stored known values, as used
for PDE-based image compression, Sec. 1).

The forward pass runs a fixed number of FSI cycles through eed4_inpaint and
keeps the cycle-start states as checkpoints; the backward pass calls
eed4_backward, which recomputes each cycle from its checkpoint and reverses
it step by step on the GPU.  torch only holds memory and chains the
gradient of the initial guess (when it is built from the known values).
"""
from __future__ import annotations

from typing import List, Optional

import torch

from . import eed4_backward, eed4_inpaint, params


class EED4Inpaint(torch.autograd.Function):
    """u = inpaint(known, lam, u_init; mask) over M fixed FSI cycles.

    known, u_init: float32 [B,H,W] on the GPU; mask: uint8 [B,H,W];
    lam: 0-dim float tensor (one contrast for the batch); flags: EED4_* flags
    (e.g. a tensor variant, EED4_DIFFUSIVITY(d) | EED4_MU3(r)).
    Gradients: d/dknown (on the mask), d/dlam (summed over the batch),
    d/du_init (off the mask)."""

    @staticmethod
    def forward(ctx, known, lam, u_init, mask, sigma: float, tau: float, n: int, M: int,
                flags: int = 0):
        p = params(float(lam), sigma, tau, n, M, flags=flags)
        u = u_init.detach().clone().contiguous()
        known_c = known.detach().contiguous()
        ck = torch.empty((M,) + tuple(u.shape), dtype=torch.float32, device=u.device)
        eed4_inpaint(u, mask, known_c, p, ckpt=ck)
        ctx.save_for_backward(ck, mask, known_c)
        ctx.p = p
        ctx.M = M
        ctx.lam_shape = lam.shape
        return u

    @staticmethod
    def backward(ctx, grad_u):
        ck, mask, known = ctx.saved_tensors
        g = grad_u.contiguous()
        gk = torch.empty_like(g)
        gi = torch.empty_like(g)
        B = g.shape[0] if g.dim() == 3 else 1
        gl = torch.empty(B, dtype=torch.float32, device=g.device)
        eed4_backward(ck, mask, known, ctx.p, ctx.M, g, gk, gi, gl)
        return gk, gl.sum().reshape(ctx.lam_shape), gi, None, None, None, None, None, None


def mean_fill(known: torch.Tensor, mask: torch.Tensor) -> torch.Tensor:
    """Initial guess: known values on the mask, their mean elsewhere (per image)."""
    m = (mask != 0).to(known.dtype)
    cnt = m.sum(dim=(-2, -1), keepdim=True).clamp_min(1.0)
    mean = (known * m).sum(dim=(-2, -1), keepdim=True) / cnt
    return m * known + (1.0 - m) * mean


def inpaint(known, lam, mask, sigma, tau, n, M, u_init: Optional[torch.Tensor] = None,
            flags: int = 0):
    """Differentiable inpainting; u_init defaults to the mean fill of known."""
    if u_init is None:
        u_init = mean_fill(known, mask)
    if not torch.is_tensor(lam):
        lam = torch.tensor(float(lam), device=known.device)
    return EED4Inpaint.apply(known, lam, u_init, mask, sigma, tau, n, M, flags)


def tonal_optimize(image: torch.Tensor, mask: torch.Tensor, lam: float, sigma: float,
                   tau: float, n: int, M: int, steps: int = 50, lr: float = 5e-3,
                   optimize_lambda: bool = False, flags: int = 0) -> dict:
    """Adam on the known values (and optionally lambda) to minimise the MSE of
    the reconstruction against the original image.  Returns the loss history
    and the optimised tensors."""
    m = (mask != 0).to(image.dtype)
    known = torch.nn.Parameter((image * m).clone())
    lam_t = torch.nn.Parameter(torch.tensor(float(lam), device=image.device),
                               requires_grad=optimize_lambda)
    opt = torch.optim.Adam([known] + ([lam_t] if optimize_lambda else []), lr=lr)
    hist: List[float] = []
    for _ in range(steps):
        opt.zero_grad(set_to_none=True)
        u = inpaint(known, lam_t, mask, sigma, tau, n, M, flags=flags)
        loss = torch.mean((u - image) ** 2)
        loss.backward()
        known.grad.mul_(m)          # only stored pixels are free
        opt.step()
        hist.append(float(loss.detach()))
    with torch.no_grad():
        u = inpaint(known, lam_t, mask, sigma, tau, n, M, flags=flags)
        final = float(torch.mean((u - image) ** 2))
    return {"loss": hist, "final_loss": final, "known": known.detach(), "lam": float(lam_t)}
