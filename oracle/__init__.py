"""FP64 CPU oracle for fourth-order EED inpainting with FSI.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The HIP product path never imports it,
and it shares no code with that path.

``eed4_oracle.c`` holds the forward method (mirror-extended finite
differences, Sec. 3.3; diffusion tensor, Sec. 3.1; FSI, Sec. 3.3) and a
hand-derived adjoint; ``matrix_oracle.py`` is a second, independent NumPy
formulation with explicit matrices for tiny grids.  Parity status of each
function is recorded in its docstring; all of them are pinned by the
``-m "not gpu"`` tests.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None
_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def _lib():
    global _LIB
    if _LIB is None:
        # EED4_ORACLE_LIB names another build of the same source (the sanitizer build)
        path = os.environ.get("EED4_ORACLE_LIB")
        if not path:
            src_m = os.path.getmtime(_build.SRC)
            if not os.path.exists(_build.LIB) or os.path.getmtime(_build.LIB) < src_m:
                _build.build()
            path = _build.LIB
        L = ctypes.CDLL(path)
        L.oracle_radius.restype = ctypes.c_int
        L.oracle_radius.argtypes = [ctypes.c_double]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_gauss.argtypes = [ctypes.c_double, ctypes.c_int, _dp]
        L.oracle_charbonnier.restype = ctypes.c_double
        L.oracle_charbonnier.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_diffusivity.restype = ctypes.c_double
        L.oracle_diffusivity.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.oracle_alpha.restype = ctypes.c_double
        L.oracle_alpha.argtypes = [ctypes.c_int]
        ci = ctypes.c_int
        L.oracle_tensor.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ci, ci, _dp]
        L.oracle_e_grad.argtypes = [ctypes.c_double, ctypes.c_double, _dp, _dp,
                                    ctypes.c_double, ci, ci, _dp, _dp, _dp]
        L.oracle_apply_P.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_double, ci, ci, _dp]
        L.oracle_hessian.argtypes = [_dp, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]
        L.oracle_gradient.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp]
        L.oracle_step.argtypes = [_dp, _dp, _u8p, _dp, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_double, ci, ci, ctypes.c_double,
                                  ctypes.c_int, _dp]
        L.oracle_inpaint.restype = ctypes.c_int
        L.oracle_inpaint.argtypes = [_dp, _u8p, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_double, ci, ci, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                     _dp, _dp]
        L.oracle_jtv.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, ci, ci, _dp, _dp]
        L.oracle_backward.argtypes = [_dp, _u8p, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_double, ctypes.c_double, ci, ci, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp]
        _LIB = L
    return _LIB


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _m(a):
    a = np.ascontiguousarray(a != 0, dtype=np.uint8)
    return a, a.ctypes.data_as(_u8p)


def num_threads() -> int:
    """OpenMP threads the oracle uses."""
    return _lib().oracle_num_threads()


def set_num_threads(n: int) -> None:
    """OpenMP threads for the following oracle calls (for timing on n host cores)."""
    _lib().oracle_set_num_threads(int(n))


def radius(sigma: float) -> int:
    """Gaussian truncation radius ceil(3 sigma)."""
    return _lib().oracle_radius(float(sigma))


def gauss(sigma: float) -> np.ndarray:
    """Normalised sampled Gaussian, 2R+1 taps (Sec. 2.2 presmoothing)."""
    R = radius(sigma)
    w = np.zeros(2 * R + 1)
    _lib().oracle_gauss(float(sigma), R, w.ctypes.data_as(_dp))
    return w


def charbonnier(s2: float, lam: float) -> float:
    """g(s^2) = 1/sqrt(1 + s^2/lambda^2), eq. (CharDiff)."""
    return _lib().oracle_charbonnier(float(s2), float(lam))


#: Diffusivities of Table 7 by index (``diff`` argument); Geman-Reynolds is
#: scaled to g(0) = 1.
DIFFUSIVITIES = ("charbonnier", "perona_malik", "perona_malik_exp", "geman_reynolds")
#: Choices of mu_3 from mu_1 = g and mu_2 = 1 (Sec. 3.1, Table 1) by index
#: (``mu3`` argument): geometric mean (FOEED), arithmetic mean, maximum.
MU3_RULES = ("geometric", "arithmetic", "max")


def diffusivity(s2: float, lam: float, diff: int = 0) -> float:
    """g(s^2) of diffusivity ``diff`` (index into DIFFUSIVITIES), Table 7."""
    return _lib().oracle_diffusivity(float(s2), float(lam), int(diff))


def alpha(k: int) -> float:
    """FSI extrapolation weight alpha_k = (4k+2)/(2k+3) (Sec. 3.3)."""
    return _lib().oracle_alpha(int(k))


def tensor(gx: float, gy: float, lam: float, diff: int = 0, mu3: int = 0) -> np.ndarray:
    """d_ijkl as a 4x4 array indexed [(i,j), (k,l)] in the order xx, xy, yx, yy
    (eqs. faod_diffTensor, foad_diffTensor_entries)."""
    d = np.zeros(16)
    _lib().oracle_tensor(float(gx), float(gy), float(lam), int(diff), int(mu3),
                         d.ctypes.data_as(_dp))
    return d.reshape(4, 4)


def e_grad(gx, gy, A, Hm, lam, diff=0, mu3=0):
    """e = A : D(G) : H, de/dG and de/dlambda for 2x2 A, H (adjoint helper)."""
    A, pa = _d(np.asarray(A).reshape(4))
    Hm, ph = _d(np.asarray(Hm).reshape(4))
    e = np.zeros(1); q = np.zeros(2); dl = np.zeros(1)
    _lib().oracle_e_grad(float(gx), float(gy), pa, ph, float(lam), int(diff), int(mu3),
                         e.ctypes.data_as(_dp), q.ctypes.data_as(_dp), dl.ctypes.data_as(_dp))
    return float(e[0]), q, float(dl[0])


def apply_P(ut, x, lam, sigma, diff=0, mu3=0):
    """P(ut) x: tensor from the presmoothed gradient of ut, applied to x."""
    ut, pu = _d(ut)
    x, px = _d(x)
    H, W = ut.shape
    out = np.zeros((H, W))
    _lib().oracle_apply_P(pu, px, H, W, float(lam), float(sigma), int(diff), int(mu3),
                          out.ctypes.data_as(_dp))
    return out


def hessian(u):
    """(h_xx, h_xy, h_yy) with mirror boundary (Sec. 3.3 stencils, sign-corrected u_xy)."""
    u, pu = _d(u)
    H, W = u.shape
    a, b, c = np.zeros((H, W)), np.zeros((H, W)), np.zeros((H, W))
    _lib().oracle_hessian(pu, H, W, a.ctypes.data_as(_dp), b.ctypes.data_as(_dp),
                          c.ctypes.data_as(_dp))
    return a, b, c


def gradient(u, sigma):
    """Central-difference gradient of the presmoothed image."""
    u, pu = _d(u)
    H, W = u.shape
    gx, gy = np.zeros((H, W)), np.zeros((H, W))
    _lib().oracle_gradient(pu, H, W, float(sigma), gx.ctypes.data_as(_dp), gy.ctypes.data_as(_dp))
    return gx, gy


def step(u, uprev, mask, f, lam, sigma, tau, k, diff=0, mu3=0):
    """One FSI inner step with Dirichlet hold (Sec. 3.3, eq. genModel)."""
    u, pu = _d(u)
    uprev, pp = _d(uprev)
    H, W = u.shape
    if mask is None:
        mask = np.zeros((H, W), np.uint8)
    mask, pm = _m(mask)
    f, pf = _d(np.zeros((H, W)) if f is None else f)
    out = np.zeros((H, W))
    _lib().oracle_step(pu, pp, pm, pf, H, W, float(lam), float(sigma), int(diff), int(mu3),
                       float(tau), int(k), out.ctypes.data_as(_dp))
    return out


def inpaint(u_init, mask, known, lam, sigma, tau, n, M, tol=0.0, abs_tol=False,
            checkpoints=False, diff=0, mu3=0):
    """FOEED inpainting of one image [H,W] or an equal-size batch [B,H,W].

    Returns (u, cycles, hist[, ckpt]) with hist[m, b] = (||u^{m,n}-u^{m,0}||,
    ||u^{m,n}||) and ckpt[m] = u^{m,0}."""
    u = np.array(u_init, dtype=np.float64, copy=True)
    single = u.ndim == 2
    if single:
        u = u[None]
    B, H, W = u.shape
    mask, pm = _m(np.asarray(mask).reshape(B, H, W))
    f, pf = _d(np.asarray(known).reshape(B, H, W))
    hist = np.zeros((M, B, 2))
    ck = np.zeros((M, B, H, W)) if checkpoints else None
    cyc = _lib().oracle_inpaint(u.ctypes.data_as(_dp), pm, pf, B, H, W, float(lam), float(sigma),
                                int(diff), int(mu3), float(tau), int(n), int(M), float(tol),
                                int(bool(abs_tol)),
                                ck.ctypes.data_as(_dp) if ck is not None else None,
                                hist.ctypes.data_as(_dp))
    hist = hist[:cyc]
    if single:
        u = u[0]
        hist = hist[:, 0]
        if ck is not None:
            ck = ck[:, 0]
    if ck is not None:
        return u, cyc, hist, ck[:cyc]
    return u, cyc, hist


def jtv(u, w, lam, sigma, diff=0, mu3=0):
    """(J_F(u)^T w, <dF/dlambda, w>) for F(u) = P(u) u."""
    u, pu = _d(u)
    w, pw = _d(w)
    H, W = u.shape
    out = np.zeros((H, W)); dl = np.zeros(1)
    _lib().oracle_jtv(pu, pw, H, W, float(lam), float(sigma), int(diff), int(mu3),
                      out.ctypes.data_as(_dp), dl.ctypes.data_as(_dp))
    return out, float(dl[0])


def backward(ckpt, mask, known, lam, sigma, tau, n, grad_u, diff=0, mu3=0):
    """Adjoint of ``inpaint`` run for exactly len(ckpt) cycles.

    ckpt: [M,H,W] or [M,B,H,W] cycle-start states; grad_u: dL/du^{M,0}.
    Returns (grad_known, grad_init, grad_lambda[B or scalar])."""
    ck = np.asarray(ckpt, dtype=np.float64)
    single = ck.ndim == 3
    if single:
        ck = ck[:, None]
    M, B, H, W = ck.shape
    ck, pc = _d(ck)
    mask, pm = _m(np.asarray(mask).reshape(B, H, W))
    f, pf = _d(np.asarray(known).reshape(B, H, W))
    gu, pg = _d(np.asarray(grad_u).reshape(B, H, W))
    gf = np.zeros((B, H, W)); gi = np.zeros((B, H, W)); gl = np.zeros(B)
    _lib().oracle_backward(pc, pm, pf, B, H, W, float(lam), float(sigma), int(diff), int(mu3),
                           float(tau), int(n),
                           int(M), pg, gf.ctypes.data_as(_dp), gi.ctypes.data_as(_dp),
                           gl.ctypes.data_as(_dp))
    if single:
        return gf[0], gi[0], float(gl[0])
    return gf, gi, gl
