"""Explicit-matrix NumPy formulation of the FOEED operator for tiny grids.

TEST INFRASTRUCTURE ONLY.  A second oracle, independent of ``eed4_oracle.c``:
here every linear stage (presmoothing, gradient, Hessian) is a dense N x N
matrix built from half-sample mirror indices at the domain points, the
diffusion tensor is a 3x3 matrix in the Mandel basis (xx, yy, sqrt2*xy), and
the operator is assembled as P(u) = B^T M(u) B (Sec. 3.3 writes the explicit
step as (I - tau P_k) u^k with P_k symmetric positive semi-definite).  The C
oracle instead evaluates every stage on a mirror-extended image, so their
agreement checks that reading of the boundary condition.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft


def refl(i: int, N: int) -> int:
    p = 2 * N
    m = i % p
    return m if m < N else p - 1 - m


def gauss_weights(sigma: float) -> np.ndarray:
    if sigma <= 0:
        return np.ones(1)
    R = int(math.ceil(3.0 * sigma))
    j = np.arange(-R, R + 1, dtype=np.float64)
    w = np.exp(-j * j / (2.0 * sigma * sigma))
    return w / w.sum()


def _idx(y, x, W):
    return y * W + x


def blur_matrix(H: int, W: int, sigma: float) -> np.ndarray:
    w = gauss_weights(sigma)
    R = (len(w) - 1) // 2
    N = H * W
    Kx = np.zeros((N, N))
    Ky = np.zeros((N, N))
    for y in range(H):
        for x in range(W):
            for j in range(-R, R + 1):
                Kx[_idx(y, x, W), _idx(y, refl(x + j, W), W)] += w[j + R]
                Ky[_idx(y, x, W), _idx(refl(y + j, H), x, W)] += w[j + R]
    return Ky @ Kx


def stencil_matrix(H: int, W: int, taps) -> np.ndarray:
    """Matrix of sum_c c * u[refl(y+dy)][refl(x+dx)] over taps (dy, dx, c)."""
    N = H * W
    A = np.zeros((N, N))
    for y in range(H):
        for x in range(W):
            for dy, dx, c in taps:
                A[_idx(y, x, W), _idx(refl(y + dy, H), refl(x + dx, W), W)] += c
    return A


def derivative_matrices(H: int, W: int):
    Dx = stencil_matrix(H, W, [(0, 1, 0.5), (0, -1, -0.5)])
    Dy = stencil_matrix(H, W, [(1, 0, 0.5), (-1, 0, -0.5)])
    Bxx = stencil_matrix(H, W, [(0, -1, 1.0), (0, 0, -2.0), (0, 1, 1.0)])
    Byy = stencil_matrix(H, W, [(-1, 0, 1.0), (0, 0, -2.0), (1, 0, 1.0)])
    Bxy = stencil_matrix(H, W, [(1, 1, 0.25), (-1, -1, 0.25), (1, -1, -0.25), (-1, 1, -0.25)])
    return Dx, Dy, Bxx, Byy, Bxy


def diffusivity(s2: float, lam: float, diff: int = 0) -> float:
    """Table 7 diffusivities of t = s^2/lambda^2: Charbonnier (1+t)^-1/2,
    Perona-Malik (1+t)^-1, exponential Perona-Malik e^-t, Geman-Reynolds
    (1+t)^-2 (the table's 2 lambda^2/(s^2+lambda^2)^2 scaled to g(0) = 1)."""
    t = s2 / (lam * lam)
    if diff == 1:
        return 1.0 / (1.0 + t)
    if diff == 2:
        return math.exp(-t)
    if diff == 3:
        return 1.0 / (1.0 + t) ** 2
    return 1.0 / math.sqrt(1.0 + t)


def mu3_rule(mu1: float, mu2: float, rule: int = 0) -> float:
    """mu_3 as a mean of mu_1 and mu_2 (Sec. 3.1, Table 1): geometric
    (FOEED), arithmetic, or the maximum."""
    if rule == 1:
        return 0.5 * (mu1 + mu2)
    if rule == 2:
        return max(mu1, mu2)
    return math.sqrt(mu1 * mu2)


def mandel_tensor(gx: float, gy: float, lam: float, diff: int = 0, mu3: int = 0) -> np.ndarray:
    """3x3 Mandel form of sum_i mu_i E_i (x) E_i with mu = (g, 1, mu_3(g, 1))."""
    s2 = gx * gx + gy * gy
    g = diffusivity(s2, lam, diff)
    if s2 > 0:
        s = math.sqrt(s2)
        c, sn = gx / s, gy / s
    else:
        c, sn = 1.0, 0.0
    r2 = math.sqrt(2.0)
    e1 = np.array([c * c, sn * sn, r2 * c * sn])
    e2 = np.array([sn * sn, c * c, -r2 * c * sn])
    e3 = np.array([-r2 * c * sn, r2 * c * sn, c * c - sn * sn])
    return (g * np.outer(e1, e1) + np.outer(e2, e2)
            + mu3_rule(g, 1.0, mu3) * np.outer(e3, e3))


def P_matrix(u: np.ndarray, lam: float, sigma: float, diff: int = 0, mu3: int = 0) -> np.ndarray:
    """Dense P(u) = B^T M(u) B for an H x W image u."""
    H, W = u.shape
    N = H * W
    K = blur_matrix(H, W, sigma)
    Dx, Dy, Bxx, Byy, Bxy = derivative_matrices(H, W)
    v = K @ u.reshape(N)
    gx, gy = Dx @ v, Dy @ v
    r2 = math.sqrt(2.0)
    P = np.zeros((N, N))
    for p in range(N):
        Bp = np.stack([Bxx[p], Byy[p], r2 * Bxy[p]])
        P += Bp.T @ mandel_tensor(gx[p], gy[p], lam, diff, mu3) @ Bp
    return P


def F(u: np.ndarray, lam: float, sigma: float, diff: int = 0, mu3: int = 0) -> np.ndarray:
    """F(u) = P(u) u."""
    return (P_matrix(u, lam, sigma, diff, mu3) @ u.reshape(-1)).reshape(u.shape)


def biharmonic_symbol(H: int, W: int) -> np.ndarray:
    """Eigenvalues of P for g == 1 in the 2-D orthonormal DCT-II basis:
    16 sin^4(pi k/2H) + 16 sin^4(pi l/2W) + 2 sin^2(pi k/H) sin^2(pi l/W)."""
    k = np.arange(H)[:, None]
    l = np.arange(W)[None, :]
    return (16 * np.sin(np.pi * k / (2 * H)) ** 4 + 16 * np.sin(np.pi * l / (2 * W)) ** 4
            + 2 * np.sin(np.pi * k / H) ** 2 * np.sin(np.pi * l / W) ** 2)


def apply_biharmonic_dct(x: np.ndarray) -> np.ndarray:
    """P x for g == 1 through the DCT-II diagonalisation."""
    X = scipy.fft.dctn(x, type=2, norm="ortho")
    return scipy.fft.idctn(X * biharmonic_symbol(*x.shape), type=2, norm="ortho")
