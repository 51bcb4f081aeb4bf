"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's
formulas: they check closed forms, invariants, a second independent
formulation (explicit matrices), a DCT diagonalisation, finite differences
and brute force on tiny grids.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import matrix_oracle as mo

RNG = np.random.default_rng(12345)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")


def golden():
    out = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, val = line.split()[:2]
            out[name] = float(val)
    return out


def sym_matrix(a, b, c):
    """2x2 symmetric matrix as the oracle's 4-vector (xx, xy, yx, yy)."""
    return np.array([a, c, c, b])


# ---------------------------------------------------------------- P1 diffusivity
def test_charbonnier_closed_form():
    # eq. (CharDiff): g(s^2) = 1/sqrt(1 + s^2/lambda^2)
    lam = 0.07
    assert oracle.charbonnier(0.0, lam) == 1.0
    assert oracle.charbonnier(lam * lam, lam) == pytest.approx(1 / math.sqrt(2), rel=1e-15)
    assert oracle.charbonnier(3 * lam * lam, lam) == pytest.approx(0.5, rel=1e-15)
    assert oracle.charbonnier(1e6, 1e12) == pytest.approx(1.0, abs=1e-15)


def test_gauss_weights_normalised_and_symmetric():
    # Sec. 2.2 presmoothing: sampled Gaussian, radius ceil(3 sigma)
    for sigma, R in [(0.0, 0), (0.5, 2), (1.0, 3), (1.5, 5), (2.0, 6)]:
        assert oracle.radius(sigma) == R
        w = oracle.gauss(sigma)
        assert len(w) == 2 * R + 1
        assert w.sum() == pytest.approx(1.0, abs=1e-15)
        assert np.allclose(w, w[::-1], rtol=0, atol=0)
        if R:
            # ratio of neighbouring samples of exp(-j^2/(2 sigma^2))
            assert w[R + 1] / w[R] == pytest.approx(math.exp(-1 / (2 * sigma ** 2)), rel=1e-14)


# ---------------------------------------------------------------- P2 tensor
@pytest.mark.parametrize("gx,gy,lam", [(0.3, -0.2, 0.1), (1e-3, 2e-3, 0.05), (-2.0, 0.5, 0.7),
                                       (0.0, 0.4, 0.2)])
def test_tensor_spectrum(gx, gy, lam):
    # eqs. (faod_diffTensor), (foad_diffTensor_entries): eigenvalues g, 1, sqrt g, 0 with
    # eigentensors v1 v1^T, v2 v2^T, sym(v1 v2^T), antisym(v1 v2^T)
    d = oracle.tensor(gx, gy, lam)
    assert np.allclose(d, d.T, atol=1e-15)               # major symmetry
    s2 = gx * gx + gy * gy
    g = 1 / math.sqrt(1 + s2 / lam ** 2)
    ev, vec = np.linalg.eigh(d)
    assert np.allclose(np.sort(ev), np.sort([g, 1.0, math.sqrt(g), 0.0]), atol=1e-13)
    v1 = np.array([gx, gy]) / math.sqrt(s2)
    e1 = np.outer(v1, v1).reshape(4)
    # e1 is an eigenvector with eigenvalue g
    assert np.allclose(d @ e1, g * e1, atol=1e-13)
    v2 = np.array([-v1[1], v1[0]])
    e2 = np.outer(v2, v2).reshape(4)
    assert np.allclose(d @ e2, e2, atol=1e-13)


def test_tensor_identity_when_diffusivity_is_one():
    # Sec. 4.3: large lambda makes g close to 1, i.e. homogeneous fourth-order diffusion
    d = oracle.tensor(0.37, -0.81, 1e12)
    Hm = sym_matrix(0.3, -1.1, 0.45)
    assert np.allclose(d @ Hm, Hm, atol=1e-14)


def test_tensor_directional_form():
    # eq. (foad_diff_direc): D:H = mu1 u_v1v1 E1 + mu2 u_v2v2 E2 + mu3/sqrt2 (u_dd - u_ee) E3,
    # d, e = (v1 +- v2)/sqrt2
    for _ in range(20):
        gx, gy = RNG.normal(size=2)
        lam = RNG.uniform(0.05, 2.0)
        a, b, c = RNG.normal(size=3)
        Hm = np.array([[a, c], [c, b]])
        T = (oracle.tensor(gx, gy, lam) @ Hm.reshape(4)).reshape(2, 2)
        s = math.hypot(gx, gy)
        v1 = np.array([gx, gy]) / s
        v2 = np.array([-v1[1], v1[0]])
        g = 1 / math.sqrt(1 + s * s / lam ** 2)
        dd = (v1 + v2) / math.sqrt(2)
        ee = (v1 - v2) / math.sqrt(2)
        E1 = np.outer(v1, v1)
        E2 = np.outer(v2, v2)
        E3 = (np.outer(v1, v2) + np.outer(v2, v1)) / math.sqrt(2)
        ref = (g * (v1 @ Hm @ v1) * E1 + (v2 @ Hm @ v2) * E2
               + math.sqrt(g) / math.sqrt(2) * (dd @ Hm @ dd - ee @ Hm @ ee) * E3)
        assert np.allclose(T, ref, atol=1e-12)


# ---------------------------------------------------------------- P3 stencils
def test_stencils_exact_on_quadratics():
    # Sec. 3.3 finite differences (u_xy with corrected signs): exact second
    # derivatives of x^2, y^2, xy in the interior, zero on affine functions
    H, W = 9, 11
    y, x = np.mgrid[0:H, 0:W].astype(float)
    inner = (slice(1, -1), slice(1, -1))
    for u, ref in [(x * x, (2, 0, 0)), (y * y, (0, 0, 2)), (x * y, (0, 1, 0)),
                   (3 + 0 * x, (0, 0, 0)), (2 * x - 5 * y + 1, (0, 0, 0))]:
        hxx, hxy, hyy = oracle.hessian(u)
        assert np.allclose(hxx[inner], ref[0], atol=1e-12)
        assert np.allclose(hxy[inner], ref[1], atol=1e-12)
        assert np.allclose(hyy[inner], ref[2], atol=1e-12)


def test_gradient_of_linear_function():
    # central differences of a presmoothed affine function are exact in the interior
    H, W = 20, 24
    y, x = np.mgrid[0:H, 0:W].astype(float)
    gx, gy = oracle.gradient(0.3 * x - 0.7 * y, 1.0)
    inner = (slice(4, -4), slice(4, -4))
    assert np.allclose(gx[inner], 0.3, atol=1e-12)
    assert np.allclose(gy[inner], -0.7, atol=1e-12)


# ---------------------------------------------------------------- P4 operator, frozen tensor
@pytest.mark.parametrize("H,W,sigma,lam", [(5, 5, 1.0, 0.1), (6, 7, 1.5, 0.05), (8, 8, 0.0, 0.2),
                                           (4, 9, 2.0, 0.03), (1, 7, 1.0, 0.1)])
def test_P_symmetric_psd(H, W, sigma, lam):
    # Sec. 3.3: P_k positive semi-definite; FSI needs P symmetric
    ut = RNG.uniform(0, 1, (H, W))
    N = H * W
    P = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1
        P[:, j] = oracle.apply_P(ut, e.reshape(H, W), lam, sigma).reshape(N)
    scale = np.abs(P).max()
    assert np.abs(P - P.T).max() <= 1e-12 * scale
    ev = np.linalg.eigvalsh(0.5 * (P + P.T))
    assert ev.min() >= -1e-12 * scale
    assert ev.max() <= 32 + 1e-9
    assert np.abs(P @ np.ones(N)).max() <= 1e-12 * scale


def test_step_bound_is_sufficient():
    # eq. (timeStepBound) gives 1/17 for unit spacing; the largest eigenvalue of P is at
    # most 32, so any tau <= 2/32 is L2-stable and the paper's bound lies inside it
    gold = golden()
    assert gold["tau_bound_theory"] == pytest.approx(2 / (16 + 16 + 2), rel=1e-12)
    assert gold["tau_bound_theory"] <= 2 / 32
    sym = mo.biharmonic_symbol(64, 64)
    assert sym.max() <= 32 and sym.max() > 31.9


# ---------------------------------------------------------------- P5 g == 1 closed form
@pytest.mark.parametrize("H,W,sigma", [(9, 8, 1.0), (16, 5, 2.0), (1, 12, 1.5), (2, 3, 1.0),
                                       (33, 31, 0.0)])
def test_biharmonic_dct_closed_form(H, W, sigma):
    # with g == 1 (lambda -> infinity) the operator is the mirrored biharmonic, diagonal in
    # the 2-D DCT-II (textbook); pins stencils, mixed term signs and boundary handling
    u = RNG.uniform(0, 1, (H, W))
    x = RNG.normal(size=(H, W))
    got = oracle.apply_P(u, x, 1e12, sigma)
    ref = mo.apply_biharmonic_dct(x)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


# ---------------------------------------------------------------- P6 FSI recursion
def fsi_polynomial(n, x):
    # the FSI cycle as a polynomial in x = eigenvalue of (I - tau P), Sec. 3.3
    p_prev = np.ones_like(x)
    p = np.ones_like(x)
    for k in range(n):
        a = (4 * k + 2) / (2 * k + 3)
        p, p_prev = a * x * p + (1 - a) * p_prev, p
    return p


@pytest.mark.parametrize("n", [1, 2, 10, 15, 40])
def test_fsi_polynomial_properties(n):
    # Hafner et al. (cited in Sec. 3.3): a cycle of n steps is stable for |x| <= 1 and
    # reaches diffusion time tau * n(n+1)/3
    x = np.linspace(-1, 1, 20001)
    p = fsi_polynomial(n, x)
    assert np.abs(p).max() <= 1 + 1e-9
    h = 1e-6
    dp = (fsi_polynomial(n, np.array([1 + h])) - fsi_polynomial(n, np.array([1 - h]))) / (2 * h)
    assert dp[0] == pytest.approx(n * (n + 1) / 3, rel=1e-6)


@pytest.mark.parametrize("n,cycles", [(10, 1), (15, 2), (4, 3)])
def test_fsi_cycle_matches_dct_prediction(n, cycles):
    H, W, tau = 12, 10, 0.05
    u0 = RNG.uniform(0, 1, (H, W))
    mask = np.zeros((H, W), np.uint8)
    u, cyc, _ = oracle.inpaint(u0, mask, np.zeros((H, W)), 1e12, 1.0, tau, n, cycles)
    assert cyc == cycles
    X = mo.scipy.fft.dctn(u0, type=2, norm="ortho")
    mult = fsi_polynomial(n, 1 - tau * mo.biharmonic_symbol(H, W)) ** cycles
    ref = mo.scipy.fft.idctn(X * mult, type=2, norm="ortho")
    assert np.abs(u - ref).max() <= 1e-11


def predicted_history(u0, n, tau, M):
    """Cycle residuals of the g == 1, mask-free evolution from the DCT closed form.

    Cycle m multiplies DCT mode (k, l) by p_n(1 - tau rho_kl) (Sec. 3.3 FSI
    recursion), and the orthonormal DCT keeps 2-norms, so with X = DCT(u0):
    ||u^{m+1,0} - u^{m,0}|| = ||(p^{m+1} - p^m) X|| and ||u^{m+1,0}|| = ||p^{m+1} X||.
    Returns [M, 2] of (residual, norm)."""
    H, W = u0.shape
    X = mo.scipy.fft.dctn(u0, type=2, norm="ortho")
    p = fsi_polynomial(n, 1 - tau * mo.biharmonic_symbol(H, W))
    out = np.zeros((M, 2))
    for m in range(M):
        out[m, 0] = np.linalg.norm((p ** (m + 1) - p ** m) * X)
        out[m, 1] = np.linalg.norm(p ** (m + 1) * X)
    return out


def test_residual_history_matches_dct_closed_form():
    # the per-cycle residual and norm that the stop rule of Sec. 3.3 reads, against the
    # closed form of the linear (g == 1) evolution without known pixels
    H, W, n, tau, M = 11, 13, 10, 0.05, 25
    u0 = RNG.uniform(0, 1, (H, W))
    _, cyc, hist = oracle.inpaint(u0, np.zeros((H, W), np.uint8), np.zeros((H, W)), 1e12, 1.0,
                                  tau, n, M)
    ref = predicted_history(u0, n, tau, M)
    assert cyc == M
    assert np.allclose(hist, ref, rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("abs_tol", [False, True])
@pytest.mark.parametrize("stop_at", [1, 4, 9])
def test_stop_rule_is_first_cycle_below_tol(abs_tol, stop_at):
    # Sec. 3.3: stop after the FIRST cycle whose residual is below tol (relative to
    # ||u^{m,n}|| by default, plain with abs_tol).  tol is set halfway between the
    # predicted criterion of cycle stop_at and the smallest of the cycles before it, so
    # an oracle that stops a cycle early or late, or tests the wrong norm, fails.
    # The constant offset leaves every residual unchanged (P 1 = 0) and makes ||u|| about
    # 100, so the relative and the plain criterion stop at clearly different cycles.
    H, W, n, tau, M = 12, 9, 8, 0.05, 40
    u0 = 10.0 + np.random.default_rng(2024).uniform(0, 1, (H, W))
    ref = predicted_history(u0, n, tau, M)
    crit = ref[:, 0] if abs_tol else ref[:, 0] / ref[:, 1]
    before = crit[:stop_at].min()
    assert crit[stop_at] < before
    tol = 0.5 * (crit[stop_at] + before)
    # with the other norm the rule would stop at a different cycle (or not at all)
    other = ref[:, 0] / ref[:, 1] if abs_tol else ref[:, 0]
    below = np.flatnonzero(other < tol)
    assert below.size == 0 or below[0] != stop_at
    _, cyc, hist = oracle.inpaint(u0, np.zeros((H, W), np.uint8), np.zeros((H, W)), 1e12, 1.0,
                                  tau, n, M, tol=tol, abs_tol=abs_tol)
    assert cyc == stop_at + 1
    assert hist.shape == (stop_at + 1, 2)
    assert np.allclose(hist, ref[:stop_at + 1], rtol=1e-11, atol=1e-14)


def test_batch_stop_rule_waits_for_every_image():
    # an equal-size batch stops at the first cycle where every image's relative residual is
    # below tol: the slower image decides
    H, W, n, tau, M = 10, 10, 6, 0.05, 60
    rng = np.random.default_rng(77)
    fast = rng.uniform(0, 1, (H, W))
    slow = np.add.outer(np.linspace(0, 1, H), np.linspace(0, 0.5, W)) + 0.01 * rng.normal(size=(H, W))
    rf = predicted_history(fast, n, tau, M)
    rs = predicted_history(slow, n, tau, M)
    worst = np.maximum(rf[:, 0] / rf[:, 1], rs[:, 0] / rs[:, 1])
    c = 6
    assert worst[c] < worst[:c].min()
    tol = 0.5 * (worst[c] + worst[:c].min())
    first_fast = int(np.argmax(rf[:, 0] / rf[:, 1] < tol))
    first_slow = int(np.argmax(rs[:, 0] / rs[:, 1] < tol))
    assert first_fast != first_slow        # the two images alone would stop at different cycles
    u0 = np.stack([fast, slow])
    z = np.zeros((2, H, W))
    _, cyc, hist = oracle.inpaint(u0, np.zeros((2, H, W), np.uint8), z, 1e12, 1.0, tau, n, M,
                                  tol=tol)
    assert cyc == c + 1
    assert np.allclose(hist[:, 0], rf[:c + 1], rtol=1e-11, atol=1e-14)
    assert np.allclose(hist[:, 1], rs[:c + 1], rtol=1e-11, atol=1e-14)


# ---------------------------------------------------------------- P7 symmetries
def small_problem(H=14, W=13, density=0.15, seed=7):
    rng = np.random.default_rng(seed)
    img = rng.uniform(0, 1, (H, W))
    img[H // 3:, W // 2:] += 0.5
    mask = (rng.uniform(size=(H, W)) < density).astype(np.uint8)
    mask[0, 0] = 1
    known = np.where(mask != 0, img, 0.0)
    u0 = np.where(mask != 0, img, img[mask != 0].mean())
    return img, mask, known, u0


def test_constant_image_is_stationary():
    # constant images are steady states (zero Hessian); known pixels agree with it
    H, W = 11, 9
    c = 0.3721
    u0 = np.full((H, W), c)
    mask = np.zeros((H, W), np.uint8)
    mask[3, 4] = 1
    u, _, _ = oracle.inpaint(u0, mask, u0, 0.05, 1.5, 0.05, 10, 3)
    assert np.abs(u - c).max() <= 1e-15


def test_shift_and_scale_equivariance():
    img, mask, known, u0 = small_problem()
    lam, sigma, tau, n, M = 0.1, 1.0, 0.05, 8, 3
    u, _, _ = oracle.inpaint(u0, mask, known, lam, sigma, tau, n, M)
    us, _, _ = oracle.inpaint(u0 + 0.25, mask, known + 0.25, lam, sigma, tau, n, M)
    assert np.abs(us - (u + 0.25)).max() <= 1e-12
    a = 3.0
    ua, _, _ = oracle.inpaint(a * u0, mask, a * known, a * lam, sigma, tau, n, M)
    assert np.abs(ua - a * u).max() <= 1e-12


@pytest.mark.parametrize("op", ["fliplr", "flipud", "transpose", "rot90"])
def test_dihedral_equivariance(op):
    img, mask, known, u0 = small_problem(12, 12)
    f = {"fliplr": np.fliplr, "flipud": np.flipud, "transpose": np.transpose,
         "rot90": np.rot90}[op]
    args = (0.08, 1.0, 0.05, 6, 2)
    u, _, _ = oracle.inpaint(u0, mask, known, *args)
    ut, _, _ = oracle.inpaint(f(u0).copy(), f(mask).copy(), f(known).copy(), *args)
    assert np.abs(ut - f(u)).max() <= 1e-12


# ---------------------------------------------------------------- P8 Dirichlet
def test_known_pixels_held_exactly():
    # eq. (inpaintingModel): u = f on K for all t
    img, mask, known, u0 = small_problem()
    u, _, _ = oracle.inpaint(u0 + 0.1, mask, known, 0.1, 1.0, 0.05, 10, 2)
    assert np.array_equal(u[mask != 0], known[mask != 0])


# ---------------------------------------------------------------- P9 smoothing variant
def test_mean_preserved_without_mask():
    # Sec. 2.3: fourth-order filters preserve the average grey value
    H, W = 15, 17
    u0 = RNG.uniform(0, 1, (H, W))
    mask = np.zeros((H, W), np.uint8)
    u, _, _ = oracle.inpaint(u0, mask, np.zeros((H, W)), 0.05, 1.0, 0.05, 10, 3)
    assert abs(u.mean() - u0.mean()) <= 1e-13
    assert np.abs(u - u0).max() > 1e-3


@pytest.mark.parametrize("lam", [0.02, 0.1, 1.0])
def test_l2_stability_explicit_step(lam):
    # eq. (l2stability) for the smoothing variant at tau = 1/17 (eq. timeStepBound) and at
    # tau = 1/16.  An FSI step with k = 0 is an explicit step of size alpha_0 tau = 2 tau/3.
    H, W = 16, 14
    gold = golden()
    for tau_eff in (gold["tau_bound_theory"], 1 / 16):
        u = RNG.uniform(0, 1, (H, W))
        for _ in range(15):
            un = oracle.step(u, u, None, None, lam, 1.0, 1.5 * tau_eff, 0)
            assert np.linalg.norm(un) <= np.linalg.norm(u) * (1 + 1e-14)
            u = un


# ---------------------------------------------------------------- P10 steady state
def test_converges_to_steady_state():
    # Sec. 2.1 / 3.3: iterate until the cycle residual is small; the result is a steady
    # state, i.e. P(u)u vanishes off the mask
    img, mask, known, u0 = small_problem(12, 12, 0.2)
    lam, sigma, tau = 0.1, 1.0, 0.05
    u, cyc, hist = oracle.inpaint(u0, mask, known, lam, sigma, tau, 20, 3000, tol=1e-9)
    rel = hist[:, 0] / hist[:, 1]
    assert rel[-1] < 1e-9
    assert cyc < 3000
    r0 = oracle.apply_P(u0, u0, lam, sigma)[mask == 0]
    r = oracle.apply_P(u, u, lam, sigma)[mask == 0]
    assert np.linalg.norm(r) <= 1e-5 * np.linalg.norm(r0)


def test_initialisation_independence_report():
    # Sec. 3.3 observes a steady state independent of the initialisation; the iteration is
    # nonlinear, so this is only checked loosely
    img, mask, known, u0 = small_problem(12, 12, 0.25)
    args = (0.1, 1.0, 0.05, 20, 3000)
    ua, _, _ = oracle.inpaint(u0, mask, known, *args, tol=1e-10)
    ub, _, _ = oracle.inpaint(np.where(mask != 0, known, 0.0), mask, known, *args, tol=1e-10)
    assert np.abs(ua - ub).max() < 5e-2


# ---------------------------------------------------------------- P11 two formulations
@pytest.mark.parametrize("H,W,sigma,lam", [(5, 5, 1.0, 0.1), (6, 7, 1.5, 0.05), (8, 8, 0.0, 0.3),
                                           (3, 9, 2.0, 0.05), (7, 6, 1.0, 0.02)])
def test_extended_vs_matrix_formulation(H, W, sigma, lam):
    u = RNG.uniform(0, 1, (H, W))
    u[: H // 2] += 0.4
    got = oracle.apply_P(u, u, lam, sigma)
    ref = mo.F(u, lam, sigma)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_step_matches_matrix_form():
    # u^{k+1} = alpha (I - tau P) u^k + (1 - alpha) u^{k-1}, then hold on the mask
    H, W = 6, 7
    u = RNG.uniform(0, 1, (H, W))
    up = RNG.uniform(0, 1, (H, W))
    mask = np.zeros((H, W), np.uint8)
    mask[2, 3] = 1
    f = np.full((H, W), 0.123)
    k, tau, lam, sigma = 3, 0.05, 0.1, 1.0
    got = oracle.step(u, up, mask, f, lam, sigma, tau, k)
    a = (4 * k + 2) / (2 * k + 3)
    P = mo.P_matrix(u, lam, sigma)
    ref = (a * (u.reshape(-1) - tau * P @ u.reshape(-1)) + (1 - a) * up.reshape(-1)).reshape(H, W)
    ref[2, 3] = 0.123
    assert np.abs(got - ref).max() <= 1e-13


# ---------------------------------------------------------------- P12 adjoint
def test_e_grad_by_finite_differences():
    for _ in range(10):
        gx, gy = RNG.normal(size=2) * 0.2
        lam = RNG.uniform(0.05, 0.5)
        A = sym_matrix(*RNG.normal(size=3))
        Hm = sym_matrix(*RNG.normal(size=3))
        e, q, dl = oracle.e_grad(gx, gy, A, Hm, lam)
        d = oracle.tensor(gx, gy, lam)
        assert e == pytest.approx(A @ d @ Hm, rel=1e-13, abs=1e-15)
        h = 1e-6
        ex = lambda a, b, l=lam: oracle.e_grad(a, b, A, Hm, l)[0]
        assert q[0] == pytest.approx((ex(gx + h, gy) - ex(gx - h, gy)) / (2 * h), rel=1e-6, abs=1e-8)
        assert q[1] == pytest.approx((ex(gx, gy + h) - ex(gx, gy - h)) / (2 * h), rel=1e-6, abs=1e-8)
        assert dl == pytest.approx((ex(gx, gy, lam + h) - ex(gx, gy, lam - h)) / (2 * h),
                                   rel=1e-6, abs=1e-8)


def test_e_grad_vanishes_at_zero_gradient():
    A = sym_matrix(0.3, -0.2, 0.5)
    Hm = sym_matrix(-1.0, 0.4, 0.1)
    e, q, dl = oracle.e_grad(0.0, 0.0, A, Hm, 0.1)
    assert e == pytest.approx(A @ Hm)
    assert np.all(q == 0) and dl == 0


@pytest.mark.parametrize("H,W,sigma,lam", [(6, 5, 1.0, 0.1), (7, 8, 1.5, 0.05), (4, 4, 0.0, 0.2)])
def test_jtv_against_fd_jacobian(H, W, sigma, lam):
    u = RNG.uniform(0, 1, (H, W))
    N = H * W
    J = np.zeros((N, N))
    h = 1e-6
    for j in range(N):
        e = np.zeros(N)
        e[j] = h
        e = e.reshape(H, W)
        J[:, j] = ((mo.F(u + e, lam, sigma) - mo.F(u - e, lam, sigma)) / (2 * h)).reshape(N)
    w = RNG.normal(size=(H, W))
    got, dl = oracle.jtv(u, w, lam, sigma)
    ref = (J.T @ w.reshape(N)).reshape(H, W)
    assert np.abs(got - ref).max() <= 1e-6 * np.abs(ref).max()
    Fl = (mo.F(u, lam + h, sigma) - mo.F(u, lam - h, sigma)) / (2 * h)
    assert dl == pytest.approx(float((Fl * w).sum()), rel=1e-6)


def test_backward_against_central_differences():
    # adjoint of the full FSI evolution vs central differences with h = 1e-3
    img, mask, known, u0 = small_problem(9, 8, 0.25, seed=3)
    lam, sigma, tau, n, M = 0.1, 1.0, 0.05, 4, 3
    wgt = np.random.default_rng(5).normal(size=img.shape)

    def loss(known_, u0_, lam_):
        u, _, _ = oracle.inpaint(u0_, mask, known_, lam_, sigma, tau, n, M)
        return float((wgt * u).sum())

    u, cyc, _, ck = oracle.inpaint(u0, mask, known, lam, sigma, tau, n, M, checkpoints=True)
    gf, gi, gl = oracle.backward(ck, mask, known, lam, sigma, tau, n, wgt)
    h = 1e-3
    ks = np.argwhere(mask != 0)[:4]
    for (y, x) in ks:
        kp = known.copy(); kp[y, x] += h
        km = known.copy(); km[y, x] -= h
        fd = (loss(kp, np.where(mask != 0, kp, u0), lam) - loss(km, np.where(mask != 0, km, u0), lam)) / (2 * h)
        assert gf[y, x] == pytest.approx(fd, rel=1e-5, abs=1e-9)
    us = np.argwhere(mask == 0)[:4]
    for (y, x) in us:
        up = u0.copy(); up[y, x] += h
        um = u0.copy(); um[y, x] -= h
        fd = (loss(known, up, lam) - loss(known, um, lam)) / (2 * h)
        assert gi[y, x] == pytest.approx(fd, rel=1e-5, abs=1e-9)
    assert np.all(gf[mask == 0] == 0) and np.all(gi[mask != 0] == 0)
    fd = (loss(known, u0, lam + h) - loss(known, u0, lam - h)) / (2 * h)
    assert gl == pytest.approx(fd, rel=1e-3)
