"""Pins of the oracle's tensor variants: the diffusivities compared in Table 7
and the choices of mu_3 compared in Sec. 3.1 (Table 1).

The Charbonnier / geometric-mean tensor (FOEED) is pinned by
test_oracle_pins.py; here every other combination is pinned the same way:
structural identities of each diffusivity (not its formula re-typed), the
spectrum of the tensor against the paper's definitions of mu_3 in terms of
mu_1 and mu_2, the homogeneous limit (DCT closed form), the second (matrix)
formulation, symmetry and semi-definiteness of P, and finite differences of
the adjoint's derivatives.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import matrix_oracle as mo

RNG = np.random.default_rng(2024)
DIFFS = range(len(oracle.DIFFUSIVITIES))
RULES = range(len(oracle.MU3_RULES))
COMBOS = [(d, r) for d in DIFFS for r in RULES]


def sym_matrix(a, b, c):
    return np.array([a, c, c, b])


# ------------------------------------------------------------ diffusivities (Table 7)
@pytest.mark.parametrize("diff", DIFFS)
def test_diffusivity_is_decreasing_from_one(diff):
    # a nonnegative decreasing diffusivity (Sec. 3.1), 1 where the gradient vanishes
    lam = 0.05
    s = np.linspace(0.0, 10 * lam, 400)
    g = np.array([oracle.diffusivity(x * x, lam, diff) for x in s])
    assert g[0] == 1.0
    assert np.all(np.diff(g) < 0)
    assert np.all(g > 0) and np.all(g <= 1)


def test_charbonnier_squared_is_perona_malik():
    # Table 7: 1/sqrt(1+(s/l)^2) squared is 1/(1+(s/l)^2), for every s and lambda
    for s2, lam in [(0.0, 0.1), (1e-4, 0.02), (0.3, 0.7), (5.0, 0.05)]:
        ch = oracle.diffusivity(s2, lam, 0)
        assert ch == pytest.approx(oracle.charbonnier(s2, lam), rel=1e-15)
        assert ch * ch == pytest.approx(oracle.diffusivity(s2, lam, 1), rel=1e-14)


def test_perona_malik_reciprocal_is_affine_in_s2():
    # 1/g - 1 = (s/lambda)^2: additive in s^2 and equal to 1 at s = lambda
    lam = 0.03
    h = lambda s2: 1.0 / oracle.diffusivity(s2, lam, 1) - 1.0
    assert h(lam * lam) == pytest.approx(1.0, rel=1e-14)
    for a, b in [(1e-4, 3e-4), (2e-3, 5e-2), (0.1, 0.7)]:
        assert h(a) + h(b) == pytest.approx(h(a + b), rel=1e-12)


def test_exponential_perona_malik_is_multiplicative_in_s2():
    # exp(-(s/lambda)^2): g(a) g(b) = g(a + b) in s^2, and g = 1/e at s = lambda
    lam = 0.08
    g = lambda s2: oracle.diffusivity(s2, lam, 2)
    assert g(lam * lam) == pytest.approx(math.exp(-1.0), rel=1e-14)
    for a, b in [(1e-3, 2e-3), (0.01, 0.03), (0.2, 0.05)]:
        assert g(a) * g(b) == pytest.approx(g(a + b), rel=1e-12)


def test_geman_reynolds_is_the_printed_function_scaled_to_one():
    # Table 7 prints 2 lambda^2 / (s^2 + lambda^2)^2; the reading used divides it by its
    # value 2 / lambda^2 at s = 0; it is then the square of Perona-Malik
    for s2, lam in [(0.0, 0.1), (1e-3, 0.02), (0.4, 0.3), (2.0, 0.05)]:
        printed = 2 * lam ** 2 / (s2 + lam ** 2) ** 2
        got = oracle.diffusivity(s2, lam, 3)
        assert got == pytest.approx(printed / (2 / lam ** 2), rel=1e-14)
        assert got == pytest.approx(oracle.diffusivity(s2, lam, 1) ** 2, rel=1e-14)


# ------------------------------------------------------------ tensor spectrum (Sec. 3.1)
@pytest.mark.parametrize("diff,rule", COMBOS)
def test_tensor_spectrum_and_mu3_rule(diff, rule):
    # eigentensors v1v1^T (mu1 = g), v2v2^T (mu2 = 1), sym(v1v2^T) (mu3), antisym (0); mu3 is
    # the geometric mean, the arithmetic mean or the maximum of mu1 and mu2 (Table 1)
    for gx, gy, lam in [(0.3, -0.2, 0.1), (1e-3, 2e-3, 0.05), (-2.0, 0.5, 0.7), (0.0, 0.4, 0.2)]:
        d = oracle.tensor(gx, gy, lam, diff, rule)
        assert np.allclose(d, d.T, atol=1e-15)
        s = math.hypot(gx, gy)
        v1 = np.array([gx, gy]) / s
        v2 = np.array([-v1[1], v1[0]])
        E = [np.outer(v1, v1).reshape(4), np.outer(v2, v2).reshape(4),
             ((np.outer(v1, v2) + np.outer(v2, v1)) / math.sqrt(2)).reshape(4),
             ((np.outer(v1, v2) - np.outer(v2, v1)) / math.sqrt(2)).reshape(4)]
        mu = [float(e @ d @ e) for e in E]
        for e, m in zip(E, mu):
            assert np.allclose(d @ e, m * e, atol=1e-13)       # each E_i is an eigentensor
        assert mu[0] == pytest.approx(oracle.diffusivity(s * s, lam, diff), rel=1e-13)
        assert mu[1] == pytest.approx(1.0, abs=1e-14)
        assert mu[3] == pytest.approx(0.0, abs=1e-14)
        want = {0: math.sqrt(mu[0] * mu[1]), 1: 0.5 * (mu[0] + mu[1]), 2: max(mu[0], mu[1])}[rule]
        assert mu[2] == pytest.approx(want, rel=1e-12, abs=1e-13)
        assert np.allclose(np.sort(np.linalg.eigvalsh(d)), np.sort(mu), atol=1e-13)


@pytest.mark.parametrize("diff,rule", COMBOS)
def test_homogeneous_limit_is_the_dct_biharmonic(diff, rule):
    # lambda -> infinity: g -> 1 and every mu_3 rule gives 1, so P is the mirrored biharmonic
    H, W = 7, 9
    x = RNG.normal(size=(H, W))
    ut = RNG.uniform(0, 1, (H, W))
    got = oracle.apply_P(ut, x, 1e12, 1.0, diff, rule)
    assert np.abs(got - mo.apply_biharmonic_dct(x)).max() <= 1e-11 * np.abs(x).max()


@pytest.mark.parametrize("diff,rule", COMBOS)
def test_extended_vs_matrix_formulation(diff, rule):
    H, W, sigma, lam = 6, 7, 1.0, 0.05
    u = RNG.uniform(0, 1, (H, W))
    u[: H // 2] += 0.4
    got = oracle.apply_P(u, u, lam, sigma, diff, rule)
    ref = mo.F(u, lam, sigma, diff, rule)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("diff,rule", [(1, 0), (2, 1), (3, 2), (0, 1)])
def test_P_symmetric_psd(diff, rule):
    # Sec. 3.3: P symmetric positive semi-definite; with every mu_i in [0, 1] its spectrum
    # stays in [0, 32], so tau <= 1/16 remains sufficient
    H, W, sigma, lam = 5, 6, 1.0, 0.05
    ut = RNG.uniform(0, 1, (H, W))
    N = H * W
    P = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1
        P[:, j] = oracle.apply_P(ut, e.reshape(H, W), lam, sigma, diff, rule).reshape(N)
    scale = np.abs(P).max()
    assert np.abs(P - P.T).max() <= 1e-12 * scale
    ev = np.linalg.eigvalsh(0.5 * (P + P.T))
    assert ev.min() >= -1e-12 * scale
    assert ev.max() <= 32 + 1e-9


@pytest.mark.parametrize("diff,rule", [(1, 0), (2, 1), (3, 2), (0, 2)])
def test_constant_image_stationary_and_hold(diff, rule):
    H, W = 8, 9
    u = np.full((H, W), 0.37)
    mask = np.zeros((H, W), np.uint8)
    mask[3, 4] = 1
    f = np.full((H, W), 0.37)
    out = oracle.step(u, u, mask, f, 0.05, 1.0, 0.05, 2, diff, rule)
    assert np.abs(out - 0.37).max() <= 1e-15


# ------------------------------------------------------------ adjoint derivatives
@pytest.mark.parametrize("diff,rule", COMBOS)
def test_e_grad_by_finite_differences(diff, rule):
    for _ in range(4):
        gx, gy = RNG.normal(size=2) * 0.2
        lam = RNG.uniform(0.05, 0.5)
        A = sym_matrix(*RNG.normal(size=3))
        Hm = sym_matrix(*RNG.normal(size=3))
        e, q, dl = oracle.e_grad(gx, gy, A, Hm, lam, diff, rule)
        assert e == pytest.approx(A @ oracle.tensor(gx, gy, lam, diff, rule) @ Hm,
                                  rel=1e-13, abs=1e-15)
        h = 1e-6
        ex = lambda a, b, l=lam: oracle.e_grad(a, b, A, Hm, l, diff, rule)[0]
        assert q[0] == pytest.approx((ex(gx + h, gy) - ex(gx - h, gy)) / (2 * h), rel=1e-6, abs=1e-8)
        assert q[1] == pytest.approx((ex(gx, gy + h) - ex(gx, gy - h)) / (2 * h), rel=1e-6, abs=1e-8)
        assert dl == pytest.approx((ex(gx, gy, lam + h) - ex(gx, gy, lam - h)) / (2 * h),
                                   rel=1e-6, abs=1e-8)


def test_e_grad_finite_where_exponential_diffusivity_underflows():
    # exp(-(s/lambda)^2) is 0 in double for s >> lambda; the derivatives must stay finite
    A = sym_matrix(0.3, -0.2, 0.5)
    Hm = sym_matrix(-1.0, 0.4, 0.1)
    for rule in RULES:
        e, q, dl = oracle.e_grad(3.0, -4.0, A, Hm, 0.01, 2, rule)
        assert np.isfinite(e) and np.all(np.isfinite(q)) and np.isfinite(dl)


@pytest.mark.parametrize("diff,rule", [(1, 1), (2, 0), (3, 2)])
def test_jtv_against_fd_jacobian(diff, rule):
    H, W, sigma, lam = 6, 5, 1.0, 0.1
    u = RNG.uniform(0, 1, (H, W))
    N = H * W
    J = np.zeros((N, N))
    h = 1e-6
    for j in range(N):
        e = np.zeros(N)
        e[j] = h
        e = e.reshape(H, W)
        J[:, j] = ((mo.F(u + e, lam, sigma, diff, rule) - mo.F(u - e, lam, sigma, diff, rule))
                   / (2 * h)).reshape(N)
    w = RNG.normal(size=(H, W))
    got, dl = oracle.jtv(u, w, lam, sigma, diff, rule)
    ref = (J.T @ w.reshape(N)).reshape(H, W)
    assert np.abs(got - ref).max() <= 1e-6 * np.abs(ref).max()
    Fl = (mo.F(u, lam + h, sigma, diff, rule) - mo.F(u, lam - h, sigma, diff, rule)) / (2 * h)
    assert dl == pytest.approx(float((Fl * w).sum()), rel=1e-6)
