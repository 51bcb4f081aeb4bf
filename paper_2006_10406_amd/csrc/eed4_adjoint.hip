// Adjoint of the FSI evolution (reverse mode), for the gradient of a loss on
// the inpainted image with respect to the known values f and the contrast
// lambda.  The paper states only the forward scheme (Sec. 3.3); the reverse
// recursion below is derived from it.
//
// Forward step k (F(u) = P(u) u, P from the tensor of Sec. 3.1):
//   u^{k+1} = mbar * [alpha_k (u^k - tau F(u^k)) + (1 - alpha_k) u^{k-1}] + m * f
// Reverse step k, given ubar^{k+1}:
//   fbar += m * ubar^{k+1};  r = mbar * ubar^{k+1}
//   ubar^k     += alpha_k (r - tau J_F(u^k)^T r)
//   ubar^{k-1} += (1 - alpha_k) r                (added to ubar^0 when k = 0)
//   lambdabar  += -alpha_k tau <dF/dlambda, r>
// with J_F(u)^T r = P(u) r + C^T q, C = (grad of the presmoothed image) and
// q_p = de_p/dG_p for e_p = (B r)_p : D(G_p) : (B u)_p (B = Hessian).
// Everything is evaluated on the mirror-extended image, which makes every
// transpose exact: q_x comes out odd across vertical borders and even across
// horizontal ones, q_y the reverse.
//
// Two implementations of a reverse step:
//  - workgroup tiles: pass A computes P(u) r, q and de/dlambda into global
//    buffers; pass B applies C^T q = K_sigma (-div q) and the update;
//  - wave strips (one launch): a wave streams down a strip and carries every
//    intermediate in registers and per-wave LDS, as the forward strip kernel
//    does.  It reads the presmoothed image K_sigma * u^k, which the forward
//    recompute keeps, instead of blurring u^k again: that saves the blur's
//    arithmetic and R rows of halo at each end of a segment.
// Known pixels: r is 0 there, so ubar on a known pixel feeds nothing but fbar.
// Both implementations therefore keep on known pixels the running sum of ubar
// over the reverse steps done so far; fbar is that sum at the end.  lambdabar
// is accumulated per work item across all reverse steps and reduced once.
#include "eed4.h"
#include "eed4_host.h"
#include "eed4_internal.h"
#include "eed4_strip.h"
#include "eed4_tile.h"

#include <cmath>
#include <vector>

namespace eed4 {

constexpr int kAdjTW = 64, kAdjTH = 16;

// Per-point pieces of the adjoint.  (gx, gy) = G = grad u_sigma; A = Hessian
// of r, H = Hessian of u.  Outputs: D(G) : A, q = de/dG and s de/ds with
// e = A : D(G) : H, s = |G|; mu depends on s/lambda only, so de/dlambda =
// -(s/lambda) de/ds, and the 1/lambda goes into the per-step scale.  In the gradient frame n = G/|G|, t = n rotated by +90
// degrees, e = A:H + (mu1 - 1) a1 h1 + 2 (mu3 - 1) a3 h3 with a1 = n.A.n,
// a3 = t.A.n; d/ds and d/dtheta of it give q = (de/ds) n + (1/s)(de/dtheta) t.
// Eigenvalue data of a tensor variant (diffusivities of Table 7, mu3 choices
// of Sec. 3.1) at x = (s/lambda)^2: mu1 = g(x), mu3, their derivatives G1, G3
// with respect to x, and Q1 = (mu1 - 1)/x, Q3 = (mu3 - 1)/x, written so that
// they stay finite at x = 0 (every variant has g(0) = 1).
struct MuData {
    float mu1, mu3, G1, G3, Q1, Q3;
};

__device__ __forceinline__ MuData model_mu_data(float x, int model)
{
    const int diff = model & 0xf, rule = model >> 4;
    const float d = 1.0f + x;
    MuData m;
    if (diff == kDiffPeronaMalik) {                  // (1 + x)^-1
        m.mu1 = __builtin_amdgcn_rcpf(d);
        m.G1 = -m.mu1 * m.mu1;
        m.Q1 = -m.mu1;
    } else if (diff == kDiffPeronaMalikExp) {        // exp(-x)
        m.mu1 = expf(-x);
        m.G1 = -m.mu1;
        m.Q1 = x > 0.0f ? expm1f(-x) / x : -1.0f;
    } else if (diff == kDiffGemanReynolds) {         // (1 + x)^-2
        const float r = __builtin_amdgcn_rcpf(d);
        m.mu1 = r * r;
        m.G1 = -2.0f * m.mu1 * r;
        m.Q1 = -(2.0f + x) * m.mu1;
    } else {                                         // Charbonnier (1 + x)^-1/2
        m.mu1 = __builtin_amdgcn_rsqf(d);
        m.G1 = -0.5f * m.mu1 * m.mu1 * m.mu1;
        m.Q1 = -m.mu1 * m.mu1 * __builtin_amdgcn_rcpf(1.0f + m.mu1);
    }
    if (rule == kMu3Arithmetic) {                    // (mu1 + mu2)/2
        m.mu3 = 0.5f * (1.0f + m.mu1);
        m.G3 = 0.5f * m.G1;
        m.Q3 = 0.5f * m.Q1;
    } else if (rule == kMu3Max) {                    // max(mu1, mu2) = 1
        m.mu3 = 1.0f;
        m.G3 = 0.0f;
        m.Q3 = 0.0f;
    } else {                                         // sqrt(mu1 mu2)
        m.mu3 = __builtin_amdgcn_sqrtf(m.mu1);
        m.G3 = m.mu1 > 0.0f ? 0.5f * m.G1 * __builtin_amdgcn_rcpf(m.mu3) : 0.0f;
        m.Q3 = m.Q1 * __builtin_amdgcn_rcpf(1.0f + m.mu3);
    }
    return m;
}

template <bool GEN = false>
__device__ __forceinline__ void adjoint_point(float gx, float gy, float inv_lam2, float axx,
                                              float ayy, float axy, float hxx, float hyy,
                                              float hxy, float &txx, float &tyy, float &txy,
                                              float &qx, float &qy, float &sds, int model = 0)
{
    const float s2 = fmaf(gx, gx, gy * gy);
    float mu1, mu3;
    MuData md{};
    if constexpr (GEN) {
        md = model_mu_data(s2 * inv_lam2, model);
        mu1 = md.mu1;
        mu3 = md.mu3;
    } else {
        mu1 = __builtin_amdgcn_rsqf(fmaf(s2, inv_lam2, 1.0f));
        mu3 = __builtin_amdgcn_sqrtf(mu1);
    }
    const float rn = __builtin_amdgcn_rsqf(fmaxf(s2, 1e-30f));
    const float s = s2 * rn;                   // |G| (0 when G = 0)
    const float nx = gx * rn, ny = gy * rn;
    const float a = nx * nx, b = ny * ny, c = nx * ny;
    const float amb = a - b, c2 = c + c;
    const float a1 = fmaf(a, axx, fmaf(b, ayy, c2 * axy));
    const float a3 = fmaf(c, ayy - axx, amb * axy);
    const float h1 = fmaf(a, hxx, fmaf(b, hyy, c2 * hxy));
    const float h3 = fmaf(c, hyy - hxx, amb * hxy);
    // D : A
    const float k1 = fmaf(mu1, a1, -a1);         // (mu1 - 1) a1
    const float k3 = fmaf(mu3, a3, -a3);         // (mu3 - 1) a3
    const float k3c2 = k3 * c2;
    txx = fmaf(k1, a, axx - k3c2);
    tyy = fmaf(k1, b, ayy + k3c2);
    txy = fmaf(k1, c, fmaf(k3, amb, axy));
    float de_ds, dth;
    if constexpr (GEN) {
        // with x = s^2/lambda^2: d mu/ds = 2 s/lambda^2 dmu/dx and
        // (mu - 1)/s = s/lambda^2 (mu - 1)/x
        const float Y = fmaf(md.G1, a1 * h1, 2.0f * md.G3 * (a3 * h3));
        de_ds = 2.0f * s * inv_lam2 * Y;
        const float at = fmaf(b, axx, fmaf(a, ayy, -c2 * axy));
        const float ht = fmaf(b, hxx, fmaf(a, hyy, -c2 * hxy));
        const float p1 = fmaf(a3, h1, a1 * h3);
        const float p2 = fmaf(at - a1, h3, a3 * (ht - h1));
        dth = 2.0f * s * inv_lam2 * fmaf(md.Q1, p1, md.Q3 * p2);
    } else {
        // derivatives: dmu1/ds = -s mu1^3 / lam^2, dmu3/ds = -s mu1^(5/2) / (2 lam^2)
        const float Fm = (s * inv_lam2) * (mu1 * mu1);            // s mu1^2 / lam^2
        de_ds = -Fm * fmaf(mu1, a1 * h1, mu3 * (a3 * h3));
        // (mu1 - 1)/s = -s mu1^2 / (lam^2 (1 + mu1)), (mu3 - 1)/s = that / (1 + mu3).
        // With a + b = 1 for the unit n, t.A.t - n.A.n = (axx + ayy) - 2 a1 and the same
        // for H; where G = 0 (n = 0) the factor Fm = 0 zeroes the whole term.
        const float rp = __builtin_amdgcn_rcpf(fmaf(-0.5f, mu1, -0.5f) * (1.0f + mu3));  // -2/(..)
        const float p1 = fmaf(a3, h1, a1 * h3);
        const float p2 = fmaf(fmaf(-2.0f, a1, axx + ayy), h3, a3 * fmaf(-2.0f, h1, hxx + hyy));
        dth = (Fm * rp) * fmaf(p1, 1.0f + mu3, p2);
    }
    qx = fmaf(nx, de_ds, -ny * dth);
    qy = fmaf(ny, de_ds, nx * dth);
    sds = s * de_ds;
}

// The workgroup's sum of v, on thread 0: a pairwise tree over the lanes of
// each wave, then over the four waves (FP32, fixed order: deterministic).
__device__ __forceinline__ float block_sum(float v, float *scratch)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) scratch[wv] = v;
    __syncthreads();
    return (scratch[0] + scratch[1]) + (scratch[2] + scratch[3]);
}

template <int R>
struct AdjAGeo {
    static constexpr int TW = kAdjTW, TH = kAdjTH;
    static constexpr int h = R + 2;
    static constexpr int UH = TH + 2 * h, UWr = TW + 2 * h, UW = (UWr + 3) & ~3;
    static constexpr int XW = TW + 4, VH = TH + 4;
    static constexpr int RH = TH + 4, RW = TW + 4;      // r with halo 2
    static constexpr int PH = TH + 2, PW = TW + 2, NP = PH * PW;
    static constexpr int NU = UH * UW, NX = UH * XW, NV = VH * XW, NR = RH * RW, NT = 3 * NP;
    static constexpr int REGA = (NU + NX > NT) ? NU + NX : NT;
    static constexpr int SMEM = REGA + NV + NR;
    static constexpr int NPT = (NP + kThreads - 1) / kThreads;
};

// Pass A on one 64 x 16 tile.  r = (mask ? 0 : abar_next) is formed on the fly.
template <int R>
__global__ __launch_bounds__(256) void adjoint_a_kernel(const float *u_all, const float *an_all,
                                                        const uint8_t *__restrict__ mask_all,
                                                        int H, int W, int nbx, int tiles_per_img,
                                                        StepArgs a, float lam_scale,
                                                        float *qx_all, float *qy_all,
                                                        float *pr_all, float *lam_partials,
                                                        int lam_stride)
{
    using G = AdjAGeo<R>;
    constexpr int TW = G::TW, TH = G::TH;
    __shared__ __attribute__((aligned(16))) float smem[G::SMEM];
    float *sU = smem, *sX = smem + G::NU, *sT = smem;
    float *sV = smem + G::REGA, *sR = sV + G::NV;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int bimg = tile / tiles_per_img, t = tile - bimg * tiles_per_img;
    const int ty = t / nbx, tx = t - ty * nbx;
    const size_t off = (size_t)bimg * H * W;
    const float *u = u_all + off, *an = an_all + off;
    const uint8_t *mask = mask_all + off;
    const int tid = threadIdx.x, gx0 = tx * TW, gy0 = ty * TH;
    if constexpr (kLdsSentinel) sentinel_fill_block(smem, G::SMEM);

    // ---- load u (halo R+2) and r (halo 2) ----
    for (int i = tid; i < G::UH * G::UWr; i += kThreads) {
        int r = i / G::UWr, c = i - r * G::UWr;
        int yy = mirror_index(gy0 - G::h + r, H), xx = mirror_index(gx0 - G::h + c, W);
        sU[r * G::UW + c] = u[(size_t)yy * W + xx];
    }
    for (int i = tid; i < G::NR; i += kThreads) {
        int r = i / G::RW, c = i - r * G::RW;
        int yy = mirror_index(gy0 - 2 + r, H), xx = mirror_index(gx0 - 2 + c, W);
        size_t gi = (size_t)yy * W + xx;
        sR[i] = mask[gi] ? 0.0f : an[gi];
    }
    __syncthreads();
    // ---- presmoothing: x pass then y pass (same layout as the forward tile) ----
    for (int i = tid; i < G::UH * G::XW; i += kThreads) {
        int r = i / G::XW, c = i - r * G::XW;
        const float *src = sU + r * G::UW + c;
        float s = a.w[0] * src[0];
#pragma unroll
        for (int j = 1; j <= 2 * R; ++j) s = fmaf(a.w[j], src[j], s);
        sX[r * G::XW + c] = s;
    }
    __syncthreads();
    for (int i = tid; i < G::VH * G::XW; i += kThreads) {
        int r = i / G::XW, c = i - r * G::XW;
        float s = a.w[0] * sX[r * G::XW + c];
#pragma unroll
        for (int j = 1; j <= 2 * R; ++j) s = fmaf(a.w[j], sX[(r + j) * G::XW + c], s);
        sV[r * G::XW + c] = s;
    }
    __syncthreads();

    // ---- per point: tensor applied to Hess(r); q and de/dlambda inside the tile ----
    float txx[G::NPT], tyy[G::NPT], txy[G::NPT];
    float dlsum = 0.0f;
#pragma unroll
    for (int k = 0; k < G::NPT; ++k) {
        int p = tid + k * kThreads;
        txx[k] = tyy[k] = txy[k] = 0.0f;
        if (p < G::NP) {
            int pr = p / G::PW, pc = p - pr * G::PW;
            const float *v = sV + (pr + 1) * G::XW + (pc + 1);
            float gx = 0.5f * (v[1] - v[-1]);
            float gy = 0.5f * (v[G::XW] - v[-G::XW]);
            const float *uu = sU + (pr + G::h - 1) * G::UW + (pc + G::h - 1);
            float uc = uu[0];
            float hxx = (uu[-1] - uc) + (uu[1] - uc);
            float hyy = (uu[-G::UW] - uc) + (uu[G::UW] - uc);
            float hxy = 0.25f * ((uu[G::UW + 1] + uu[-G::UW - 1]) - (uu[G::UW - 1] + uu[-G::UW + 1]));
            const float *rr = sR + (pr + 1) * G::RW + (pc + 1);
            float rc = rr[0];
            float axx = (rr[-1] - rc) + (rr[1] - rc);
            float ayy = (rr[-G::RW] - rc) + (rr[G::RW] - rc);
            float axy = 0.25f * ((rr[G::RW + 1] + rr[-G::RW - 1]) - (rr[G::RW - 1] + rr[-G::RW + 1]));
            float qx, qy, sds;
            adjoint_point(gx, gy, a.inv_lam2, axx, ayy, axy, hxx, hyy, hxy, txx[k], tyy[k], txy[k],
                          qx, qy, sds);
            int yy = gy0 + pr - 1, xx = gx0 + pc - 1;
            if (pr >= 1 && pr <= TH && pc >= 1 && pc <= TW && yy < H && xx < W) {
                size_t gi = off + (size_t)yy * W + xx;
                qx_all[gi] = qx;
                qy_all[gi] = qy;
                dlsum += sds;
            }
        }
    }
    __syncthreads();
    if constexpr (kLdsSentinel) sentinel_fill_block(sT, G::NT);
#pragma unroll
    for (int k = 0; k < G::NPT; ++k) {
        int p = tid + k * kThreads;
        if (p < G::NP) {
            sT[p] = txx[k];
            sT[G::NP + p] = tyy[k];
            sT[2 * G::NP + p] = txy[k];
        }
    }
    __syncthreads();
    // ---- outer differences: P(u) r ----
    const int c = tid % TW, r0 = tid / TW;
    for (int r = r0; r < TH; r += kThreads / TW) {
        int yy = gy0 + r, xx = gx0 + c;
        if (yy < H && xx < W) {
            int p = (r + 1) * G::PW + (c + 1);
            const float *Txx = sT + p, *Tyy = sT + G::NP + p, *Txy = sT + 2 * G::NP + p;
            float pu = ((Txx[-1] - Txx[0]) + (Txx[1] - Txx[0])) +
                       ((Tyy[-G::PW] - Tyy[0]) + (Tyy[G::PW] - Tyy[0])) +
                       0.5f * ((Txy[G::PW + 1] + Txy[-G::PW - 1]) - (Txy[G::PW - 1] + Txy[-G::PW + 1]));
            pr_all[off + (size_t)yy * W + xx] = pu;
        }
    }
    __syncthreads();
    const float tot = block_sum(dlsum, smem);
    if (threadIdx.x == 0) lam_partials[(size_t)bimg * lam_stride + t] = lam_scale * tot;
}

template <int R>
struct AdjBGeo {
    static constexpr int TW = kAdjTW, TH = kAdjTH;
    static constexpr int QH = TH + 2 * R + 2, QW = TW + 2 * R + 2;   // q with halo R+1
    static constexpr int DH = TH + 2 * R, DW = TW + 2 * R;           // -div q with halo R
    static constexpr int NQ = QH * QW, ND = DH * DW, NX = DH * TW;
    static constexpr int SMEM = 2 * NQ + ND + NX;
};

// q with the parity of a gradient component across the mirror borders.
__device__ __forceinline__ float load_q(const float *q, int y, int x, int H, int W, bool odd_x)
{
    int py = 2 * H, px = 2 * W;
    int my = y % py, mx = x % px;
    if (my < 0) my += py;
    if (mx < 0) mx += px;
    bool fy = my >= H, fx = mx >= W;
    int yy = fy ? py - 1 - my : my, xx = fx ? px - 1 - mx : mx;
    float v = q[(size_t)yy * W + xx];
    bool flip = odd_x ? fx : fy;
    return flip ? -v : v;
}

// Pass B on one 64 x 16 tile: C^T q and the pointwise reverse-step update.
template <int R>
__global__ __launch_bounds__(256) void adjoint_b_kernel(const float *qx_all, const float *qy_all,
                                                        const float *pr_all, const float *an_all,
                                                        float *ac_all, float *ap_all,
                                                        const uint8_t *__restrict__ mask_all,
                                                        int H, int W, int nbx,
                                                        int tiles_per_img, StepArgs a, int kflags)
{
    using G = AdjBGeo<R>;
    constexpr int TW = G::TW, TH = G::TH;
    __shared__ float smem[G::SMEM];
    float *sQx = smem, *sQy = smem + G::NQ, *sD = smem + 2 * G::NQ, *sX = sD + G::ND;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int bimg = tile / tiles_per_img, t = tile - bimg * tiles_per_img;
    const int ty = t / nbx, tx = t - ty * nbx;
    const size_t off = (size_t)bimg * H * W;
    const int tid = threadIdx.x, gx0 = tx * TW, gy0 = ty * TH;
    if constexpr (kLdsSentinel) sentinel_fill_block(smem, G::SMEM);

    for (int i = tid; i < G::NQ; i += kThreads) {
        int r = i / G::QW, c = i - r * G::QW;
        int yy = gy0 - R - 1 + r, xx = gx0 - R - 1 + c;
        sQx[i] = load_q(qx_all + off, yy, xx, H, W, true);
        sQy[i] = load_q(qy_all + off, yy, xx, H, W, false);
    }
    __syncthreads();
    // d = -div q = -(D_x q_x + D_y q_y) with central differences
    for (int i = tid; i < G::ND; i += kThreads) {
        int r = i / G::DW, c = i - r * G::DW;
        int p = (r + 1) * G::QW + (c + 1);
        sD[i] = -0.5f * ((sQx[p + 1] - sQx[p - 1]) + (sQy[p + G::QW] - sQy[p - G::QW]));
    }
    __syncthreads();
    for (int i = tid; i < G::NX; i += kThreads) {
        int r = i / TW, c = i - r * TW;
        const float *src = sD + r * G::DW + c;
        float s = a.w[0] * src[0];
#pragma unroll
        for (int j = 1; j <= 2 * R; ++j) s = fmaf(a.w[j], src[j], s);
        sX[i] = s;
    }
    __syncthreads();
    const int c = tid % TW, r0 = tid / TW;
    for (int r = r0; r < TH; r += kThreads / TW) {
        int yy = gy0 + r, xx = gx0 + c;
        if (yy >= H || xx >= W) continue;
        float cq = a.w[0] * sX[r * TW + c];
#pragma unroll
        for (int j = 1; j <= 2 * R; ++j) cq = fmaf(a.w[j], sX[(r + j) * TW + c], cq);
        size_t gi = off + (size_t)yy * W + xx;
        const float anv = an_all[gi];
        const bool m = mask_all[gi] != 0;
        const float rv = m ? 0.0f : anv;
        const float z = pr_all[gi] + cq;
        const float acold = (kflags & 2) ? 0.0f : ac_all[gi];  // a cycle's first reverse step
        float acv = fmaf(a.alpha, fmaf(-a.tau, z, rv), acold);
        const float back = (1.0f - a.alpha) * rv;
        if (kflags & 1) acv += back;
        else ap_all[gi] = back;
        if (m) acv += anv;              // known pixel: running sum of ubar
        ac_all[gi] = acv;
    }
}

// ---- fused reverse step on wave strips ----
//
// A wave owns 64 consecutive columns c = X0-2-R .. X0+61-R (one per lane) and
// streams down the rows of a segment.  For each stream row i it loads the
// presmoothed image v = K_sigma * u^k (kept by the forward recompute), u^k and
// r = mbar ubar^{k+1} of the row, then
//   S3  at row g = i-1: gradient of v, Hessians of u and of r (the last three
//       rows in registers, lane neighbours by DPP) and the adjoint point
//       quantities D:A, q, de/dlambda;
//   S4  at row g-1: P(u) r from the outer differences of D:A, and
//       d = -div q, whose x pass goes through a one-row LDS buffer into a
//       register window;
//   S5  at row o = i-R-2: y pass of d (C^T q) and the reverse update.
// Lanes R+2 .. 61-R own output columns (60-2R per wave).  The input halo is
// R+2 rows each way: R+1 for the y pass of d and one more for q.
template <int R, int ROWS>
struct AdjStripGeo {
    static constexpr int P = 2 * R + 1;                       // d window length
    static constexpr int U = P;                               // unroll (window slots constant)
    static constexpr int h = R + 2;                           // input row halo
    static constexpr int hc = R + 2;                          // first output lane
    static constexpr int SW = 64 - 2 * hc;                    // output columns per wave
    static constexpr int ND = 64 + 2 * R;                     // d row, R pad on each side
    static constexpr int M = (ROWS + 2 * h + U - 1) / U;      // main-loop iterations
    static constexpr int NROW = M * U;                        // rows streamed per wave
    static constexpr int OH = NROW - 2 * h;                   // output rows per wave
    static constexpr int LDS = ND + P * 64;                   // floats of LDS per wave
};

struct AdjStripArgs {
    const float *v, *u, *an;    // K_sigma * u^k, u^k, ubar^{k+1}
    float *ac, *ap;             // ubar^k (accumulated in place), ubar^{k-1} contribution
    const uint8_t *mask;
    int H, W, X0, Y0;
    float tau, alpha, il2;      // il2 = 1/lambda^2
    int first;                  // k == 0: the (1-alpha) r term goes to ubar^k itself
    int fresh;                  // k == n-1: ubar^k starts at 0 (not read)
    int model;                  // tensor variant (GEN kernels only)
    int prio;                   // lower the issue priority along the segment
};

// Global loads of one stream row: v, u^k and r of the row itself, and
// ubar^{k+1}, ubar^k and the mask of the output row it serves.
struct AdjStripRow {
    float v, u, rn, oa, oc;
    unsigned rmk, omk;
};

template <int R, int ROWS, bool GEN = false>
__device__ __forceinline__ void adjoint_strip_step(float *lds, const AdjStripArgs &s,
                                                   const float (&w)[2 * kRMax + 1],
                                                   float *partial, float lam_scale)
{
    using G = AdjStripGeo<R, ROWS>;
    constexpr int P = G::P, U = G::U, h = G::h;
    const int lane = threadIdx.x & 63;
    const int H = s.H, W = s.W;
    const unsigned W4 = 4u * (unsigned)W;
    if constexpr (kLdsSentinel) sentinel_fill_wave(lds, G::LDS);

    // resources based at the lowest row a needed value comes from (as in
    // the forward strip)
    const int ybase = s.Y0 - h;                               // image row of stream row 0
    const int b0 = ybase > 0 ? ybase : 0;
    const int nb = (H - b0 < G::NROW) ? H - b0 : G::NROW;
    const size_t base = (size_t)b0 * W;
    const __amdgpu_buffer_rsrc_t rs_v = buffer_rsrc(s.v + base, (unsigned)nb * W4);
    const __amdgpu_buffer_rsrc_t rs_u = buffer_rsrc(s.u + base, (unsigned)nb * W4);
    const __amdgpu_buffer_rsrc_t rs_an = buffer_rsrc(s.an + base, (unsigned)nb * W4);
    const __amdgpu_buffer_rsrc_t rs_ac = buffer_rsrc(s.ac + base, (unsigned)nb * W4);
    // ubar^k as read: no records in a cycle's first reverse step, where it
    // starts at 0 (its loads then read 0, and no clearing pass is needed)
    const __amdgpu_buffer_rsrc_t rs_acl = buffer_rsrc(s.ac + base, s.fresh ? 0u : (unsigned)nb * W4);
    // at k = 0 the (1 - alpha) r term stays in ubar^k: the ubar^{k-1} resource
    // then has no records, so its stores are dropped
    const __amdgpu_buffer_rsrc_t rs_ap = buffer_rsrc(s.ap + base, s.first ? 0u : (unsigned)nb * W4);
    const float keep_back = s.first ? 1.0f : 0.0f;
    const __amdgpu_buffer_rsrc_t rs_m = buffer_rsrc(s.mask + base, (unsigned)nb * (unsigned)W);

    const int cl = s.X0 - G::hc + lane;                       // this lane's column
    const unsigned cm = (unsigned)mirror_reflect(cl, W);      // ... mirrored into the image
    const bool out_lane = lane >= G::hc && lane < 64 - G::hc && cl < W;
    const unsigned vo4 = out_lane ? 4u * (unsigned)cl : kOffNone;
    const unsigned vo1 = out_lane ? (unsigned)cl : kOffNone;
    const int yend = s.Y0 + G::OH < H ? s.Y0 + G::OH : H;     // rows owned: [Y0, yend)

    // the d row (lane l at l + R), then P(u) r of the last P rows (slot j,
    // lane l at j * 64 + l): a slot is read R rows after it is written, and a
    // register window would cost more VGPRs than its P values
    float *dw = lds + lane;
    float *prr = lds + G::ND + lane;

    float dwin[P];                    // x-pass d; stream row j in slot j % P
#pragma unroll
    for (int j = 0; j < P; ++j) dwin[j] = 0.0f;
    float v_m1 = 0.0f, v_m2 = 0.0f;                          // v at rows g, g-1
    float u_m1 = 0.0f, u_m2 = 0.0f;                          // u at rows g, g-1
    float r_m1 = 0.0f, r_m2 = 0.0f;                          // r at rows g, g-1
    // lane-neighbour sums (row g) and differences (rows g, g-1) of u and r: each
    // row's two lane shifts are taken once, when it arrives
    float su_m1 = 0.0f, du_m1 = 0.0f, du_m2 = 0.0f;
    float sr_m1 = 0.0f, dr_m1 = 0.0f, dr_m2 = 0.0f;
    float txx_p = 0.0f, tyy_p = 0.0f, tyy_pp = 0.0f;         // D:A at rows g-1 (g-2 for yy)
    float z_p = 0.0f, z_pp = 0.0f;                           // (D:A)xy(l+1)-(D:A)xy(l-1)
    float qx_p = 0.0f, qy_p = 0.0f, qy_pp = 0.0f;            // q at rows g-1 (g-2 for y)
    float dsum = 0.0f;                                       // de/dlambda over the lane's rows

    RowTrack ty;                      // next prefetch: its mirrored image row
    ty.init(ybase, H);
    int on = ybase - h;                                       // output row it serves
    // ubar^{k+1} and the mask at output row o are those the stream read at its
    // row o, h rows earlier (same column on output lanes, no mirroring inside
    // the image).  Where the unrolled row block covers h + 1 rows (R >= 2) they
    // are kept in registers indexed by stream row % U instead of being loaded
    // again: by then the rows have left L2 (about 5 of the 22 bytes a pixel
    // otherwise fetches).
    constexpr bool OREG = U >= h + 1;
    constexpr int OQ = OREG ? U : 1;
    float rnq[OQ];
    unsigned rmq[OQ];
#pragma unroll
    for (int j = 0; j < OQ; ++j) {
        rnq[j] = 0.0f;
        rmq[j] = 0u;
    }
    auto prefetch = [&](AdjStripRow &r) {
        const unsigned sr = (unsigned)((ty.y > b0 ? ty.y : b0) - b0);
        r.v = buf_f32(rs_v, 4u * cm, sr * W4);
        r.u = buf_f32(rs_u, 4u * cm, sr * W4);
        r.rn = buf_f32(rs_an, 4u * cm, sr * W4);
        r.rmk = __builtin_amdgcn_raw_buffer_load_b8(rs_m, cm, sr * (unsigned)W, 0);
        int oc = on < b0 ? b0 : on;                           // clamped; unused rows are not stored
        oc = oc > H - 1 ? H - 1 : oc;
        const unsigned ro = (unsigned)(oc - b0);
        if constexpr (!OREG) {
            r.oa = buf_f32(rs_an, vo4, ro * W4);
            r.omk = __builtin_amdgcn_raw_buffer_load_b8(rs_m, vo1, ro * (unsigned)W, 0);
        }
        r.oc = buf_f32(rs_acl, vo4, ro * W4);
        ty.next(H);
        ++on;
    };
    AdjStripRow r0, r1;
    r0.oa = r1.oa = 0.0f;
    r0.omk = r1.omk = 0u;
    prefetch(r0);
    prefetch(r1);

#pragma unroll 1
    for (int it = 0; it < G::M; ++it) {
        // With every wave of the launch resident at once, waves further down
        // their segment yield issue slots to those behind, as in the forward
        // strip; when the launch needs more than one round of waves the host
        // leaves this off (late waves would then hold the top priority).  Only
        // the short segments, which small problems use, carry the code.  The
        // levels stay above 0, the level of the recompute steps that run beside
        // this kernel on the other stream, so these waves, the critical path,
        // issue first.
        if (ROWS <= 28 && s.prio) {
            const int left = G::M - it;
            if (left >= 3) __builtin_amdgcn_s_setprio(3);
            else if (left == 2) __builtin_amdgcn_s_setprio(2);
            else __builtin_amdgcn_s_setprio(1);
        }
#pragma unroll
        for (int ph = 0; ph < U; ++ph) {
            const int i = it * U + ph;                        // stream row (wave-uniform)
            const AdjStripRow cur = r0;
            r0 = r1;
            prefetch(r1);
            if constexpr (OREG) {
                rnq[ph] = cur.rn;                                    // stream row i % U = ph
                rmq[ph] = cur.rmk;
            }

            // ---- S3 at row g = i - 1 (rows g-1, g, g+1: m2, m1, this row) ----
            const float v_p1 = cur.v, u_p1 = cur.u;
            const float r_p1 = cur.rmk ? 0.0f : cur.rn;
            const float gxs = from_next_lane(v_m1) - from_prev_lane(v_m1);  // 2 gx
            const float gys = v_p1 - v_m2;                                   // 2 gy
            const float pu = from_prev_lane(u_p1), nu = from_next_lane(u_p1);
            const float pr_ = from_prev_lane(r_p1), nr = from_next_lane(r_p1);
            const float su_p1 = pu + nu, du_p1 = nu - pu;                    // row g+1
            const float sr_p1 = pr_ + nr, dr_p1 = nr - pr_;
            const float hxx = fmaf(-2.0f, u_m1, su_m1);
            const float hyy = fmaf(-2.0f, u_m1, u_m2 + u_p1);
            const float hxy = 0.25f * (du_p1 - du_m2);
            const float axx = fmaf(-2.0f, r_m1, sr_m1);
            const float ayy = fmaf(-2.0f, r_m1, r_m2 + r_p1);
            const float axy = 0.25f * (dr_p1 - dr_m2);
            v_m2 = v_m1;
            v_m1 = v_p1;
            u_m2 = u_m1;
            u_m1 = u_p1;
            r_m2 = r_m1;
            r_m1 = r_p1;
            su_m1 = su_p1;
            du_m2 = du_m1;
            du_m1 = du_p1;
            sr_m1 = sr_p1;
            dr_m2 = dr_m1;
            dr_m1 = dr_p1;
            float tx, ty_, txy, qx, qy, sds;
            adjoint_point<GEN>(0.5f * gxs, 0.5f * gys, s.il2, axx, ayy, axy, hxx, hyy, hxy, tx, ty_,
                               txy, qx, qy, sds, s.model);
            const int g = ybase + i - 1;                              // image row of S3
            dsum += (g >= s.Y0 && g < yend && out_lane) ? sds : 0.0f;
            const float z = from_next_lane(txy) - from_prev_lane(txy);

            // ---- S4 at row g - 1: P(u) r and d = -div q ----
            const float sxx = from_prev_lane(txx_p) + from_next_lane(txx_p);
            const float pr = fmaf(-2.0f, txx_p + tyy_p, sxx + (tyy_pp + ty_)) + 0.5f * (z - z_pp);
            const float d = -0.5f * ((from_next_lane(qx_p) - from_prev_lane(qx_p)) + (qy - qy_pp));
            dw[R] = d;
            wave_lds_sync();
            float dx = w[0] * dw[0];
#pragma unroll
            for (int j = 1; j <= 2 * R; ++j) dx = fmaf(w[j], dw[j], dx);
            const int jd = ((ph - 2) % P + P) % P;                    // slot of stream row i - 2
            dwin[jd] = dx;
            prr[jd * 64] = pr;
            tyy_pp = tyy_p;
            tyy_p = ty_;
            txx_p = tx;
            z_pp = z_p;
            z_p = z;
            qy_pp = qy_p;
            qy_p = qy;
            qx_p = qx;

            // ---- S5: output row o (stream row i - h) ----
            const int o = ybase + i - h;
            if (i >= 2 * h && o < H) {
                float cq = 0.0f;                                     // stream rows i-h-R .. i-2
#pragma unroll
                for (int j = 0; j <= 2 * R; ++j)
                    cq = fmaf(w[j], dwin[((ph - h - R + j) % P + P) % P], cq);
                const float pro = prr[((ph - h) % P + P) % P * 64];
                const int so = ((ph - h) % U + U) % U;              // stream row i - h
                const float anv = OREG ? rnq[so] : cur.oa;
                const bool mk = (OREG ? rmq[so] : cur.omk) != 0;
                const float rv = mk ? 0.0f : anv;
                float acv = fmaf(s.alpha, fmaf(-s.tau, pro + cq, rv), cur.oc);
                const float back = (1.0f - s.alpha) * rv;
                const unsigned ro = (unsigned)(o - b0) * W4;
                acv = fmaf(keep_back, back, acv);
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(back), rs_ap, vo4, ro, 0);
                if (mk) acv += anv;                                  // known pixel: running sum
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(acv), rs_ac, vo4, ro, 0);
            }
        }
    }
    // pairwise tree over the lanes; every lane stores lane 0's total (no
    // lane-dependent branch)
    for (int off = 32; off > 0; off >>= 1) dsum += __shfl_down(dsum, off, 64);
    const float tot = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dsum), 0));
    partial[0] = lam_scale * tot;
}

template <int R, int ROWS, bool GEN>
__device__ __forceinline__ void adjoint_strip_body(const float *v_all, const float *u_all,
                                                   const float *an_all,
                                                   float *ac_all, float *ap_all,
                                                   const uint8_t *__restrict__ mask_all, int H,
                                                   int W, int nstrip, int per_img, int nitems,
                                                   const StepArgs &a, float lam_scale,
                                                   int kflags, int prio, float *lam_partials,
                                                   int lam_stride)
{
    using G = AdjStripGeo<R, ROWS>;
    __shared__ float lds[4 * G::LDS];
    const int wave = threadIdx.x >> 6;
    const int item = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * 4 + wave);
    if (item >= nitems) return;  // whole wave; the kernel has no workgroup barrier
    const int b = item / per_img;
    const int r = item - b * per_img;
    const int seg = r / nstrip, strip = r - seg * nstrip;
    const size_t off = (size_t)b * H * W;
    AdjStripArgs s;
    s.v = v_all + off;
    s.u = u_all + off;
    s.an = an_all + off;
    s.ac = ac_all + off;
    s.ap = ap_all + off;
    s.mask = mask_all + off;
    s.H = H;
    s.W = W;
    s.X0 = strip * G::SW;
    s.Y0 = seg * G::OH;
    s.tau = a.tau;
    s.alpha = a.alpha;
    s.il2 = a.inv_lam2;
    s.first = kflags & 1;
    s.fresh = (kflags >> 1) & 1;
    s.model = a.model;
    s.prio = prio;
    adjoint_strip_step<R, ROWS, GEN>(lds + wave * G::LDS, s, a.w,
                                     lam_partials + (size_t)b * lam_stride + r, lam_scale);
}

template <int R, int ROWS>
__global__ __launch_bounds__(256) void adjoint_strip_kernel(const float *v_all, const float *u_all,
                                                            const float *an_all,
                                                            float *ac_all, float *ap_all,
                                                            const uint8_t *__restrict__ mask_all,
                                                            int H, int W, int nstrip, int per_img,
                                                            int nitems, StepArgs a,
                                                            float lam_scale, int kflags,
                                                            int prio, float *lam_partials,
                                                            int lam_stride)
{
    adjoint_strip_body<R, ROWS, false>(v_all, u_all, an_all, ac_all, ap_all, mask_all, H, W, nstrip,
                                       per_img, nitems, a, lam_scale, kflags, prio,
                                       lam_partials, lam_stride);
}

// The reverse step of the tensor variants (diffusivities of Table 7, mu3
// choices of Sec. 3.1) on strips of >= 28 rows.
template <int R>
__global__ __launch_bounds__(256) void adjoint_strip_model_kernel(
    const float *v_all, const float *u_all, const float *an_all, float *ac_all, float *ap_all,
    const uint8_t *__restrict__ mask_all, int H, int W, int nstrip, int per_img, int nitems,
    StepArgs a, float lam_scale, int kflags, int prio, float *lam_partials,
    int lam_stride)
{
    adjoint_strip_body<R, 28, true>(v_all, u_all, an_all, ac_all, ap_all, mask_all, H, W, nstrip,
                                    per_img, nitems, a, lam_scale, kflags, prio, lam_partials,
                                    lam_stride);
}

// ---- small helper kernels ----
__global__ __launch_bounds__(256) void fill_kernel(float *p, size_t n, float v)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// One pass of the pairwise lambda reduction: out[b][c] = the sum of the c-th
// run of 2048 values of image b's row of in (length L, zero-padded), by a
// pairwise tree in LDS.  Passes repeat until one value per image remains.
__global__ __launch_bounds__(1024) void pairwise_pass_kernel(const float *in, long long L,
                                                             float *out, int nout)
{
    __shared__ float sv[2048];
    const int c = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
    const float *p = in + (size_t)b * L + (size_t)c * 2048;
    const long long lim = L - (long long)c * 2048;
    sv[tid] = tid < lim ? p[tid] : 0.0f;
    sv[tid + 1024] = tid + 1024 < lim ? p[tid + 1024] : 0.0f;
    __syncthreads();
    for (int s = 1024; s > 0; s >>= 1) {
        if (tid < s) sv[tid] = sv[tid] + sv[tid + s];
        __syncthreads();
    }
    if (tid == 0) out[(size_t)b * nout + c] = sv[0];
}

// Cascade of the per-cycle sums over cycles (a pairwise tree built like a
// binary counter): slot i holds the sum of a block of 2^i cycles.  Adding the
// j-th cycle sum merges it with the t = (trailing ones of j) lowest slots and
// stores the block in slot t.
__device__ __forceinline__ void lambda_carry(float v, float *slots, int B, int b, int t)
{
    for (int i = 0; i < t; ++i) v = slots[(size_t)i * B + b] + v;
    slots[(size_t)t * B + b] = v;
}

__global__ void lambda_carry_kernel(const float *cyc, float *slots, int B, int t)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    lambda_carry(cyc[b], slots, B, b, t);
}

// Both of the above in one launch when a cycle's partials fit one pairwise
// pass (L <= 2048 per image): the same tree and the same cascade, so the same
// bits, with one launch per cycle instead of two.
__global__ __launch_bounds__(1024) void lambda_cycle_kernel(const float *in, long long L,
                                                            float *slots, int B, int t)
{
    __shared__ float sv[2048];
    const int b = blockIdx.x, tid = threadIdx.x;
    const float *p = in + (size_t)b * L;
    sv[tid] = tid < L ? p[tid] : 0.0f;
    sv[tid + 1024] = tid + 1024 < L ? p[tid + 1024] : 0.0f;
    __syncthreads();
    for (int s = 1024; s > 0; s >>= 1) {
        if (tid < s) sv[tid] = sv[tid] + sv[tid + s];
        __syncthreads();
    }
    if (tid == 0) lambda_carry(sv[0], slots, B, b, t);
}

// dL/dlambda = the occupied slots (the set bits of the cycle count M), largest
// block first.
__global__ void lambda_final_kernel(const float *slots, int B, unsigned M, float *out)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float v = 0.0f;
    bool any = false;
    for (int i = 31; i >= 0; --i)
        if ((M >> i) & 1u) {
            const float x = slots[(size_t)i * B + b];
            v = any ? v + x : x;
            any = true;
        }
    out[b] = v;
}

// On known pixels abar0 holds the sum of ubar over every state (ubar^{0,0}
// included): that is dL/df.  Elsewhere abar0 = ubar^{0,0} = dL/du_init.
__global__ __launch_bounds__(256) void adjoint_final_kernel(const float *abar0,
                                                            const uint8_t *__restrict__ mask,
                                                            float *gk, float *gi, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const float v = abar0[i];
        const bool m = mask[i] != 0;
        gk[i] = m ? v : 0.0f;
        gi[i] = m ? 0.0f : v;
    }
}

static unsigned grid_for(size_t n)
{
    size_t b = (n + 255) / 256;
    return (unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

static int adjoint_tiles_per_image(int H, int W)
{
    return ((W + kAdjTW - 1) / kAdjTW) * ((H + kAdjTH - 1) / kAdjTH);
}

template <int R, int ROWS>
static int adj_strip_items_t(int H, int W)
{
    using G = AdjStripGeo<R, ROWS>;
    return ((W + G::SW - 1) / G::SW) * ((H + G::OH - 1) / G::OH);
}

// Segment heights of the strip reverse step per forward strip shape.  The
// 64-row shapes map to segments of >= 80 rows: at 4096^2 and R = 6 those
// launch 4,042 waves, which all fit at once at 4 waves per SIMD (>= 64 rows
// launch 4,730, and the last 16 % ran as a second, nearly empty round).
template <int R>
static int adj_items_r(int shape, int H, int W)
{
    switch (shape) {
    case kShapeStrip:
    case kShapeStripWide: return adj_strip_items_t<R, 80>(H, W);
    case kShapeStripTall: return adj_strip_items_t<R, 136>(H, W);
    case kShapeStripShort:
    case kShapeStripWideShort: return adj_strip_items_t<R, 28>(H, W);
    case kShapeStripTiny: return adj_strip_items_t<R, 8>(H, W);
    default: return adjoint_tiles_per_image(H, W);
    }
}

#define EED4_RSWITCH(CALL)                                                          \
    switch (R) {                                                                    \
    case 0: return CALL(0); case 1: return CALL(1); case 2: return CALL(2);         \
    case 3: return CALL(3); case 4: return CALL(4); case 5: return CALL(5);         \
    case 6: return CALL(6); case 7: return CALL(7); case 8: return CALL(8);         \
    default: break;                                                                 \
    }

// Work items per image of a reverse step: tiles (every tile shape, one adjoint
// tile shape) or strip segments of the given height.
static int adjoint_items(int R, int shape, int H, int W)
{
#define EED4_CALL_N(r) adj_items_r<r>(shape, H, W)
    EED4_RSWITCH(EED4_CALL_N)
#undef EED4_CALL_N
    return 0;
}

static int max_adjoint_items(int R, int H, int W)
{
    int m = 0;
    for (int sh = 0; sh < kNumShapes; ++sh) m = std::max(m, adjoint_items(R, sh, H, W));
    return m;
}

// Buffers of one reverse step.
struct RevStep {
    const float *v;          // K_sigma * u^k (strip path only)
    const float *u, *an;     // u^k, ubar^{k+1}
    float *ac, *ap;          // ubar^k (in place), ubar^{k-1} contribution
    float *qx, *qy, *pr;     // tile path only
    const uint8_t *mask;
    float *lp;               // lambda partials of this step: image b, item r at lp[b * ls + r]
    int ls;                  // ... image stride (cycle_len * items per image)
    int B, H, W, R, shape, first;
    int fresh;               // a cycle's first reverse step: ubar^k starts at 0 (not read)
    int kflags() const { return (first ? 1 : 0) | (fresh ? 2 : 0); }
};

template <int R>
static hipError_t launch_rev_tile(const RevStep &t, const StepArgs &a, float ls,
                                  hipStream_t s)
{
    const int nbx = (t.W + kAdjTW - 1) / kAdjTW;
    const int tpi = adjoint_tiles_per_image(t.H, t.W);
    hipLaunchKernelGGL((adjoint_a_kernel<R>), dim3((unsigned)(tpi * t.B)), dim3(256), 0, s, t.u,
                       t.an, t.mask, t.H, t.W, nbx, tpi, a, ls, t.qx, t.qy, t.pr, t.lp,
                       t.ls);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((adjoint_b_kernel<R>), dim3((unsigned)(tpi * t.B)), dim3(256), 0, s, t.qx,
                       t.qy, t.pr, t.an, t.ac, t.ap, t.mask, t.H, t.W, nbx, tpi, a, t.kflags());
    return hipGetLastError();
}

// Waves of kernel k (256-thread workgroups) the current device holds at once;
// 0 if the runtime cannot tell.  The launchers keep the first answer (the
// devices of one node are alike); a wrong answer only switches the issue
// priority schedule on or off, never the results.
template <typename K>
static long long resident_waves(K k)
{
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, 0) != hipSuccess) return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return 4LL * per_cu * cus;
}

template <int R, int ROWS>
static hipError_t launch_rev_strip(const RevStep &t, const StepArgs &a, float ls,
                                   hipStream_t s)
{
    using G = AdjStripGeo<R, ROWS>;
    const int nstrip = (t.W + G::SW - 1) / G::SW;
    const int per_img = adj_strip_items_t<R, ROWS>(t.H, t.W);
    const long long nitems = (long long)per_img * t.B;
    if (nitems > (1LL << 31) - 4) return hipErrorInvalidValue;
    const unsigned nblk = (unsigned)((nitems + 3) / 4);
    // the issue-priority schedule only when every wave is resident at once
    static const long long cap = resident_waves(adjoint_strip_kernel<R, ROWS>);
    const int prio = nitems <= cap ? 1 : 0;
    hipLaunchKernelGGL((adjoint_strip_kernel<R, ROWS>), dim3(nblk), dim3(256), 0, s, t.v, t.u, t.an,
                       t.ac, t.ap, t.mask, t.H, t.W, nstrip, per_img, (int)nitems, a, ls,
                       t.kflags(), prio, t.lp, t.ls);
    return hipGetLastError();
}

template <int R>
static hipError_t launch_rev_model(const RevStep &t, const StepArgs &a, float ls,
                                   hipStream_t s)
{
    using G = AdjStripGeo<R, 28>;
    const int nstrip = (t.W + G::SW - 1) / G::SW;
    const int per_img = adj_strip_items_t<R, 28>(t.H, t.W);
    const long long nitems = (long long)per_img * t.B;
    if (nitems > (1LL << 31) - 4) return hipErrorInvalidValue;
    const unsigned nblk = (unsigned)((nitems + 3) / 4);
    static const long long cap = resident_waves(adjoint_strip_model_kernel<R>);
    const int prio = nitems <= cap ? 1 : 0;
    hipLaunchKernelGGL((adjoint_strip_model_kernel<R>), dim3(nblk), dim3(256), 0, s, t.v, t.u, t.an,
                       t.ac, t.ap, t.mask, t.H, t.W, nstrip, per_img, (int)nitems, a, ls,
                       t.kflags(), prio, t.lp, t.ls);
    return hipGetLastError();
}

template <int R>
static hipError_t launch_rev_r(const RevStep &t, const StepArgs &a, float ls,
                               hipStream_t s)
{
    // tensor variants: one kernel shape (strips of >= 28 rows)
    if (a.model != 0)
        return t.shape == kShapeStripShort ? launch_rev_model<R>(t, a, ls, s)
                                           : hipErrorInvalidValue;
    switch (t.shape) {
    case kShapeStrip:
    case kShapeStripWide: return launch_rev_strip<R, 80>(t, a, ls, s);
    case kShapeStripTall: return launch_rev_strip<R, 136>(t, a, ls, s);
    case kShapeStripShort:
    case kShapeStripWideShort: return launch_rev_strip<R, 28>(t, a, ls, s);
    case kShapeStripTiny: return launch_rev_strip<R, 8>(t, a, ls, s);
    default: return launch_rev_tile<R>(t, a, ls, s);
    }
}

// One reverse step k (alpha_k; the pixels' s de/ds sum to dL/dlambda with the
// scale alpha_k tau / lambda).
static hipError_t launch_reverse_step(const RevStep &t, const eed4_params *p, int k,
                                      hipStream_t s)
{
    const StepArgs a = make_args(p->sigma, t.R, p->tau, p->lambda, k, model_of_flags(p->flags));
    const float ls = (float)((double)a.alpha * a.tau / p->lambda);
    const int R = t.R;
#define EED4_CALL_REV(r) launch_rev_r<r>(t, a, ls, s)
    EED4_RSWITCH(EED4_CALL_REV)
#undef EED4_CALL_REV
    return hipErrorInvalidValue;
}
#undef EED4_RSWITCH

static hipError_t launch_fill(float *p, size_t n, float v, hipStream_t s)
{
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// Pairwise sum of each image's row of L values (in[b * L + i]) into out[b],
// through tmp1 / tmp2 (B * ceil(L / 2048) and B * ceil(L / 2048^2) floats).
static hipError_t launch_pairwise_sum(const float *in, long long L, int B, float *tmp1,
                                      float *tmp2, float *out, hipStream_t s)
{
    const float *src = in;
    float *bufs[2] = {tmp1, tmp2};
    int which = 0;
    for (;;) {
        const long long nout = (L + 2047) / 2048;
        float *dst = nout == 1 ? out : bufs[which];
        hipLaunchKernelGGL(pairwise_pass_kernel, dim3((unsigned)nout, (unsigned)B), dim3(1024), 0,
                           s, src, L, dst, (int)nout);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || nout == 1) return e;
        src = dst;
        L = nout;
        which ^= 1;
    }
}

static hipError_t launch_lambda_carry(const float *cyc, float *slots, int B, int t, hipStream_t s)
{
    hipLaunchKernelGGL(lambda_carry_kernel, dim3((B + 255) / 256), dim3(256), 0, s, cyc, slots, B,
                       t);
    return hipGetLastError();
}

static hipError_t launch_lambda_final(const float *slots, int B, int M, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(lambda_final_kernel, dim3((B + 255) / 256), dim3(256), 0, s, slots, B,
                       (unsigned)M, out);
    return hipGetLastError();
}

static hipError_t launch_adjoint_final(const float *abar0, const uint8_t *mask, float *gk,
                                       float *gi, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(adjoint_final_kernel, dim3(grid_for(n)), dim3(256), 0, s, abar0, mask, gk,
                       gi, n);
    return hipGetLastError();
}

// ---- workspace layout of eed4_backward ----
struct BackwardLayout {
    size_t U, V, an, ac, ap, qx, qy, pr, lp, t1, t2, cyc, slots, total;
};

static BackwardLayout backward_layout(int B, int H, int W, int n, int R)
{
    BackwardLayout L{};
    const size_t N = (size_t)B * H * W;
    size_t o = 0;
    // two sets of recompute buffers: cycle m-1 is recomputed while cycle m is reversed
    L.U = o; o = align_up(o + sizeof(float) * N * 2 * (size_t)(n > 1 ? n - 1 : 1));
    // ... and K_sigma * u^{m,k}, k = 0 .. n-1, for the strip reverse step
    L.V = o; o = align_up(o + sizeof(float) * N * 2 * (size_t)(n > 0 ? n : 1));
    L.an = o; o = align_up(o + sizeof(float) * N);
    L.ac = o; o = align_up(o + sizeof(float) * N);
    L.ap = o; o = align_up(o + sizeof(float) * N);
    L.qx = o; o = align_up(o + sizeof(float) * N);
    L.qy = o; o = align_up(o + sizeof(float) * N);
    L.pr = o; o = align_up(o + sizeof(float) * N);
    // lambda: one FP32 partial per work item and reverse step of a cycle, the
    // pairwise passes over them, the cycle sum and 32 cascade slots (per image)
    const size_t per_img = (size_t)(n > 0 ? n : 1) * (size_t)max_adjoint_items(R, H, W);
    const size_t n1 = (per_img + 2047) / 2048, n2 = (n1 + 2047) / 2048;
    L.lp = o; o = align_up(o + sizeof(float) * per_img * B);
    L.t1 = o; o = align_up(o + sizeof(float) * n1 * B);
    L.t2 = o; o = align_up(o + sizeof(float) * n2 * B);
    L.cyc = o; o = align_up(o + sizeof(float) * (size_t)B);
    L.slots = o; o = align_up(o + sizeof(float) * 32 * (size_t)B);
    L.total = o;
    return L;
}

size_t backward_workspace(int B, int H, int W, const eed4_params *p)
{
    const int R = eed4_radius(p->sigma);
    return R < 0 ? 0 : backward_layout(B, H, W, p->cycle_len, R).total;
}

static std::string adjoint_tune_key(int R, int B, int H, int W)
{
    char buf[96];
    std::snprintf(buf, sizeof(buf), "adjoint_R%d_B%d_H%d_W%d", R, B, H, W);
    return buf;
}

// Reverse-step implementation: a forced shape (tile shapes select the tile
// passes, strip shapes the strip kernel of that height; the reverse strip
// has one column per lane), else the tuned
// choice for this problem size, else the timing of one reverse step of each
// on the caller's data (t holds real buffers; what it writes is scratch).
static int adjoint_shape(const eed4_params *p, RevStep t, hipStream_t s, int *shape)
{
    TraceRange range("eed4 reverse-step shape %dx%dx%d", t.B, t.H, t.W);
    if (model_of_flags(p->flags) != 0) { *shape = kShapeStripShort; return EED4_OK; }
    const int forced = (p->flags >> 8) & 0xff;
    if (forced >= 1 && forced <= kNumShapes) { *shape = forced - 1; return EED4_OK; }
    if (p->flags & EED4_TILE_KERNEL) { *shape = 0; return EED4_OK; }
    const std::string key = adjoint_tune_key(t.R, t.B, t.H, t.W);
    if (tune_lookup(key, shape)) return EED4_OK;
    // the wide forward shapes map onto the same reverse strips as their heights
    const int cands[] = {kShapeStrip, 0, kShapeStripTall, kShapeStripShort, kShapeStripTiny};
    const size_t N = (size_t)t.B * t.H * t.W;
    // the strip candidates read the presmoothed state t.v
    const StepArgs a0 = make_args(p->sigma, t.R, p->tau, p->lambda, 0, model_of_flags(p->flags));
    hipError_t e = launch_blur(t.R, t.u, const_cast<float *>(t.v), t.B, t.H, t.W, a0, s);
    if (e == hipSuccess) e = launch_fill(t.ac, N, 0.0f, s);
    if (e != hipSuccess) return hip_fail(e, "adjoint autotune");
    int best = cands[0];
    const int rc = tune_pick(
        cands, (int)(sizeof(cands) / sizeof(cands[0])), s,
        [&](int c) {
            t.shape = c;
            t.first = 0;
            t.fresh = 0;                       // ac was cleared above
            return (int)EED4_OK;
        },
        [&](int) { return launch_reverse_step(t, p, p->cycle_len - 1, s); }, "adjoint autotune",
        &best, nullptr);
    if (rc != EED4_OK) return rc;
    tune_remember(key, best);
    *shape = best;
    return EED4_OK;
}

}  // namespace eed4

using namespace eed4;

extern "C" int eed4_backward(const float *ckpt, const uint8_t *mask, const float *known, int B,
                             int H, int W, const eed4_params *p, int M, const float *grad_u,
                             float *grad_known, float *grad_init, float *grad_lambda, void *ws,
                             size_t ws_bytes, void *stream)
{
    TraceRange range("eed4_backward %dx%dx%d, %d cycles of %d", B, H, W, M, p ? p->cycle_len : 0);
    int rc = check_params(p, B, H, W);
    if (rc != EED4_OK) return rc;
    if (!ckpt || !mask || !known || !grad_u || !grad_known || !grad_init || !grad_lambda || M < 1)
        return EED4_EINVAL;
    const int n = p->cycle_len, R = eed4_radius(p->sigma);
    BackwardLayout L = backward_layout(B, H, W, n, R);
    if ((rc = check_ws(ws, ws_bytes, L.total)) != EED4_OK) return rc;
    char *base = (char *)ws;
    hipStream_t s = (hipStream_t)stream;
    const size_t N = (size_t)B * H * W;
    float *Ubuf = (float *)(base + L.U);
    float *lp = (float *)(base + L.lp), *cyc = (float *)(base + L.cyc);
    float *slots = (float *)(base + L.slots);
    RevStep t{};
    t.an = (float *)(base + L.an);
    t.ac = (float *)(base + L.ac);
    t.ap = (float *)(base + L.ap);
    t.qx = (float *)(base + L.qx);
    t.qy = (float *)(base + L.qy);
    t.pr = (float *)(base + L.pr);
    t.mask = mask;
    t.lp = lp;
    t.ls = n * max_adjoint_items(R, H, W);     // the tuner's steps below write within this
    t.B = B;
    t.H = H;
    t.W = W;
    t.R = R;
    const int fshape = step_shape(p, B, H, W);      // forward recompute
    hipError_t e;
#define EED4_TRY(x, what)                                    \
    do {                                                     \
        e = (x);                                             \
        if (e != hipSuccess) return hip_fail(e, what);       \
    } while (0)

    float *Vbuf = (float *)(base + L.V);
    {   // choose the reverse-step kernel (the timing runs write only scratch)
        RevStep probe = t;
        probe.u = ckpt + (size_t)(M - 1) * N;
        probe.an = grad_u;
        probe.v = Vbuf;
        if ((rc = adjoint_shape(p, probe, s, &t.shape)) != EED4_OK) return rc;
    }
    const bool keep_v = is_strip(t.shape);      // the strip reverse step reads K_sigma * u^k
    const int items = adjoint_items(R, t.shape, H, W);
    t.ls = n * items;
    EED4_TRY(hipMemcpyAsync((void *)t.an, grad_u, sizeof(float) * N, hipMemcpyDeviceToDevice, s),
             "seed copy");

    // The recompute of cycle m-1 (from its checkpoint) does not depend on the
    // reverse sweep of cycle m: it runs on a second stream into the other
    // buffer set.  rec[j] marks set j recomputed, done[j] marks the reverse
    // sweep that read set j finished (a stream wait takes the event's latest
    // record at the time of the call, so two of each suffice).
    hipStream_t s1 = recompute_stream();
    if (!s1) return hip_fail(hipErrorInvalidValue, "recompute stream");
    hipEvent_t ev[5] = {};
    for (auto &x : ev) {
        e = hipEventCreateWithFlags(&x, hipEventDisableTiming);
        if (e != hipSuccess) {
            for (auto &y : ev) if (y) (void)hipEventDestroy(y);
            return hip_fail(e, "event");
        }
    }
    hipEvent_t *rec = ev, *done = ev + 2, start = ev[4];
    const size_t nU = (size_t)(n > 1 ? n - 1 : 1);
    float *Uset[2] = {Ubuf, Ubuf + nU * N};
    float *Vset[2] = {Vbuf, Vbuf + (size_t)n * N};
    std::vector<const float *> Ur[2] = {std::vector<const float *>(n), std::vector<const float *>(n)};
    // u^{m,1..n-1} from the checkpoint, on s1, and (strip reverse step) v^{m,k} =
    // K_sigma * u^{m,k} for k = 0 .. n-1: the steps keep the v they compute, and
    // the last one, which no recomputed step forms, comes from the blur kernel
    auto recompute = [&](int m) -> hipError_t {
        trace_mark("eed4 recompute of cycle %d queued", m);
        std::vector<const float *> &U = Ur[m & 1];
        float *V = Vset[m & 1];
        U[0] = ckpt + (size_t)m * N;
        for (int k = 0; k + 1 < n; ++k) {
            float *out = Uset[m & 1] + (size_t)k * N;
            StepArgs a = make_args(p->sigma, R, p->tau, p->lambda, k, model_of_flags(p->flags));
            hipError_t r = keep_v
                ? launch_step_keepv(R, fshape, U[k], U[k > 0 ? k - 1 : 0], out, V + (size_t)k * N,
                                    mask, B, H, W, a, s1)
                : launch_step(R, fshape, U[k], U[k > 0 ? k - 1 : 0], out, nullptr, mask, B, H, W,
                              a, nullptr, s1);
            if (r != hipSuccess) return r;
            U[k + 1] = out;
        }
        if (keep_v) {
            const StepArgs a = make_args(p->sigma, R, p->tau, p->lambda, 0, model_of_flags(p->flags));
            hipError_t r = launch_blur(R, U[n - 1], V + (size_t)(n - 1) * N, B, H, W, a, s1);
            if (r != hipSuccess) return r;
        }
        return hipEventRecord(rec[m & 1], s1);
    };
    float *an = (float *)t.an, *ac = t.ac, *ap = t.ap;
    int rc2 = EED4_OK;
#define EED4_TRY2(x, what)                                                  \
    if (rc2 == EED4_OK && (e = (x)) != hipSuccess) rc2 = hip_fail(e, what)
    EED4_TRY2(hipEventRecord(start, s), "event record");      // the seed and the checkpoints
    EED4_TRY2(hipStreamWaitEvent(s1, start, 0), "stream wait");
    EED4_TRY2(recompute(M - 1), "recompute step");
    for (int m = M - 1; m >= 0 && rc2 == EED4_OK; --m) {
        trace_mark("eed4 reverse sweep of cycle %d queued", m);
        EED4_TRY2(hipStreamWaitEvent(s, rec[m & 1], 0), "stream wait");
        if (m >= 1) {
            // set (m-1) & 1 was last read by the reverse sweep of cycle m+1
            if (m + 1 <= M - 1) EED4_TRY2(hipStreamWaitEvent(s1, done[(m + 1) & 1], 0), "stream wait");
            EED4_TRY2(recompute(m - 1), "recompute step");
        }
        const std::vector<const float *> &U = Ur[m & 1];
        for (int k = n - 1; k >= 0 && rc2 == EED4_OK; --k) {
            t.u = U[k];
            t.v = Vset[m & 1] + (size_t)k * N;
            t.an = an;
            t.ac = ac;
            t.ap = ap;
            t.first = k == 0 ? 1 : 0;
            t.fresh = k == n - 1 ? 1 : 0;          // ubar^{n-1} starts at 0
            t.lp = lp + (size_t)k * items;
            EED4_TRY2(launch_reverse_step(t, p, k, s), "reverse step");
            // ubar^k is complete in ac; ap holds the start of ubar^{k-1}
            float *tmp = an;
            an = ac;
            ac = ap;
            ap = tmp;
        }
        EED4_TRY2(hipEventRecord(done[m & 1], s), "event record");
        // this cycle's lambda partials: pairwise sum per image, then into the cascade
        const int j = M - 1 - m;                              // cycles summed before this one
        int carries = 0;
        while ((j >> carries) & 1) ++carries;
        const long long np = (long long)n * items;
        if (np <= 2048) {
            hipLaunchKernelGGL(lambda_cycle_kernel, dim3(B), dim3(1024), 0, s, lp, np, slots, B,
                               carries);
            EED4_TRY2(hipGetLastError(), "lambda sum");
        } else {
            EED4_TRY2(launch_pairwise_sum(lp, np, B, (float *)(base + L.t1),
                                          (float *)(base + L.t2), cyc, s), "lambda sum");
            EED4_TRY2(launch_lambda_carry(cyc, slots, B, carries, s), "lambda cascade");
        }
    }
#undef EED4_TRY2
    // on an error the recompute stream may still hold queued work on the
    // caller's workspace: let it finish before the caller can free it
    if (rc2 != EED4_OK) (void)hipStreamSynchronize(s1);
    for (auto &x : ev) (void)hipEventDestroy(x);
    if (rc2 != EED4_OK) return rc2;
    EED4_TRY(launch_adjoint_final(an, mask, grad_known, grad_init, N, s), "final");
    EED4_TRY(launch_lambda_final(slots, B, M, grad_lambda, s), "lambda final");
#undef EED4_TRY
    return EED4_OK;
}
