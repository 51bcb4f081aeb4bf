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
// Pass A computes P(u) r, q and de/dlambda; pass B applies
// C^T q = K_sigma (-div q) and the pointwise update.  Both evaluate on the
// mirror-extended image: q_x is odd across vertical borders and even across
// horizontal ones, q_y the reverse, which makes every transpose exact.
#include "eed4.h"
#include "eed4_host.h"
#include "eed4_internal.h"
#include "eed4_tile.h"

#include <cmath>
#include <vector>

namespace eed4 {

constexpr int kAdjTW = 64, kAdjTH = 16;

// Per-point pieces of the adjoint.  (gx, gy) = G = grad u_sigma; A = Hessian
// of r, H = Hessian of u.  Outputs: D(G) : A, q = de/dG and de/dlambda with
// e = A : D(G) : H.  In the gradient frame n = G/|G|, t = n rotated by +90
// degrees, e = A:H + (mu1 - 1) a1 h1 + 2 (mu3 - 1) a3 h3 with a1 = n.A.n,
// a3 = t.A.n; d/ds and d/dtheta of it give q = (de/ds) n + (1/s)(de/dtheta) t.
__device__ __forceinline__ void adjoint_point(float gx, float gy, float lam, float inv_lam2,
                                              float axx, float ayy, float axy, float hxx,
                                              float hyy, float hxy, float &txx, float &tyy,
                                              float &txy, float &qx, float &qy, float &dl)
{
    const float s2 = fmaf(gx, gx, gy * gy);
    const float mu1 = __builtin_amdgcn_rsqf(fmaf(s2, inv_lam2, 1.0f));
    const float mu3 = __builtin_amdgcn_sqrtf(mu1);
    const float rn = __builtin_amdgcn_rsqf(fmaxf(s2, 1e-30f));
    const float s = s2 * rn;                   // |G| (0 when G = 0)
    const float nx = gx * rn, ny = gy * rn;
    const float a = nx * nx, b = ny * ny, c = nx * ny;
    const float amb = a - b, c2 = c + c;
    const float a1 = fmaf(a, axx, fmaf(b, ayy, c2 * axy));
    const float a3 = fmaf(c, ayy - axx, amb * axy);
    const float at = fmaf(b, axx, fmaf(a, ayy, -c2 * axy));
    const float h1 = fmaf(a, hxx, fmaf(b, hyy, c2 * hxy));
    const float h3 = fmaf(c, hyy - hxx, amb * hxy);
    const float ht = fmaf(b, hxx, fmaf(a, hyy, -c2 * hxy));
    // D : A
    const float k1 = (mu1 - 1.0f) * a1;
    const float k3 = (mu3 - 1.0f) * a3;
    const float k3c2 = k3 * c2;
    txx = fmaf(k1, a, axx - k3c2);
    tyy = fmaf(k1, b, ayy + k3c2);
    txy = fmaf(k1, c, fmaf(k3, amb, axy));
    // derivatives: dmu1/ds = -s mu1^3 / lam^2, dmu3/ds = -s mu1^(5/2) / (2 lam^2)
    const float m12 = mu1 * mu1;
    const float X = fmaf(m12 * mu1, a1 * h1, m12 * mu3 * (a3 * h3));
    const float de_ds = -s * inv_lam2 * X;
    dl = (s2 * inv_lam2 / lam) * X;
    // (mu1 - 1)/s = -s mu1^2 / (lam^2 (1 + mu1)), (mu3 - 1)/s = that / (1 + mu3)
    const float rp = __builtin_amdgcn_rcpf((1.0f + mu1) * (1.0f + mu3));
    const float p1 = fmaf(a3, h1, a1 * h3);
    const float p2 = fmaf(at - a1, h3, a3 * (ht - h1));
    const float dth = -2.0f * s * m12 * inv_lam2 * rp * fmaf(p1, 1.0f + mu3, p2);
    qx = fmaf(nx, de_ds, -ny * dth);
    qy = fmaf(ny, de_ds, nx * dth);
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
                                                        StepArgs a, float lam, float lam_scale,
                                                        float *qx_all, float *qy_all,
                                                        float *pr_all, double *lam_partials)
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
    double dlsum = 0.0;
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
            float qx, qy, dl;
            adjoint_point(gx, gy, lam, a.inv_lam2, axx, ayy, axy, hxx, hyy, hxy, txx[k], tyy[k],
                          txy[k], qx, qy, dl);
            int yy = gy0 + pr - 1, xx = gx0 + pc - 1;
            if (pr >= 1 && pr <= TH && pc >= 1 && pc <= TW && yy < H && xx < W) {
                size_t gi = off + (size_t)yy * W + xx;
                qx_all[gi] = qx;
                qy_all[gi] = qy;
                dlsum += (double)dl;
            }
        }
    }
    __syncthreads();
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
    block_sum2(dlsum * (double)lam_scale, 0.0, reinterpret_cast<double *>(smem),
               lam_partials + 2 * (size_t)tile);
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
                                                        const float *pr_all, float *an_all,
                                                        float *ac_all,
                                                        const uint8_t *__restrict__ mask_all,
                                                        float *gk_all, int H, int W, int nbx,
                                                        int tiles_per_img, StepArgs a, int first)
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
        float acv = fmaf(a.alpha, fmaf(-a.tau, z, rv), ac_all[gi]);
        const float back = (1.0f - a.alpha) * rv;
        if (first) acv += back;
        ac_all[gi] = acv;
        if (!first) an_all[gi] = back;
        if (m) gk_all[gi] += anv;
    }
}

// ---- small helper kernels ----
__global__ __launch_bounds__(256) void fill_kernel(float *p, size_t n, float v)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ __launch_bounds__(256) void fill_double_kernel(double *p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// acc[b] += fixed-order sum of image b's tile partials (first double of each)
__global__ __launch_bounds__(256) void lambda_reduce_kernel(const double *partials,
                                                            int tiles_per_img, double *acc)
{
    __shared__ double sd[256];
    const int b = blockIdx.x;
    const double *p = partials + 2 * (size_t)b * tiles_per_img;
    double d = 0.0;
    for (int i = threadIdx.x; i < tiles_per_img; i += 256) d += p[2 * i];
    sd[threadIdx.x] = d;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sd[threadIdx.x] += sd[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) acc[b] += sd[0];
}

__global__ void lambda_store_kernel(const double *acc, float *out, int B)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) out[b] = (float)acc[b];
}

// fbar += m * ubar^{0,0}; dL/du_init = mbar * ubar^{0,0}
__global__ __launch_bounds__(256) void adjoint_final_kernel(const float *abar0,
                                                            const uint8_t *__restrict__ mask,
                                                            float *gk, float *gi, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        if (mask[i]) {
            gk[i] += abar0[i];
            gi[i] = 0.0f;
        } else {
            gi[i] = abar0[i];
        }
    }
}

static unsigned grid_for(size_t n)
{
    size_t b = (n + 255) / 256;
    return (unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

int adjoint_tiles_per_image(int H, int W)
{
    return ((W + kAdjTW - 1) / kAdjTW) * ((H + kAdjTH - 1) / kAdjTH);
}

template <int R>
static hipError_t launch_a_t(const float *u, const float *an, const uint8_t *mask, int B, int H,
                             int W, const StepArgs &a, float lam, float lam_scale, float *qx,
                             float *qy, float *pr, double *lp, hipStream_t s)
{
    const int nbx = (W + kAdjTW - 1) / kAdjTW;
    const int tpi = adjoint_tiles_per_image(H, W);
    hipLaunchKernelGGL((adjoint_a_kernel<R>), dim3((unsigned)(tpi * B)), dim3(256), 0, s, u, an,
                       mask, H, W, nbx, tpi, a, lam, lam_scale, qx, qy, pr, lp);
    return hipGetLastError();
}

template <int R>
static hipError_t launch_b_t(const float *qx, const float *qy, const float *pr, float *an,
                             float *ac, const uint8_t *mask, float *gk, int B, int H, int W,
                             const StepArgs &a, int first, hipStream_t s)
{
    const int nbx = (W + kAdjTW - 1) / kAdjTW;
    const int tpi = adjoint_tiles_per_image(H, W);
    hipLaunchKernelGGL((adjoint_b_kernel<R>), dim3((unsigned)(tpi * B)), dim3(256), 0, s, qx, qy,
                       pr, an, ac, mask, gk, H, W, nbx, tpi, a, first);
    return hipGetLastError();
}

#define EED4_RSWITCH(CALL)                                                          \
    switch (R) {                                                                    \
    case 0: return CALL(0); case 1: return CALL(1); case 2: return CALL(2);         \
    case 3: return CALL(3); case 4: return CALL(4); case 5: return CALL(5);         \
    case 6: return CALL(6); case 7: return CALL(7); case 8: return CALL(8);         \
    default: return hipErrorInvalidValue;                                           \
    }

hipError_t launch_adjoint_a(int R, const float *u, const float *an, const uint8_t *mask, int B,
                            int H, int W, const StepArgs &a, float lam, float lam_scale,
                            float *qx, float *qy, float *pr, double *lp, hipStream_t s)
{
#define EED4_CALL_A(r) launch_a_t<r>(u, an, mask, B, H, W, a, lam, lam_scale, qx, qy, pr, lp, s)
    EED4_RSWITCH(EED4_CALL_A)
#undef EED4_CALL_A
}

hipError_t launch_adjoint_b(int R, const float *qx, const float *qy, const float *pr, float *an,
                            float *ac, const uint8_t *mask, float *gk, int B, int H, int W,
                            const StepArgs &a, int first, hipStream_t s)
{
#define EED4_CALL_B(r) launch_b_t<r>(qx, qy, pr, an, ac, mask, gk, B, H, W, a, first, s)
    EED4_RSWITCH(EED4_CALL_B)
#undef EED4_CALL_B
}

hipError_t launch_fill(float *p, size_t n, float v, hipStream_t s)
{
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_double(double *p, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(fill_double_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_lambda_reduce(const double *lp, int tiles_per_img, int B, double *acc,
                                hipStream_t s)
{
    hipLaunchKernelGGL(lambda_reduce_kernel, dim3(B), dim3(256), 0, s, lp, tiles_per_img, acc);
    return hipGetLastError();
}

hipError_t launch_lambda_store(const double *acc, float *out, int B, hipStream_t s)
{
    hipLaunchKernelGGL(lambda_store_kernel, dim3((B + 255) / 256), dim3(256), 0, s, acc, out, B);
    return hipGetLastError();
}

hipError_t launch_adjoint_final(const float *abar0, const uint8_t *mask, float *gk, float *gi,
                                size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(adjoint_final_kernel, dim3(grid_for(n)), dim3(256), 0, s, abar0, mask, gk,
                       gi, n);
    return hipGetLastError();
}

// ---- workspace layout of eed4_backward ----
struct BackwardLayout {
    size_t U, an, ac, qx, qy, pr, lp, acc, total;
};

static BackwardLayout backward_layout(int B, int H, int W, int n)
{
    BackwardLayout L{};
    const size_t N = (size_t)B * H * W;
    const size_t tiles = (size_t)adjoint_tiles_per_image(H, W) * B;
    size_t o = 0;
    L.U = o; o = align_up(o + sizeof(float) * N * (size_t)(n > 1 ? n - 1 : 1));
    L.an = o; o = align_up(o + sizeof(float) * N);
    L.ac = o; o = align_up(o + sizeof(float) * N);
    L.qx = o; o = align_up(o + sizeof(float) * N);
    L.qy = o; o = align_up(o + sizeof(float) * N);
    L.pr = o; o = align_up(o + sizeof(float) * N);
    L.lp = o; o = align_up(o + sizeof(double) * 2 * tiles);
    L.acc = o; o = align_up(o + sizeof(double) * (size_t)B);
    L.total = o;
    return L;
}

size_t backward_workspace(int B, int H, int W, const eed4_params *p)
{
    return backward_layout(B, H, W, p->cycle_len).total;
}

}  // namespace eed4

using namespace eed4;

extern "C" int eed4_backward(const float *ckpt, const uint8_t *mask, const float *known, int B,
                             int H, int W, const eed4_params *p, int M, const float *grad_u,
                             float *grad_known, float *grad_init, float *grad_lambda, void *ws,
                             size_t ws_bytes, void *stream)
{
    int rc = check_params(p, B, H, W);
    if (rc != EED4_OK) return rc;
    if (!ckpt || !mask || !known || !grad_u || !grad_known || !grad_init || !grad_lambda || M < 1)
        return EED4_EINVAL;
    const int n = p->cycle_len, R = eed4_radius(p->sigma);
    BackwardLayout L = backward_layout(B, H, W, n);
    if ((rc = check_ws(ws, ws_bytes, L.total)) != EED4_OK) return rc;
    char *base = (char *)ws;
    hipStream_t s = (hipStream_t)stream;
    const size_t N = (size_t)B * H * W;
    float *Ubuf = (float *)(base + L.U);
    float *an = (float *)(base + L.an), *ac = (float *)(base + L.ac);
    float *qx = (float *)(base + L.qx), *qy = (float *)(base + L.qy), *pr = (float *)(base + L.pr);
    double *lp = (double *)(base + L.lp), *acc = (double *)(base + L.acc);
    const int tpi = adjoint_tiles_per_image(H, W);
    const int shape = step_shape(p, B, H, W);
    hipError_t e;
#define EED4_TRY(x, what)                                    \
    do {                                                     \
        e = (x);                                             \
        if (e != hipSuccess) return hip_fail(e, what);       \
    } while (0)

    EED4_TRY(launch_fill(grad_known, N, 0.0f, s), "fill");
    EED4_TRY(launch_fill_double(acc, (size_t)B, s), "fill");
    EED4_TRY(hipMemcpyAsync(an, grad_u, sizeof(float) * N, hipMemcpyDeviceToDevice, s), "seed copy");
    std::vector<const float *> U(n);
    for (int m = M - 1; m >= 0; --m) {
        // recompute u^{m,1..n-1} from the checkpoint
        U[0] = ckpt + (size_t)m * N;
        for (int k = 0; k + 1 < n; ++k) {
            float *out = Ubuf + (size_t)k * N;
            StepArgs a = make_args(p->sigma, R, p->tau, p->lambda, k);
            EED4_TRY(launch_step(R, shape, U[k], U[k > 0 ? k - 1 : 0], out, nullptr, mask, B, H,
                                 W, a, nullptr, s),
                     "recompute step");
            U[k + 1] = out;
        }
        EED4_TRY(launch_fill(ac, N, 0.0f, s), "fill");
        for (int k = n - 1; k >= 0; --k) {
            StepArgs a = make_args(p->sigma, R, p->tau, p->lambda, k);
            const float lam_scale = -a.alpha * a.tau;
            EED4_TRY(launch_adjoint_a(R, U[k], an, mask, B, H, W, a, p->lambda, lam_scale, qx, qy,
                                      pr, lp, s),
                     "adjoint pass A");
            EED4_TRY(launch_lambda_reduce(lp, tpi, B, acc, s), "lambda reduce");
            EED4_TRY(launch_adjoint_b(R, qx, qy, pr, an, ac, mask, grad_known, B, H, W, a,
                                      k == 0 ? 1 : 0, s),
                     "adjoint pass B");
            float *t = an;
            an = ac;
            ac = t;
        }
    }
    EED4_TRY(launch_adjoint_final(an, mask, grad_known, grad_init, N, s), "final");
    EED4_TRY(launch_lambda_store(acc, grad_lambda, B, s), "lambda store");
#undef EED4_TRY
    return EED4_OK;
}
