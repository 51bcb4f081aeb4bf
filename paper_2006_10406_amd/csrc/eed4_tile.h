// Device code of one fused FOEED/FSI inner step on one output tile.
//
// One workgroup of NTH threads (256 unless given) computes a TW x TH tile of u^{k+1} from u^k
// (read with a halo of R+2 pixels, R = Gaussian radius) and u^{k-1}:
//   A  load u^k (tile + halo) into LDS; border tiles gather through the
//      half-sample mirror, which realises the Neumann condition (Sec. 2.1)
//   B  x pass of the separable Gaussian presmoothing (Sec. 2.2)
//   C  y pass
//   D  at every point of the tile grown by one pixel: central-difference
//      gradient of u_sigma, fourth-order diffusion tensor from it (Sec. 3.1,
//      eigenvalues g, 1, sqrt g, 0), Hessian of u (Sec. 3.3 stencils, mixed
//      term with corrected signs) and the contraction T = D : H
//   E  outer second differences of T (eq. genModel), explicit step,
//      FSI extrapolation (Sec. 3.3) and Dirichlet hold of the known pixels;
//      optionally the FP64 cycle residual.
// Every intermediate is evaluated on the mirror-extended image, so the halo
// values of T carry the parity the boundary needs and P stays symmetric.
#pragma once

#include "eed4_internal.h"
#include "eed4_pointwise.h"

namespace eed4 {

__device__ __forceinline__ int mirror_index(int i, int n)
{
    int p = 2 * n;
    int m = i % p;
    if (m < 0) m += p;
    return m < n ? m : p - 1 - m;
}

template <int R, int TW, int TH, int NTH = kThreads>
struct TileGeo {
    static_assert(TW % 4 == 0 && NTH % TW == 0, "tile width");
    static constexpr int h = R + 2;                       // input halo
    static constexpr int UH = TH + 2 * h;                 // rows of u in LDS
    static constexpr int UWr = TW + 2 * h;                // used columns of u
    static constexpr int UW = (UWr + 3) & ~3;             // padded row stride
    static constexpr int XW = TW + 4;                     // columns after the x pass
    static constexpr int VH = TH + 4;                     // rows after the y pass
    static constexpr int PH = TH + 2, PW = TW + 2;        // tensor points
    static constexpr int NU = UH * UW, NX = UH * XW, NV = VH * XW, NP = PH * PW;
    static constexpr int NT = 3 * NP;
    static constexpr int REGA = (NU + NX > NT) ? NU + NX : NT;  // u + x pass, later T
    static constexpr int SMEM = REGA + NV;                // floats of LDS
    static constexpr int NF4 = (4 + 2 * R + 3) / 4;       // float4 loads per x window
    static constexpr int NQ = XW / 4;                     // x-pass items per row
    static constexpr int nyr()
    {
        int r = 4;
        while (((VH + r - 1) / r) * XW > NTH && r < VH) ++r;
        return r;
    }
    static constexpr int NYR = nyr();                     // rows per y-pass item
    static constexpr int NRUN = (VH + NYR - 1) / NYR;
    static constexpr int NPT = (NP + NTH - 1) / NTH;
    static constexpr int RPP = NTH / TW;                  // output rows per pass
    static_assert(TH % RPP == 0, "tile height");
    static_assert(UW * UH >= 0, "");
};

// Accumulates sum (un - ref)^2 and sum un^2 of the tile in FP64 and writes
// them to out[0..1] (thread 0).  Fixed reduction order: deterministic.
template <int NTH = kThreads>
__device__ __forceinline__ void block_sum2(double d2, double n2, double *scratch, double *out)
{
    for (int o = 32; o > 0; o >>= 1) {
        d2 += __shfl_down(d2, o, 64);
        n2 += __shfl_down(n2, o, 64);
    }
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        scratch[2 * wv] = d2;
        scratch[2 * wv + 1] = n2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int i = 0; i < NTH / 64; ++i) {
            a += scratch[2 * i];
            b += scratch[2 * i + 1];
        }
        out[0] = a;
        out[1] = b;
    }
}

// One tile.  ucur/uprev/uout/ref/mask point at the image (H x W).  ref, when
// not null, is the cycle-start state for the residual (it may equal uout: each
// pixel is read before it is written by the same thread).
template <int R, int TW, int TH, int NTH = kThreads>
__device__ __forceinline__ void step_tile(float *smem, const float *ucur, const float *uprev,
                                          float *uout, const float *ref,
                                          const uint8_t *__restrict__ mask, int H, int W, int ty,
                                          int tx, const float (&w)[2 * kRMax + 1], float tau,
                                          float alpha, float il2q, double *partial)
{
    using G = TileGeo<R, TW, TH, NTH>;
    float *sU = smem;
    float *sX = smem + G::NU;
    float *sV = smem + G::REGA;
    float *sT = smem;  // [3][PH][PW], written after sU and sX are dead
    const int tid = threadIdx.x;
    const int gx0 = tx * TW, gy0 = ty * TH;
    if constexpr (kLdsSentinel) sentinel_fill_block(smem, G::SMEM);

    // The pointwise operands of this thread's outputs (stage E: rows rr,
    // rr + RPP, ... of column c) are loaded first, so that their memory
    // latency overlaps stages A-D instead of following them.  Tiles with
    // more than 4 outputs per thread load them in stage E (the registers
    // would cost more waves than the latency they hide).
    constexpr int NE = TH / G::RPP;
    constexpr bool PF = NE <= 4;
    const int c = tid % TW, rr = tid / TW;
    float ek[NE], ep[NE], ef[NE];
    int em[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const int gy = gy0 + rr + e * G::RPP, gx = gx0 + c;
        ek[e] = ep[e] = ef[e] = 0.0f;
        em[e] = 0;
        if (PF && gy < H && gx < W) {
            const size_t gi = (size_t)gy * W + gx;
            ek[e] = ucur[gi];
            ep[e] = uprev[gi];
            em[e] = mask[gi];
            if (ref) ef[e] = ref[gi];
        }
    }

    // ---- A: u^k with halo ----
    {
        const int x0 = gx0 - G::h, y0 = gy0 - G::h;
        const bool inside = x0 >= 0 && y0 >= 0 && x0 + G::UWr <= W && y0 + G::UH <= H;
        if (inside) {
            for (int i = tid; i < G::UH * G::UWr; i += NTH) {
                int r = i / G::UWr, c = i - r * G::UWr;
                sU[r * G::UW + c] = ucur[(size_t)(y0 + r) * W + (x0 + c)];
            }
        } else {
            for (int i = tid; i < G::UH * G::UWr; i += NTH) {
                int r = i / G::UWr, c = i - r * G::UWr;
                int yy = mirror_index(y0 + r, H), xx = mirror_index(x0 + c, W);
                sU[r * G::UW + c] = ucur[(size_t)yy * W + xx];
            }
        }
    }
    __syncthreads();

    // ---- B: x pass, 4 outputs per item ----
    for (int i = tid; i < G::UH * G::NQ; i += NTH) {
        int r = i / G::NQ, q = i - r * G::NQ;
        const float4 *src = reinterpret_cast<const float4 *>(sU + r * G::UW + 4 * q);
        float win[4 * G::NF4];
#pragma unroll
        for (int f = 0; f < G::NF4; ++f) {
            float4 v = src[f];
            win[4 * f] = v.x;
            win[4 * f + 1] = v.y;
            win[4 * f + 2] = v.z;
            win[4 * f + 3] = v.w;
        }
        float o[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float s = w[0] * win[e];
#pragma unroll
            for (int j = 1; j <= 2 * R; ++j) s = fmaf(w[j], win[e + j], s);
            o[e] = s;
        }
        *reinterpret_cast<float4 *>(sX + r * G::XW + 4 * q) = make_float4(o[0], o[1], o[2], o[3]);
    }
    __syncthreads();

    // ---- C: y pass, NYR outputs per item ----
    for (int i = tid; i < G::NRUN * G::XW; i += NTH) {
        int run = i / G::XW, c = i - run * G::XW;
        int r0 = run * G::NYR;
        float win[G::NYR + 2 * R];
#pragma unroll
        for (int j = 0; j < G::NYR + 2 * R; ++j)
            win[j] = (r0 + j < G::UH) ? sX[(r0 + j) * G::XW + c] : 0.0f;
#pragma unroll
        for (int e = 0; e < G::NYR; ++e) {
            if (r0 + e < G::VH) {
                sV[(r0 + e) * G::XW + c] = ypass_sym<R>(w, [&](int j) { return win[e + R + j]; });
            }
        }
    }
    __syncthreads();

    // ---- D: gradient, tensor, Hessian, contraction on the tile grown by 1 ----
    float txx[G::NPT], tyy[G::NPT], txy[G::NPT];
#pragma unroll
    for (int k = 0; k < G::NPT; ++k) {
        int p = tid + k * NTH;
        txx[k] = tyy[k] = txy[k] = 0.0f;
        if (p < G::NP) {
            int pr = p / G::PW, pc = p - pr * G::PW;
            const float *v = sV + (pr + 1) * G::XW + (pc + 1);
            const float gxs = v[1] - v[-1];                          // 2 gx
            const float gys = v[G::XW] - v[-G::XW];                  // 2 gy
            const float *u = sU + (pr + G::h - 1) * G::UW + (pc + G::h - 1);
            const float uc = u[0];
            const float hxx = second_diff(u[-1], uc, u[1]);
            const float hyy = second_diff(u[-G::UW], uc, u[G::UW]);
            const float hxy = mixed_diff(xdiff(u[G::UW - 1], u[G::UW + 1]),
                                         xdiff(u[-G::UW - 1], u[-G::UW + 1]));
            const float s2 = grad2_sq(gxs, gys);                     // 4 |grad|^2
            float mu1, mu3;
            foeed_mu(s2, il2q, mu1, mu3);
            contract(gxs, gys, s2, mu1, mu3, hxx, hyy, hxy, txx[k], tyy[k], txy[k]);
        }
    }
    __syncthreads();
    if constexpr (kLdsSentinel) sentinel_fill_block(sT, G::NT);
#pragma unroll
    for (int k = 0; k < G::NPT; ++k) {
        int p = tid + k * NTH;
        if (p < G::NP) {
            sT[p] = txx[k];
            sT[G::NP + p] = tyy[k];
            sT[2 * G::NP + p] = txy[k];
        }
    }
    __syncthreads();

    // ---- E: outer differences, FSI step, Dirichlet hold, residual ----
    double d2 = 0.0, n2 = 0.0;
    constexpr int UE = PF ? NE : 2;
#pragma unroll UE
    for (int e = 0; e < NE; ++e) {
        const int r = rr + e * G::RPP;
        int gy = gy0 + r, gx = gx0 + c;
        if (gy < H && gx < W) {
            int p = (r + 1) * G::PW + (c + 1);
            const float *Txx = sT + p;
            const float *Tyy = sT + G::NP + p;
            const float *Txy = sT + 2 * G::NP + p;
            const float pu = outer_div(Txx[0], Tyy[0], Txx[-1] + Txx[1], Tyy[-G::PW] + Tyy[G::PW],
                                       Txy[G::PW + 1] - Txy[G::PW - 1],
                                       Txy[-G::PW + 1] - Txy[-G::PW - 1]);
            size_t gi = (size_t)gy * W + gx;
            const float uk = PF ? ek[e] : ucur[gi];
            const float up = PF ? ep[e] : uprev[gi];
            const float un = fsi_update(pu, uk, up, tau, alpha, (PF ? em[e] : mask[gi]) != 0);
            if (ref) {
                double dd = (double)un - (double)(PF ? ef[e] : ref[gi]);
                d2 = fma(dd, dd, d2);
                n2 = fma((double)un, (double)un, n2);
            }
            uout[gi] = un;
        }
    }
    if (ref) {
        __syncthreads();
        block_sum2<NTH>(d2, n2, reinterpret_cast<double *>(smem), partial);
    }
}

// Workgroup -> tile map that gives each XCD (workgroups are dealt round-robin
// over 8 XCDs) a contiguous run of tiles, so neighbouring tiles, which share
// halo rows, usually meet in the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb)
{
    const int nx = 8;
    int q = nb / nx, rem = nb % nx;
    int xcd = bid % nx, idx = bid / nx;
    int base = xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q;
    return base + idx;
}

}  // namespace eed4
