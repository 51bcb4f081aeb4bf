// Device code of one fused FOEED/FSI inner step on a vertical strip, one
// wavefront per strip, no workgroup barriers.
//
// A wave owns NL = 64 CPL consecutive columns c = X0-2 .. X0+NL-3 (CPL
// adjacent columns per lane) and streams down the rows of a segment.  For
// each input row y it
//   S1  stages u^k(y, X0-2-R .. X0+NL-3+R) in a per-wave LDS ring (mirrored
//       indices realise the Neumann condition, Sec. 2.1) and takes the x pass
//       of the Gaussian presmoothing (Sec. 2.2) at its columns;
//   S2  completes the y pass at row y-R from a register window of the last
//       2R+1 x-pass values (the row loop is unrolled over that window);
//   S3  at row g = y-R-1: central-difference gradient of u_sigma, fourth-order
//       diffusion tensor (Sec. 3.1: eigenvalues g, 1, sqrt g), Hessian of u
//       from the LDS ring (Sec. 3.3 stencils, sign-corrected u_xy) and
//       T = D : H;
//   S4  at row o = g-1: outer differences of T (eq. genModel), explicit step,
//       FSI extrapolation (Sec. 3.3), Dirichlet hold; optional FP64 residual;
//       optionally also the presmoothed image v = K_sigma * u^k at row o (the
//       adjoint's recompute keeps it for the reverse step).
// Horizontal neighbours inside a lane are its own registers; across lanes
// they come from DPP wave shifts.  Outputs are the NL-4 columns X0 ..
// X0+NL-5.  Every intermediate lives on the mirror-extended image, so P stays
// symmetric, and each pixel's arithmetic is the same for every CPL.
#pragma once

#include "eed4_internal.h"
#include "eed4_pointwise.h"

namespace eed4 {

// Half-sample mirror by repeated reflection (any i, n >= 1).
__device__ __forceinline__ int mirror_reflect(int i, int n)
{
    while (i < 0 || i >= n) i = (i < 0) ? -1 - i : 2 * n - 1 - i;
    return i;
}

// Value held by lane+1 / lane-1 (DPP wave shifts; edge lanes read 0).
__device__ __forceinline__ float from_next_lane(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ float from_prev_lane(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}

// Lane 0's value of a double, wave-uniform.
__device__ __forceinline__ double lane0_double(double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, 0);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), 0);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Orders LDS accesses of different lanes of one wave (a wave executes its LDS
// instructions in order; this only stops the compiler from reordering them).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// ROWS is the least number of output rows of a wave's segment (the segment
// is rounded up to whole unrolled iterations).
//
// The LDS ring holds the last D staged rows column-major: staged column c
// (0 .. NU-1) of ring row r is at (c + 1) * CS + r, with an empty column on
// each side.  A lane addresses everything it reads (x-pass taps, Hessian
// neighbours) as compile-time offsets from its own column, which stay within
// the reach of paired LDS reads, and the odd stride CS keeps the 64 lanes on
// distinct banks.
template <int R, int ROWS = 64, int CPL = 1>
struct StripGeo {
    static constexpr int P = 2 * R + 1;                       // y window length
    static constexpr int U = P * ((R + 3 + P - 1) / P);       // unroll = LDS ring depth
    static constexpr int D = U;                               // (a multiple of P, >= R+3)
    static constexpr int h = R + 2;                           // input halo
    static constexpr int NL = 64 * CPL;                       // columns held by the lanes
    static constexpr int SW = NL - 4;                         // output columns per wave
    static constexpr int NU = NL + 2 * R;                     // staged u columns per row
    static constexpr int CS = D | 1;                          // ring column stride (odd)
    static constexpr int M = (ROWS + 4 + U - 1) / U;          // main-loop iterations
    static constexpr int NROW = 2 * R + M * U;                // rows streamed per wave
    static constexpr int OH = NROW - 2 * h;                   // output rows per wave
    static constexpr int LDS = (NU + 2) * CS;                 // floats of LDS per wave
};

// Per-wave constants of a strip step.
struct StripArgs {
    const float *ucur, *uprev;
    float *uout;
    const float *ref;           // cycle start for the residual (RES variant only)
    float *vout;                // K_sigma * u^k at the output pixels (VST variant only)
    const uint8_t *mask;
    int H, W, X0, Y0;
    float tau, alpha, il2q;     // il2q = 1 / (4 lambda^2)
    int model;                  // tensor variant (GEN kernels only)
    int up;                     // stream the segment bottom up (see strip_step)
};

// mu1 = g(x) and mu3 of the tensor variants, x = (s/lambda)^2: the
// diffusivities of Table 7 (Geman-Reynolds scaled to g(0) = 1) and the mu3
// choices of Sec. 3.1 (geometric mean, arithmetic mean or maximum of mu1 and
// mu2 = 1).  model = diffusivity | rule << 4, uniform over the launch.
__device__ __forceinline__ void model_mu(float x, int model, float &mu1, float &mu3)
{
#pragma clang fp contract(off)
    const int diff = model & 0xf, rule = model >> 4;
    const float d = 1.0f + x;
    float g;
    if (diff == kDiffPeronaMalik) {
        g = __builtin_amdgcn_rcpf(d);
    } else if (diff == kDiffPeronaMalikExp) {
        // exp(-x) = 2^(-x log2 e) on the hardware exp2 (1 ulp): two instructions
        // instead of the library's range reduction
        g = __builtin_amdgcn_exp2f(-x * 1.44269504088896341f);
    } else if (diff == kDiffGemanReynolds) {
        const float r = __builtin_amdgcn_rcpf(d);
        g = r * r;
    } else {
        g = __builtin_amdgcn_rsqf(d);
    }
    mu1 = g;
    mu3 = rule == kMu3Arithmetic ? 0.5f * (1.0f + g)
        : rule == kMu3Max        ? 1.0f
                                 : __builtin_amdgcn_sqrtf(g);
}

// Raw buffer resource over the `bytes` bytes from `base` (gfx9 descriptor:
// stride 0, no swizzle).  A load at a byte offset at or beyond `bytes` reads 0
// and a store there is dropped: lanes without an output pixel use kOffNone.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *base, unsigned bytes)
{
    // The empty asm makes the size and flag words opaque, so resources with
    // equal words get SGPRs of their own: otherwise the compiler keeps one copy
    // and rebuilds the four-register descriptor before every access in the loop.
    int flags = 0x00020000;
    asm volatile("" : "+s"(bytes), "+s"(flags));
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             flags);
}
constexpr unsigned kOffNone = 0x80000000u;

__device__ __forceinline__ float buf_f32(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// Image row of consecutive stream rows under the half-sample mirror: the row
// moves in direction dir; at an edge it repeats once and the direction flips.
struct RowTrack {
    int y, dir;
    __device__ __forceinline__ void init(int y0, int H)
    {
        y = mirror_reflect(y0, H);
        const int k = y0 >= 0 ? y0 / H : -1 - (-1 - y0) / H;   // mirror copy index
        dir = (k & 1) ? -1 : 1;
    }
    __device__ __forceinline__ void next(int H)
    {
        int nx = y + dir;
        if ((unsigned)nx >= (unsigned)H) {
            dir = -dir;
            nx = y;
        }
        y = nx;
    }
};

// Global loads of one stream row: u^k of the row itself (the lane's columns
// and one right-halo column), and u^{k-1}, the mask and the residual
// reference of the output row it serves.
template <int CPL>
struct StripRow {
    float a[CPL], b, pv[CPL], rf[CPL];
    unsigned mk[CPL];
};

// Column q's left / right neighbour of a per-column register quantity.
template <int CPL>
__device__ __forceinline__ float left_of(const float (&x)[CPL], int q)
{
    return q > 0 ? x[q - 1] : from_prev_lane(x[CPL - 1]);
}
template <int CPL>
__device__ __forceinline__ float right_of(const float (&x)[CPL], int q)
{
    return q < CPL - 1 ? x[q + 1] : from_next_lane(x[0]);
}

// Addressing: every plane is seen through a buffer resource based at image
// row b0 = max(Y0 - h, 0) (the lowest row a needed value comes from) and
// covering nb = min(H - b0, NROW) rows, so a row offset is one 32-bit scalar
// (the library keeps NROW * W * 4 below 2^31) and the per-lane column offsets
// stay fixed for the whole strip.
//
// Direction: with segments of >= 64 rows, callers stream odd segments bottom
// up and even ones top down, so the 2h rows two neighbouring segments share
// are read by both at nearly the same time (near the end of both streams, or
// near the start of both) and the second read usually hits in L2; with every
// segment streaming down, one reads them first and the other last, a whole
// launch later.  (Measured at 4096^2 and 8192^2: the 64-row strips as fast in
// the cache-resident case and 5 % faster out of it; 28-row strips 8 % slower,
// so they all stream down.)  The stencils are symmetric in y: streaming up
// only negates the y-odd quantities (G_y, u_xy, T_xy and its x differences)
// exactly, and the y pass is symmetric, so u^{k+1} (and the kept v) are
// bitwise those of the downward stream; only the FP64 residual partials add
// the rows in the other order.
constexpr bool strip_alternates(int rows) { return rows >= 64; }

template <int R, bool RES, int ROWS = 64, int CPL = 1, bool GEN = false, bool VST = false>
__device__ __forceinline__ void strip_step(float *ring, const StripArgs &s,
                                           const float (&w)[2 * kRMax + 1], double *partial)
{
    using G = StripGeo<R, ROWS, CPL>;
    constexpr int P = G::P, U = G::U, D = G::D, NL = G::NL, CS = G::CS;
    const int lane = threadIdx.x & 63;
    const int H = s.H, W = s.W;
    const unsigned W4 = 4u * (unsigned)W;
    if constexpr (kLdsSentinel) sentinel_fill_wave(ring, G::LDS);

    const int ybase = s.Y0 - G::h;                            // top streamed row
    const int dir = s.up ? -1 : 1;                            // image rows per stream row
    const int ystart = s.up ? ybase + G::NROW - 1 : ybase;    // image row of stream row 0
    const int b0 = ybase > 0 ? ybase : 0;
    const int nb = (H - b0 < G::NROW) ? H - b0 : G::NROW;
    const size_t base = (size_t)b0 * W;
    const __amdgpu_buffer_rsrc_t rs_u = buffer_rsrc(s.ucur + base, (unsigned)nb * W4);
    const __amdgpu_buffer_rsrc_t rs_p = buffer_rsrc(s.uprev + base, (unsigned)nb * W4);
    const __amdgpu_buffer_rsrc_t rs_o = buffer_rsrc(s.uout + base, (unsigned)nb * W4);
    const __amdgpu_buffer_rsrc_t rs_m = buffer_rsrc(s.mask + base, (unsigned)nb * (unsigned)W);
    __amdgpu_buffer_rsrc_t rs_r = rs_p;
    if constexpr (RES) rs_r = buffer_rsrc(s.ref + base, (unsigned)nb * W4);
    __amdgpu_buffer_rsrc_t rs_v = rs_o;
    if constexpr (VST) rs_v = buffer_rsrc(s.vout + base, (unsigned)nb * W4);

    // Staged columns (fixed for the whole strip): staged column j is image
    // column X0-2-R+j.  Lane l stages j = CPL l + q (q < CPL), and the 2R
    // right-halo columns j = NL .. NL+2R-1 go to lane l = j - NL mod 2R
    // (lanes with the same halo column load and write the same value).
    const int lb = R > 0 ? lane % (2 * R > 0 ? 2 * R : 1) : 0;
    const unsigned cb = 4u * (unsigned)mirror_reflect(s.X0 - 2 - R + NL + lb, W);
    unsigned ca[CPL], vo4[CPL], vo1[CPL];
    bool out_col[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        const int j = CPL * lane + q;                        // this column, within the wave
        const int cl = s.X0 - 2 + j;                         // ... and in the image
        ca[q] = 4u * (unsigned)mirror_reflect(cl - R, W);
        out_col[q] = j >= 2 && j < NL - 2 && cl < W;
        vo4[q] = out_col[q] ? 4u * (unsigned)cl : kOffNone;
        vo1[q] = out_col[q] ? (unsigned)cl : kOffNone;
    }
    float *col = ring + (CPL * lane + 1) * CS;               // ring column of staged column CPL l
    float *bcol = ring + (NL + lb + 1) * CS;                 // right-halo column it stages

    float win[CPL][P];        // x-pass values, row i in slot i % P
#pragma unroll
    for (int q = 0; q < CPL; ++q)
#pragma unroll
        for (int j = 0; j < P; ++j) win[q][j] = 0.0f;
    float v_m1[CPL], v_m2[CPL];                          // v at rows g, g-1 (before update)
    float txx_p[CPL], tyy_p[CPL], tyy_pp[CPL];           // T at rows g-1 (and g-2 for Tyy)
    float z_p[CPL], z_pp[CPL];                           // Txy(c+1)-Txy(c-1) at rows g-1, g-2
    float uc_p[CPL];                                     // u^k(g-1, c)
#pragma unroll
    for (int q = 0; q < CPL; ++q)
        v_m1[q] = v_m2[q] = txx_p[q] = tyy_p[q] = tyy_pp[q] = z_p[q] = z_pp[q] = uc_p[q] = 0.0f;
    double d2 = 0.0, n2 = 0.0;

    // the next row to prefetch: its mirrored image row and the output row it serves
    RowTrack ty;
    ty.init(ystart, H);
    if (s.up) ty.dir = -ty.dir;
    int on = ystart - dir * (R + 2);

    // Loads run two stream rows ahead, always in the same order, so waiting
    // for one row never waits for a later row's loads.
    auto prefetch = [&](StripRow<CPL> &r) {
        const unsigned su = (unsigned)((ty.y > b0 ? ty.y : b0) - b0) * W4;
#pragma unroll
        for (int q = 0; q < CPL; ++q) r.a[q] = buf_f32(rs_u, ca[q], su);
        if constexpr (R > 0) r.b = buf_f32(rs_u, cb, su);
        int oc = on < b0 ? b0 : on;                      // clamped; unused rows are not stored
        oc = oc > H - 1 ? H - 1 : oc;
        const unsigned ro = (unsigned)(oc - b0);
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            r.pv[q] = buf_f32(rs_p, vo4[q], ro * W4);
            r.mk[q] = __builtin_amdgcn_raw_buffer_load_b8(rs_m, vo1[q], ro * (unsigned)W, 0);
            if constexpr (RES) r.rf[q] = buf_f32(rs_r, vo4[q], ro * W4);
        }
        ty.next(H);
        on += dir;
    };
    StripRow<CPL> r0, r1;
    r0.b = r1.b = 0.0f;
#pragma unroll
    for (int q = 0; q < CPL; ++q) r0.rf[q] = r1.rf[q] = 0.0f;
    prefetch(r0);
    prefetch(r1);

    // The Hessian of u at row g needs u(x-1), u(x), u(x+1) at rows g-1, g, g+1.
    // With segments of >= 64 rows (about 4 waves per SIMD, registers to spare)
    // they are kept per staged row, as u(x), u(x-1) + u(x+1) and u(x+1) - u(x-1),
    // in registers indexed like the ring (slot i % D), from the x-pass taps
    // R-1, R, R+1 of row i; the shorter strips, which need 8 waves per SIMD,
    // read them back from the ring.
    constexpr bool HREG = CPL == 1 && ROWS >= 64;
    constexpr int HD = HREG ? D : 1;
    float hc[HD], hs[HD], hd[HD];
#pragma unroll
    for (int j = 0; j < HD; ++j) hc[j] = hs[j] = hd[j] = 0.0f;

    // stage one row of u^k into ring row rr and take its x pass into window slot ws
    auto stage_xpass = [&](const StripRow<CPL> &cur, int rr, int ws) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) col[q * CS + rr] = cur.a[q];
        if constexpr (R > 0) bcol[rr] = cur.b;
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            float acc = w[0] * col[q * CS + rr];
#pragma unroll
            for (int j = 1; j <= 2 * R; ++j) acc = fmaf(w[j], col[(q + j) * CS + rr], acc);
            win[q][ws] = acc;
        }
        if constexpr (HREG) {
            const float l = col[(R - 1) * CS + rr], c = col[R * CS + rr], r = col[(R + 1) * CS + rr];
            hc[rr] = c;
            hs[rr] = l + r;
            hd[rr] = xdiff(l, r);
        }
    };

    // ---- prologue: stage rows 0 .. 2R-1 and their x pass ----
#pragma unroll
    for (int i = 0; i < 2 * R; ++i) {
        const StripRow<CPL> cur = r0;
        r0 = r1;
        prefetch(r1);
        stage_xpass(cur, i % D, i % P);
    }

#pragma unroll 1
    for (int it = 0; it < G::M; ++it) {
        // Issue priority falls as the wave moves down its segment, so waves
        // that are behind get the SIMD first and all waves progress together.
        // With the default oldest-first order the early waves finish first and
        // the launch ends with few waves per SIMD to hide latency (about 4.4 of
        // 8 resident on average at 4096^2); this schedule took the 64-row
        // strips from 49 to 44.5 us there, with bitwise the same results.
        // The adjoint's recompute steps (VST) stay at the lowest priority: they
        // run beside the reverse steps, which are the critical path.
        if constexpr (!VST) {
            const int left = G::M - it;
            if (left >= 4) __builtin_amdgcn_s_setprio(3);
            else if (left == 3) __builtin_amdgcn_s_setprio(2);
            else if (left == 2) __builtin_amdgcn_s_setprio(1);
            else __builtin_amdgcn_s_setprio(0);
        }
#pragma unroll
        for (int ph = 0; ph < U; ++ph) {
            const int i = 2 * R + it * U + ph;           // stream row (wave-uniform)
            const StripRow<CPL> cur = r0;
            r0 = r1;
            prefetch(r1);                                 // mirrored: always valid rows

            // ---- S1: stage u^k row i and take the x pass ----
            stage_xpass(cur, (2 * R + ph) % D, (2 * R + ph) % P);   // constants once unrolled

            // ---- S2: y pass at stream row i - R ----
            // stream row i - R + j is in slot (ph + R + j) % P
            float v[CPL];
#pragma unroll
            for (int q = 0; q < CPL; ++q)
                v[q] = ypass_sym<R>(w, [&](int j) { return win[q][(ph + R + j) % P]; });

            // ---- S3: gradient, tensor, Hessian, contraction at row g = i - R - 1 ----
            // (the first rows of the loop produce values that only feed unstored rows)
            float txx[CPL], tyy[CPL], txy[CPL], uc[CPL], vo[CPL];
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                vo[q] = v_m2[q];                                              // v at row g - 1
                const float gxs = right_of(v_m1, q) - left_of(v_m1, q);      // 2 gx
                const float gys = v[q] - v_m2[q];                             // 2 gy
                // rows g-1, g, g+1 are in ring slots sm, sg, sp
                const int sm = (R - 2 + ph + D) % D, sg = (R - 1 + ph + D) % D, sp = (R + ph) % D;
                float hxx, hyy, hxy;
                if constexpr (HREG) {
                    uc[q] = hc[sg];
                    hxx = second_diff_sum(hs[sg], uc[q]);
                    hyy = second_diff(hc[sm], uc[q], hc[sp]);
                    hxy = mixed_diff(hd[sp], hd[sm]);
                } else {
                    // column q of this lane is staged column CPL l + q + R
                    const float *um = col + (q + R) * CS + sm;
                    const float *u0 = col + (q + R) * CS + sg;
                    const float *up = col + (q + R) * CS + sp;
                    uc[q] = u0[0];
                    hxx = second_diff(u0[-CS], uc[q], u0[CS]);
                    hyy = second_diff(um[0], uc[q], up[0]);
                    hxy = mixed_diff(xdiff(up[-CS], up[CS]), xdiff(um[-CS], um[CS]));
                }

                const float s2 = grad2_sq(gxs, gys);                          // 4 |grad|^2
                float mu1, mu3;
                if constexpr (GEN) {
                    model_mu(s2 * s.il2q, s.model, mu1, mu3);
                } else {                                     // FOEED: Charbonnier, sqrt
                    foeed_mu(s2, s.il2q, mu1, mu3);
                }
                contract(gxs, gys, s2, mu1, mu3, hxx, hyy, hxy, txx[q], tyy[q], txy[q]);
            }
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                v_m2[q] = v_m1[q];
                v_m1[q] = v[q];
            }

            // ---- S4: output row o = g - 1 (stream row i - R - 2) ----
            float z[CPL];
#pragma unroll
            for (int q = 0; q < CPL; ++q) z[q] = right_of(txy, q) - left_of(txy, q);
            const int o = ystart + dir * (i - R - 2);
            if (i >= 2 * G::h && o < H) {      // first output row: Y0 (down), Y0 + OH - 1 (up)
                const unsigned ro = (unsigned)(o - b0) * W4;
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    const float sxx = left_of(txx_p, q) + right_of(txx_p, q);
                    const float pu = outer_div(txx_p[q], tyy_p[q], sxx, tyy_pp[q] + tyy[q], z[q],
                                               z_pp[q]);
                    const float un = fsi_update(pu, uc_p[q], cur.pv[q], s.tau, s.alpha,
                                                cur.mk[q] != 0);
                    if constexpr (RES) {
                        // columns without a pixel read 0 for the reference; add 0
                        const double du = out_col[q] ? (double)un : 0.0;
                        const double dd = du - (double)cur.rf[q];
                        d2 = fma(dd, dd, d2);
                        n2 = fma(du, du, n2);
                    }
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(un), rs_o, vo4[q], ro, 0);
                    if constexpr (VST)
                        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(vo[q]), rs_v, vo4[q],
                                                              ro, 0);
                }
            }
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                tyy_pp[q] = tyy_p[q];
                tyy_p[q] = tyy[q];
                txx_p[q] = txx[q];
                z_pp[q] = z_p[q];
                z_p[q] = z[q];
                uc_p[q] = uc[q];
            }
        }
    }
    if constexpr (RES) {
        for (int off = 32; off > 0; off >>= 1) {
            d2 += __shfl_down(d2, off, 64);
            n2 += __shfl_down(n2, off, 64);
        }
        // lane 0 holds the sums; every lane stores that same value (no
        // lane-dependent branch at the end of a batched queue-loop body)
        const double d2s = lane0_double(d2), n2s = lane0_double(n2);
        partial[0] = d2s;
        partial[1] = n2s;
    }
}

}  // namespace eed4
