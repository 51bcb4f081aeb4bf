// Per-pixel arithmetic of one FOEED/FSI inner step, shared by every fused
// step kernel (wave strips, workgroup tiles, the batched queue versions).
//
// Each kernel gathers the neighbours its own way (LDS ring, DPP lane shifts,
// LDS tiles), but every value is formed by these functions with the same
// operands in the same order, so all kernel shapes give bitwise the same
// result for every pixel.  Floating-point contraction is switched off inside
// them and every fused multiply-add is written out: otherwise the compiler
// fuses a product into a neighbouring add in one kernel and not in another,
// depending on how the surrounding code is laid out, and the roundings differ.
#pragma once

#include "eed4_internal.h"

namespace eed4 {

// Second differences of u (Sec. 3.3 stencils): centre c and the sum of its
// two neighbours on one axis, a + b (taken in that order), ...
__device__ __forceinline__ float second_diff_sum(float ab, float c)
{
#pragma clang fp contract(off)
    return fmaf(-2.0f, c, ab);
}
// ... or the neighbours a and b themselves.
__device__ __forceinline__ float second_diff(float a, float c, float b)
{
#pragma clang fp contract(off)
    return second_diff_sum(a + b, c);
}

// Central x difference along one row, u(x+1) - u(x-1).
__device__ __forceinline__ float xdiff(float left, float right)
{
#pragma clang fp contract(off)
    return right - left;
}

// Mixed difference u_xy with the signs of a derivative (Sec. 3.3 prints four
// plus signs), from the x differences of the rows below and above:
// dp = u(y+1, x+1) - u(y+1, x-1), dm = u(y-1, x+1) - u(y-1, x-1).
__device__ __forceinline__ float mixed_diff(float dp, float dm)
{
#pragma clang fp contract(off)
    return 0.25f * (dp - dm);
}

// The y pass of the Gaussian presmoothing (Sec. 3.1, K_sigma) at one pixel
// from the x-pass values of its column, at(j) = the value j rows below it
// (j = -R..R): the centre first, then the pairs at distance 1, 2, ..., R
// (the sampled kernel is symmetric, w[R - j] = w[R + j]).  The operations do
// not depend on which end of the column is read first, so strips that stream
// down or up, tiles and the presmoothing kernel agree bitwise.
template <int R, typename At>
__device__ __forceinline__ float ypass_sym(const float *w, At at)
{
#pragma clang fp contract(off)
    float acc = w[R] * at(0);
#pragma unroll
    for (int j = 1; j <= R; ++j) acc = fmaf(w[R + j], at(-j) + at(j), acc);
    return acc;
}

// Squared norm of twice the regularised gradient: gxs, gys are the central
// differences v(x+1) - v(x-1), v(y+1) - v(y-1) of the presmoothed image
// (2 grad u_sigma, Sec. 3.1).
__device__ __forceinline__ float grad2_sq(float gxs, float gys)
{
#pragma clang fp contract(off)
    return fmaf(gxs, gxs, gys * gys);
}

// FOEED eigenvalues (eq. CharDiff, Sec. 3.1): mu1 = g = (1 + |grad|^2 /
// lambda^2)^(-1/2) with |grad|^2 = s2 / 4 (il2q = 1 / (4 lambda^2)), mu2 = 1,
// mu3 = sqrt(mu1 mu2).
__device__ __forceinline__ void foeed_mu(float s2, float il2q, float &mu1, float &mu3)
{
#pragma clang fp contract(off)
    mu1 = __builtin_amdgcn_rsqf(fmaf(s2, il2q, 1.0f));
    mu3 = __builtin_amdgcn_sqrtf(mu1);
}

// T = D : H for the tensor with eigenvalues mu1, 1, mu3 along E1 = n n^T,
// E2 = t t^T, E3 = (n t^T + t n^T)/sqrt2 (eqs. faod_diffTensor,
// foad_diffTensor_entries), in rank-2 update form:
//   T = H + (mu1 - 1)(E1 : H) E1 + (mu3 - 1)(E3 : H) E3,
//   (E3 : H) E3 = [c (hyy - hxx) + (a - b) hxy] [[-2c, a - b], [a - b, 2c]],
// a = nx^2, b = ny^2, c = nx ny, n the unit gradient direction (taken as 0
// where the gradient vanishes: there mu1 = mu3 = 1 and T = H).
__device__ __forceinline__ void contract(float gxs, float gys, float s2, float mu1, float mu3,
                                         float hxx, float hyy, float hxy, float &txx, float &tyy,
                                         float &txy)
{
#pragma clang fp contract(off)
    const float rn = __builtin_amdgcn_rsqf(fmaxf(s2, 1e-30f));
    const float nx = gxs * rn, ny = gys * rn;
    const float aa = nx * nx, bb = ny * ny, c = nx * ny;
    const float amb = aa - bb, c2 = c + c;
    const float e1h = fmaf(aa, hxx, fmaf(bb, hyy, c2 * hxy));
    const float x3 = fmaf(c, hyy - hxx, amb * hxy);
    const float k1 = fmaf(mu1, e1h, -e1h);
    const float k3 = fmaf(mu3, x3, -x3);
    const float k3c2 = k3 * c2;
    txx = fmaf(k1, aa, hxx - k3c2);
    tyy = fmaf(k1, bb, hyy + k3c2);
    txy = fmaf(k1, c, fmaf(k3, amb, hxy));
}

// Outer divergence (eq. genModel) at pixel (o, x):
//   Pu = D_xx T_xx + 2 D_xy T_xy + D_yy T_yy
// from txx_c = Txx(o, x), tyy_c = Tyy(o, x), sxx = Txx(o, x-1) + Txx(o, x+1),
// syy = Tyy(o-1, x) + Tyy(o+1, x), and zd / zu = Txy(r, x+1) - Txy(r, x-1) at
// rows r = o+1 / o-1.
__device__ __forceinline__ float outer_div(float txx_c, float tyy_c, float sxx, float syy,
                                           float zd, float zu)
{
#pragma clang fp contract(off)
    return fmaf(0.5f, zd - zu, fmaf(-2.0f, txx_c + tyy_c, sxx + syy));
}

// Explicit step and FSI extrapolation (Sec. 3.3),
//   u^{k+1} = u^{k-1} + alpha_k ((u^k - tau Pu) - u^{k-1}),
// then the Dirichlet hold u = f on K (u^k already equals f there).
__device__ __forceinline__ float fsi_update(float pu, float uk, float uprev, float tau,
                                            float alpha, bool known)
{
#pragma clang fp contract(off)
    const float wv = fmaf(-tau, pu, uk);
    const float un = fmaf(alpha, wv - uprev, uprev);
    return known ? uk : un;
}

}  // namespace eed4
