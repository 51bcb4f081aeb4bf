// Forward kernels: Dirichlet hold, fused FSI inner step over a grid of
// tiles (one workgroup per tile, batch of equal-size images), and the
// deterministic FP64 reduction of the per-tile cycle residuals.
#include "eed4_internal.h"
#include "eed4_tile.h"
#include "eed4_strip.h"

namespace eed4 {

// u = f on the known set K (eq. inpaintingModel).  Four pixels per thread,
// with the four mask bytes loaded (as one word when the mask is 4-byte
// aligned) before any of them is used, so the loads overlap.
__global__ __launch_bounds__(256) void hold_kernel(float *u, const uint8_t *__restrict__ mask,
                                                   const float *__restrict__ known, size_t n)
{
    const size_t i0 = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i0 >= n) return;
    unsigned m[4];
    if ((((uintptr_t)mask) & 3) == 0 && i0 + 4 <= n) {
        const unsigned wd = *reinterpret_cast<const unsigned *>(mask + i0);
#pragma unroll
        for (int j = 0; j < 4; ++j) m[j] = (wd >> (8 * j)) & 0xffu;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) m[j] = i0 + j < n ? mask[i0 + j] : 0u;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (m[j]) u[i0 + j] = known[i0 + j];
}

template <int R, int TW, int TH>
__global__ __launch_bounds__(tile_threads(TW, TH)) void step_kernel(
    const float *ucur, const float *uprev, float *uout, const float *ref,
    const uint8_t *__restrict__ mask, int H, int W, int nbx, int tiles_per_img, StepArgs a,
    double *partials)
{
    constexpr int NTH = tile_threads(TW, TH);
    __shared__ __attribute__((aligned(16))) float smem[TileGeo<R, TW, TH, NTH>::SMEM];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int b = tile / tiles_per_img;
    const int t = tile - b * tiles_per_img;
    const int ty = t / nbx, tx = t - ty * nbx;
    const size_t off = (size_t)b * H * W;
    step_tile<R, TW, TH, NTH>(smem, ucur + off, uprev + off, uout + off,
                              ref ? ref + off : nullptr, mask + off, H, W, ty, tx, a.w, a.tau,
                              a.alpha, 0.25f * a.inv_lam2,
                              partials ? partials + 2 * (size_t)tile : nullptr);
}

// Fused step over wave strips.  GEN selects the tensor variant at run time
// (StepArgs::model); without it the kernel is the FOEED tensor.  VST also
// writes the presmoothed image K_sigma * u^k (into vout).
template <int R, bool RES, int ROWS, int CPL, bool GEN, bool VST = false>
__device__ __forceinline__ void strip_kernel_body(const float *ucur, const float *uprev,
                                                  float *uout, const float *ref,
                                                  const uint8_t *__restrict__ mask, int H, int W,
                                                  int nstrip, int per_img, int nitems,
                                                  const StepArgs &a, double *partials,
                                                  float *vout = nullptr)
{
    using G = StripGeo<R, ROWS, CPL>;
    __shared__ float lds[4 * G::LDS];
    const int wave = threadIdx.x >> 6;
    // wave-uniform: keep the work item (and all that derives from it) in SGPRs
    const int item = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * 4 + wave);
    if (item >= nitems) return;  // whole wave; the kernel has no workgroup barrier
    const int b = item / per_img;
    const int r = item - b * per_img;
    const int seg = r / nstrip, strip = r - seg * nstrip;
    const size_t off = (size_t)b * H * W;
    StripArgs s;
    s.ucur = ucur + off;
    s.uprev = uprev + off;
    s.uout = uout + off;
    s.ref = RES ? ref + off : nullptr;
    s.vout = VST ? vout + off : nullptr;
    s.mask = mask + off;
    s.H = H;
    s.W = W;
    s.X0 = strip * G::SW;
    s.Y0 = seg * G::OH;
    s.tau = a.tau;
    s.alpha = a.alpha;
    s.il2q = 0.25f * a.inv_lam2;
    s.model = a.model;
    s.up = strip_alternates(ROWS) ? seg & 1 : 0;
    strip_step<R, RES, ROWS, CPL, GEN, VST>(lds + wave * G::LDS, s, a.w,
                                            RES ? partials + 2 * (size_t)item : nullptr);
}

template <int R, bool RES, int ROWS, int CPL>
__global__ __launch_bounds__(256) void strip_kernel(const float *ucur, const float *uprev,
                                                    float *uout, const float *ref,
                                                    const uint8_t *__restrict__ mask, int H, int W,
                                                    int nstrip, int per_img, int nitems, StepArgs a,
                                                    double *partials)
{
    strip_kernel_body<R, RES, ROWS, CPL, false>(ucur, uprev, uout, ref, mask, H, W, nstrip,
                                                per_img, nitems, a, partials);
}

// The tensor variants (diffusivities of Table 7, mu3 choices of Sec. 3.1) on
// 60-column strips of >= 28 rows.
template <int R, bool RES>
__global__ __launch_bounds__(256) void strip_model_kernel(const float *ucur, const float *uprev,
                                                          float *uout, const float *ref,
                                                          const uint8_t *__restrict__ mask, int H,
                                                          int W, int nstrip, int per_img,
                                                          int nitems, StepArgs a, double *partials)
{
    strip_kernel_body<R, RES, 28, 1, true>(ucur, uprev, uout, ref, mask, H, W, nstrip, per_img,
                                           nitems, a, partials);
}

// The step of the adjoint's forward recompute: u^{k+1} as strip_kernel (or
// strip_model_kernel when GEN) computes it, and K_sigma * u^k for the reverse
// step.
template <int R, int ROWS, bool GEN>
__global__ __launch_bounds__(256) void strip_keepv_kernel(const float *ucur, const float *uprev,
                                                          float *uout, float *vout,
                                                          const uint8_t *__restrict__ mask, int H,
                                                          int W, int nstrip, int per_img,
                                                          int nitems, StepArgs a)
{
    strip_kernel_body<R, false, ROWS, 1, GEN, true>(ucur, uprev, uout, nullptr, mask, H, W, nstrip,
                                                    per_img, nitems, a, nullptr, vout);
}

// v = K_sigma * u on the mirror-extended image (the presmoothing of Sec. 2.2)
// over 64 x 16 tiles: the same taps in the same order as the x and y passes of
// the fused step, so v is bitwise the one a step from u computes.
constexpr int kBlurTW = 64, kBlurTH = 16;
template <int R>
__global__ __launch_bounds__(256) void blur_kernel(const float *u_all, float *v_all, int H, int W,
                                                   int nbx, int tiles_per_img, StepArgs a)
{
    constexpr int TW = kBlurTW, TH = kBlurTH, SH = TH + 2 * R, SWu = TW + 2 * R;
    __shared__ float su[SH * SWu];
    __shared__ float sx[SH * TW];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int b = tile / tiles_per_img;
    const int t = tile - b * tiles_per_img;
    const int y0 = (t / nbx) * TH, x0 = (t - (t / nbx) * nbx) * TW;
    const float *u = u_all + (size_t)b * H * W;
    float *v = v_all + (size_t)b * H * W;
    if constexpr (kLdsSentinel) {
        sentinel_fill_block(su, SH * SWu);
        sentinel_fill_block(sx, SH * TW);
    }
    for (int k = threadIdx.x; k < SH * SWu; k += 256) {
        const int rr = k / SWu, cc = k - rr * SWu;
        const int y = mirror_reflect(y0 - R + rr, H), x = mirror_reflect(x0 - R + cc, W);
        su[k] = u[(size_t)y * W + x];
    }
    __syncthreads();
    for (int k = threadIdx.x; k < SH * TW; k += 256) {
        const int rr = k / TW, c = k - rr * TW;
        const float *row = su + rr * SWu + c;
        float acc = a.w[0] * row[0];
#pragma unroll
        for (int j = 1; j <= 2 * R; ++j) acc = fmaf(a.w[j], row[j], acc);
        sx[k] = acc;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < TH * TW; k += 256) {
        const int r = k / TW, c = k - r * TW;
        const int y = y0 + r, x = x0 + c;
        if (y >= H || x >= W) continue;
        const float *colp = sx + (r + R) * TW + c;
        v[(size_t)y * W + x] = ypass_sym<R>(a.w, [&](int j) { return colp[j * TW]; });
    }
}

// sums[b] = fixed-order sum of the residual partials of image b's tiles.
__global__ __launch_bounds__(1024) void reduce_kernel(const double *partials, int tiles_per_img,
                                                      double *sums)
{
    __shared__ double sd[1024], sn[1024];
    const int b = blockIdx.x;
    const double *p = partials + 2 * (size_t)b * tiles_per_img;
    double d = 0.0, n = 0.0;
#pragma unroll 4
    for (int i = threadIdx.x; i < tiles_per_img; i += 1024) {
        d += p[2 * i];
        n += p[2 * i + 1];
    }
    sd[threadIdx.x] = d;
    sn[threadIdx.x] = n;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sd[threadIdx.x] += sd[threadIdx.x + s];
            sn[threadIdx.x] += sn[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sums[2 * b] = sd[0];
        sums[2 * b + 1] = sn[0];
    }
}

hipError_t launch_hold(float *u, const uint8_t *mask, const float *known, size_t n,
                       hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const size_t blocks = (n + 1023) / 1024;      // <= 2^26 for the largest batch
    hipLaunchKernelGGL(hold_kernel, dim3((unsigned)blocks), dim3(256), 0, s, u, mask, known, n);
    return hipGetLastError();
}

template <int R>
static int strip_oh(int shape)
{
    switch (shape) {
    case kShapeStripTall: return StripGeo<R, 136>::OH;
    case kShapeStripShort: return StripGeo<R, 28>::OH;
    case kShapeStripTiny: return StripGeo<R, 8>::OH;
    case kShapeStripWideShort: return StripGeo<R, 28, 2>::OH;
    case kShapeStripWide: return StripGeo<R, 64, 2>::OH;
    default: return StripGeo<R, 64>::OH;
    }
}

int strip_rows(int R, int shape)
{
    switch (R) {
#define EED4_CASE(r) case r: return strip_oh<r>(shape);
        EED4_CASE(0) EED4_CASE(1) EED4_CASE(2) EED4_CASE(3) EED4_CASE(4)
        EED4_CASE(5) EED4_CASE(6) EED4_CASE(7) EED4_CASE(8)
#undef EED4_CASE
    default: return 0;
    }
}

int tiles_per_image(int shape, int R, int H, int W)
{
    if (is_strip(shape)) {
        const int oh = strip_rows(R, shape), sw = strip_width(shape);
        if (oh <= 0) return 0;
        return ((W + sw - 1) / sw) * ((H + oh - 1) / oh);
    }
    const TileShape ts = kTileShapes[tile_index(shape)];
    return ((W + ts.tw - 1) / ts.tw) * ((H + ts.th - 1) / ts.th);
}

template <int R, int ROWS, int CPL = 1, bool GEN = false>
static hipError_t launch_strip_t(const float *ucur, const float *uprev, float *uout,
                                 const float *ref, const uint8_t *mask, int B, int H, int W,
                                 const StepArgs &a, double *partials, hipStream_t s)
{
    using G = StripGeo<R, ROWS, CPL>;
    const int nstrip = (W + G::SW - 1) / G::SW;
    const int per_img = nstrip * ((H + G::OH - 1) / G::OH);
    const long long nitems = (long long)per_img * B;
    const long long nblk = (nitems + 3) / 4;
    if (nitems <= 0 || nblk > 0x7fffffffLL) return hipErrorInvalidValue;
    static_assert(!GEN || (ROWS == 28 && CPL == 1), "tensor variants run 28-row strips");
    if constexpr (GEN) {
        if (ref)
            hipLaunchKernelGGL((strip_model_kernel<R, true>), dim3((unsigned)nblk), dim3(256), 0, s,
                               ucur, uprev, uout, ref, mask, H, W, nstrip, per_img, (int)nitems, a,
                               partials);
        else
            hipLaunchKernelGGL((strip_model_kernel<R, false>), dim3((unsigned)nblk), dim3(256), 0, s,
                               ucur, uprev, uout, ref, mask, H, W, nstrip, per_img, (int)nitems, a,
                               partials);
    } else if (ref) {
        hipLaunchKernelGGL((strip_kernel<R, true, ROWS, CPL>), dim3((unsigned)nblk), dim3(256), 0, s,
                           ucur, uprev, uout, ref, mask, H, W, nstrip, per_img, (int)nitems, a,
                           partials);
    } else {
        hipLaunchKernelGGL((strip_kernel<R, false, ROWS, CPL>), dim3((unsigned)nblk), dim3(256), 0, s,
                           ucur, uprev, uout, ref, mask, H, W, nstrip, per_img, (int)nitems, a,
                           partials);
    }
    return hipGetLastError();
}

template <int R, int ROWS, bool GEN>
static hipError_t launch_keepv_t(const float *ucur, const float *uprev, float *uout, float *vout,
                                 const uint8_t *mask, int B, int H, int W, const StepArgs &a,
                                 hipStream_t s)
{
    using G = StripGeo<R, ROWS, 1>;
    const int nstrip = (W + G::SW - 1) / G::SW;
    const int per_img = nstrip * ((H + G::OH - 1) / G::OH);
    const long long nitems = (long long)per_img * B;
    const long long nblk = (nitems + 3) / 4;
    if (nitems <= 0 || nblk > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((strip_keepv_kernel<R, ROWS, GEN>), dim3((unsigned)nblk), dim3(256), 0, s,
                       ucur, uprev, uout, vout, mask, H, W, nstrip, per_img, (int)nitems, a);
    return hipGetLastError();
}

// Strip height of the keep-v step for a forward step shape: tensor variants
// run 28-row strips; FOEED keeps the height of a strip shape (wide shapes map
// to their height) and runs 8-row strips in place of a tile shape (small
// images, where tiles win).
static int keepv_rows(int shape, int model)
{
    if (model != 0) return 28;
    switch (shape) {
    case kShapeStrip: case kShapeStripTall: case kShapeStripWide: return 64;
    case kShapeStripShort: case kShapeStripWideShort: return 28;
    default: return 8;
    }
}

template <int R>
static hipError_t launch_keepv_r(int shape, const float *ucur, const float *uprev, float *uout,
                                 float *vout, const uint8_t *mask, int B, int H, int W,
                                 const StepArgs &a, hipStream_t s)
{
    const int rows = keepv_rows(shape, a.model);
    if (a.model != 0) return launch_keepv_t<R, 28, true>(ucur, uprev, uout, vout, mask, B, H, W, a, s);
    if (rows == 64) return launch_keepv_t<R, 64, false>(ucur, uprev, uout, vout, mask, B, H, W, a, s);
    if (rows == 28) return launch_keepv_t<R, 28, false>(ucur, uprev, uout, vout, mask, B, H, W, a, s);
    return launch_keepv_t<R, 8, false>(ucur, uprev, uout, vout, mask, B, H, W, a, s);
}

template <int R>
static hipError_t launch_blur_r(const float *u, float *v, int B, int H, int W, const StepArgs &a,
                                hipStream_t s)
{
    const int nbx = (W + kBlurTW - 1) / kBlurTW, nby = (H + kBlurTH - 1) / kBlurTH;
    const long long ntiles = (long long)nbx * nby * B;
    if (ntiles <= 0 || ntiles > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((blur_kernel<R>), dim3((unsigned)ntiles), dim3(256), 0, s, u, v, H, W, nbx,
                       nbx * nby, a);
    return hipGetLastError();
}

template <int R, int TW, int TH>
static hipError_t launch_step_t(const float *ucur, const float *uprev, float *uout,
                                const float *ref, const uint8_t *mask, int B, int H, int W,
                                const StepArgs &a, double *partials, hipStream_t s)
{
    const int nbx = (W + TW - 1) / TW, nby = (H + TH - 1) / TH;
    const int tpi = nbx * nby;
    const long long ntiles = (long long)tpi * B;
    if (ntiles <= 0 || ntiles > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((step_kernel<R, TW, TH>), dim3((unsigned)ntiles), dim3(tile_threads(TW, TH)),
                       0, s, ucur,
                       uprev, uout, ref, mask, H, W, nbx, tpi, a, partials);
    return hipGetLastError();
}

template <int R>
static hipError_t launch_step_r(int shape, const float *ucur, const float *uprev, float *uout,
                                const float *ref, const uint8_t *mask, int B, int H, int W,
                                const StepArgs &a, double *partials, hipStream_t s)
{
    // tensor variants: one kernel shape (60-column strips of >= 28 rows)
    if (a.model != 0)
        return shape == kShapeStripShort
                   ? launch_strip_t<R, 28, 1, true>(ucur, uprev, uout, ref, mask, B, H, W, a, partials, s)
                   : hipErrorInvalidValue;
    switch (shape) {
    case 0: return launch_step_t<R, 64, 32>(ucur, uprev, uout, ref, mask, B, H, W, a, partials, s);
    case 1: return launch_step_t<R, 64, 16>(ucur, uprev, uout, ref, mask, B, H, W, a, partials, s);
    case 2: return launch_step_t<R, 32, 32>(ucur, uprev, uout, ref, mask, B, H, W, a, partials, s);
    case kShapeStrip: return launch_strip_t<R, 64>(ucur, uprev, uout, ref, mask, B, H, W, a, partials, s);
    case kShapeStripTall: return launch_strip_t<R, 136>(ucur, uprev, uout, ref, mask, B, H, W, a, partials, s);
    case kShapeStripShort: return launch_strip_t<R, 28>(ucur, uprev, uout, ref, mask, B, H, W, a, partials, s);
    case kShapeStripTiny: return launch_strip_t<R, 8>(ucur, uprev, uout, ref, mask, B, H, W, a, partials, s);
    case kShapeStripWide: return launch_strip_t<R, 64, 2>(ucur, uprev, uout, ref, mask, B, H, W, a, partials, s);
    case kShapeStripWideShort: return launch_strip_t<R, 28, 2>(ucur, uprev, uout, ref, mask, B, H, W, a, partials, s);
    case kShapeTile32x16: return launch_step_t<R, 32, 16>(ucur, uprev, uout, ref, mask, B, H, W, a, partials, s);
    case kShapeTile16x16: return launch_step_t<R, 16, 16>(ucur, uprev, uout, ref, mask, B, H, W, a, partials, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step(int R, int shape, const float *ucur, const float *uprev, float *uout,
                       const float *ref, const uint8_t *mask, int B, int H, int W,
                       const StepArgs &a, double *partials, hipStream_t s)
{
    switch (R) {
#define EED4_CASE(r) \
    case r: return launch_step_r<r>(shape, ucur, uprev, uout, ref, mask, B, H, W, a, partials, s);
        EED4_CASE(0) EED4_CASE(1) EED4_CASE(2) EED4_CASE(3) EED4_CASE(4)
        EED4_CASE(5) EED4_CASE(6) EED4_CASE(7) EED4_CASE(8)
#undef EED4_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_keepv(int R, int shape, const float *ucur, const float *uprev,
                             float *uout, float *vout, const uint8_t *mask, int B, int H, int W,
                             const StepArgs &a, hipStream_t s)
{
    switch (R) {
#define EED4_CASE(r) \
    case r: return launch_keepv_r<r>(shape, ucur, uprev, uout, vout, mask, B, H, W, a, s);
        EED4_CASE(0) EED4_CASE(1) EED4_CASE(2) EED4_CASE(3) EED4_CASE(4)
        EED4_CASE(5) EED4_CASE(6) EED4_CASE(7) EED4_CASE(8)
#undef EED4_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_blur(int R, const float *u, float *v, int B, int H, int W, const StepArgs &a,
                       hipStream_t s)
{
    switch (R) {
#define EED4_CASE(r) case r: return launch_blur_r<r>(u, v, B, H, W, a, s);
        EED4_CASE(0) EED4_CASE(1) EED4_CASE(2) EED4_CASE(3) EED4_CASE(4)
        EED4_CASE(5) EED4_CASE(6) EED4_CASE(7) EED4_CASE(8)
#undef EED4_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_reduce(const double *partials, int tiles_per_img, int B, double *sums,
                         hipStream_t s)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(B), dim3(1024), 0, s, partials, tiles_per_img, sums);
    return hipGetLastError();
}

}  // namespace eed4
