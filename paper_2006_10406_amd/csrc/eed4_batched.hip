// Batched inpainting of images of uneven sizes: one launch per inner FSI step
// over a work queue spanning every image, the cycle captured once as a
// hipGraph, per-image stop, and an autotuner that picks the kernel shape
// (workgroup tiles, or wave strips of four heights and two widths) by timing
// one step on the actual batch.
//
// The queue holds one entry per work item (a tile of a workgroup, or a strip
// segment of a wave) of every image still iterating.  A launch has one wave or
// workgroup per item of the full queue and walks the queue with a static
// stride (a no-op loop unless the grid is smaller than the queue); every XCD
// takes contiguous runs of items, so neighbouring items share its L2.  (A
// global atomic work counter was tried first: with one device-scope counter
// for all XCDs the pulls serialise and the step took twice as long.  A grid
// capped at the resident capacity was tried next: where the kernel's occupancy
// left fewer wave slots than items, some waves took a second item after the
// others had finished, which cost a third on the 64-image batch.)  The queue
// length lives in device memory: dropping a converged image rewrites the queue
// without re-capturing the graph; waves past its end exit at once.
#include "eed4.h"
#include "eed4_host.h"
#include "eed4_internal.h"
#include "eed4_strip.h"
#include "eed4_tile.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

namespace eed4 {

struct BImage {            // device-side image descriptor
    float *buf[3];         // S (caller's u), X, Y
    const uint8_t *mask;
    int H, W;
    float inv_lam2;
    int nx;                // work items per row of items
};

struct BItem {             // one queue entry
    int img, iy, ix, slot; // item row / column inside the image; residual slot
};

__device__ __forceinline__ float *pick(const BImage &d, int sel)
{
    return sel == 0 ? d.buf[0] : (sel == 1 ? d.buf[1] : d.buf[2]);
}

// Wave-uniform copies of values loaded from the queue and the descriptors.
// The loads use a uniform address, but their results land in VGPRs; buffer
// resources built from them would make the compiler wrap every buffer access
// in a loop over distinct lane values.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
template <typename T>
__device__ __forceinline__ T *uni(T *p)
{
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (T *)(((unsigned long long)hi << 32) | lo);
}

// Wave-strip shapes: wave w of the launch takes items w, w + nw, w + 2 nw, ...
// (w counted in XCD-contiguous order).  GEN: tensor variant chosen at run time.
template <int R, int ROWS, bool RES, int CPL, bool GEN>
__device__ __forceinline__ void bstrip_body(const BImage *imgs, const BItem *queue,
                                            const int *qlen_p, int sc, int sp, int so,
                                            const StepArgs &a, double *partials)
{
    using G = StripGeo<R, ROWS, CPL>;
    __shared__ float lds[4 * G::LDS];
    const int wave = threadIdx.x >> 6;
    const int nw = 4 * gridDim.x;
    const int w0 = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * 4 + wave);
    const int qlen = *qlen_p;
    for (int it = w0; it < qlen; it += nw) {
        const BItem t = queue[it];
        const BImage d = imgs[t.img];
        StripArgs s;
        s.ucur = uni(pick(d, sc));
        s.uprev = uni(pick(d, sp));
        s.uout = uni(pick(d, so));
        s.ref = uni(d.buf[0]);
        s.mask = uni(d.mask);
        s.H = uni(d.H);
        s.W = uni(d.W);
        s.X0 = uni(t.ix) * G::SW;
        s.Y0 = uni(t.iy) * G::OH;
        s.tau = a.tau;
        s.alpha = a.alpha;
        s.il2q = 0.25f * __int_as_float(uni(__float_as_int(d.inv_lam2)));
        s.model = a.model;
        s.up = strip_alternates(ROWS) ? uni(t.iy) & 1 : 0;   // as in the single-image kernels
        strip_step<R, RES, ROWS, CPL, GEN>(lds + wave * G::LDS, s, a.w,
                                           partials + 2 * (size_t)uni(t.slot));
    }
}

template <int R, int ROWS, bool RES, int CPL>
__global__ __launch_bounds__(256) void bstrip_kernel(const BImage *imgs, const BItem *queue,
                                                     const int *qlen_p, int sc, int sp, int so,
                                                     StepArgs a, double *partials)
{
    bstrip_body<R, ROWS, RES, CPL, false>(imgs, queue, qlen_p, sc, sp, so, a, partials);
}

// The tensor variants (diffusivities of Table 7, mu3 choices of Sec. 3.1) on
// 60-column strips of >= 28 rows.
template <int R, bool RES>
__global__ __launch_bounds__(256) void bstrip_model_kernel(const BImage *imgs, const BItem *queue,
                                                           const int *qlen_p, int sc, int sp,
                                                           int so, StepArgs a, double *partials)
{
    bstrip_body<R, 28, RES, 1, true>(imgs, queue, qlen_p, sc, sp, so, a, partials);
}

// Workgroup-tile shapes: workgroup g takes tiles g, g + G, g + 2 G, ...
template <int R, int TW, int TH>
__global__ __launch_bounds__(tile_threads(TW, TH)) void btile_kernel(
    const BImage *imgs, const BItem *queue, const int *qlen_p, int sc, int sp, int so,
    int residual, StepArgs a, double *partials)
{
    constexpr int NTH = tile_threads(TW, TH);
    __shared__ __attribute__((aligned(16))) float smem[TileGeo<R, TW, TH, NTH>::SMEM];
    const int qlen = *qlen_p;
    for (int it = xcd_tile(blockIdx.x, gridDim.x); it < qlen; it += gridDim.x) {
        __syncthreads();           // the previous tile's last LDS reads are done
        const BItem t = queue[it];
        const BImage d = imgs[t.img];
        step_tile<R, TW, TH, NTH>(smem, uni(pick(d, sc)), uni(pick(d, sp)), uni(pick(d, so)),
                                  residual ? uni(d.buf[0]) : nullptr, uni(d.mask), uni(d.H),
                                  uni(d.W), uni(t.iy), uni(t.ix), a.w, a.tau, a.alpha,
                                  0.25f * __int_as_float(uni(__float_as_int(d.inv_lam2))),
                                  residual ? partials + 2 * (size_t)uni(t.slot) : nullptr);
    }
}

// Copy X -> S over the items of the queue (cycles of length 1 end in X).
__global__ __launch_bounds__(256) void bcopy_kernel(const BImage *imgs, const BItem *queue,
                                                    const int *qlen_p, int tw, int th)
{
    const int qlen = *qlen_p;
    for (int it = blockIdx.x; it < qlen; it += gridDim.x) {
        const BItem t = queue[it];
        const BImage d = imgs[t.img];
        const int x0 = t.ix * tw, y0 = t.iy * th;
        for (int i = threadIdx.x; i < tw * th; i += blockDim.x) {
            int y = y0 + i / tw, x = x0 + i % tw;
            if (y < d.H && x < d.W) {
                size_t gi = (size_t)y * d.W + x;
                d.buf[0][gi] = d.buf[1][gi];
            }
        }
    }
}

// sums[b] = fixed-order sum of the partials of image b's items
__global__ __launch_bounds__(256) void breduce_kernel(const double *partials, const int *slot0,
                                                      const int *nslot, double *sums)
{
    __shared__ double sd[256], sn[256];
    const int b = blockIdx.x;
    const double *p = partials + 2 * (size_t)slot0[b];
    const int n = nslot[b];
    double d = 0.0, q = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        d += p[2 * i];
        q += p[2 * i + 1];
    }
    sd[threadIdx.x] = d;
    sn[threadIdx.x] = q;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
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

__global__ __launch_bounds__(256) void bhold_kernel(float *u, const uint8_t *__restrict__ mask,
                                                    const float *__restrict__ known, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        if (mask[i]) u[i] = known[i];
}

// ---------------------------------------------------------------- host side

// item size of a shape in pixels
static void item_dims(int shape, int R, int *iw, int *ih)
{
    if (is_strip(shape)) {
        *iw = strip_width(shape);
        *ih = strip_rows(R, shape);
        return;
    }
    *iw = kTileShapes[tile_index(shape)].tw;
    *ih = kTileShapes[tile_index(shape)].th;
}

template <int R>
static hipError_t launch_bstep_r(int shape, int grid, const BImage *imgs, const BItem *queue,
                                 const int *qlen, int sc, int sp, int so, bool res,
                                 const StepArgs &a, double *partials, hipStream_t s)
{
    dim3 g(grid), b(256);
#define EED4_BTILE(TW, TH)                                                                   \
    hipLaunchKernelGGL((btile_kernel<R, TW, TH>), g, dim3(tile_threads(TW, TH)), 0, s, imgs, \
                       queue, qlen, sc, sp, so, res ? 1 : 0, a, partials)
#define EED4_BSTRIP(ROWS, CPL)                                                           \
    if (res)                                                                             \
        hipLaunchKernelGGL((bstrip_kernel<R, ROWS, true, CPL>), g, b, 0, s, imgs, queue, \
                           qlen, sc, sp, so, a, partials);                               \
    else                                                                                 \
        hipLaunchKernelGGL((bstrip_kernel<R, ROWS, false, CPL>), g, b, 0, s, imgs, queue, \
                           qlen, sc, sp, so, a, partials)
    if (a.model != 0) {              // tensor variants: one kernel shape
        if (shape != kShapeStripShort) return hipErrorInvalidValue;
        if (res)
            hipLaunchKernelGGL((bstrip_model_kernel<R, true>), g, b, 0, s, imgs, queue, qlen, sc,
                               sp, so, a, partials);
        else
            hipLaunchKernelGGL((bstrip_model_kernel<R, false>), g, b, 0, s, imgs, queue, qlen, sc,
                               sp, so, a, partials);
        return hipGetLastError();
    }
    switch (shape) {
    case 0: EED4_BTILE(64, 32); break;
    case 1: EED4_BTILE(64, 16); break;
    case 2: EED4_BTILE(32, 32); break;
    case kShapeStrip: EED4_BSTRIP(64, 1); break;
    case kShapeStripTall: EED4_BSTRIP(136, 1); break;
    case kShapeStripShort: EED4_BSTRIP(28, 1); break;
    case kShapeStripTiny: EED4_BSTRIP(8, 1); break;
    case kShapeStripWide: EED4_BSTRIP(64, 2); break;
    case kShapeStripWideShort: EED4_BSTRIP(28, 2); break;
    case kShapeTile32x16: EED4_BTILE(32, 16); break;
    case kShapeTile16x16: EED4_BTILE(16, 16); break;
    default: return hipErrorInvalidValue;
    }
#undef EED4_BTILE
#undef EED4_BSTRIP
    return hipGetLastError();
}

static hipError_t launch_bstep(int R, int shape, int grid, const BImage *imgs, const BItem *queue,
                               const int *qlen, int sc, int sp, int so, bool res,
                               const StepArgs &a, double *partials, hipStream_t s)
{
    switch (R) {
#define EED4_CASE(r) \
    case r: return launch_bstep_r<r>(shape, grid, imgs, queue, qlen, sc, sp, so, res, a, partials, s);
        EED4_CASE(0) EED4_CASE(1) EED4_CASE(2) EED4_CASE(3) EED4_CASE(4)
        EED4_CASE(5) EED4_CASE(6) EED4_CASE(7) EED4_CASE(8)
#undef EED4_CASE
    default: return hipErrorInvalidValue;
    }
}

struct BatchLayout {
    std::vector<size_t> X, Y;
    size_t imgs, queue, qlen, partials, slot0, nslot, sums, total;
};

static int max_items(int B, const eed4_image *im, int R)
{
    int m = 0;
    for (int sh = 0; sh < kNumShapes; ++sh) {
        long long t = 0;
        for (int i = 0; i < B; ++i) t += tiles_per_image(sh, R, im[i].H, im[i].W);
        if (t > m) m = (int)std::min<long long>(t, 0x7fffffff);
    }
    return m;
}

static BatchLayout batch_layout(const eed4_image *im, int B, const eed4_params *p)
{
    BatchLayout L;
    const int R = eed4_radius(p->sigma);
    size_t o = 0;
    L.X.resize(B);
    L.Y.resize(B);
    for (int i = 0; i < B; ++i) {
        size_t n = (size_t)im[i].H * im[i].W;
        L.X[i] = o; o = align_up(o + sizeof(float) * n);
        L.Y[i] = o; o = align_up(o + sizeof(float) * n);
    }
    const size_t items = (size_t)max_items(B, im, R);
    L.imgs = o; o = align_up(o + sizeof(BImage) * (size_t)B);
    L.queue = o; o = align_up(o + sizeof(BItem) * items);
    L.qlen = o; o = align_up(o + sizeof(int));
    L.partials = o; o = align_up(o + sizeof(double) * 2 * items);
    L.slot0 = o; o = align_up(o + sizeof(int) * (size_t)B);
    L.nslot = o; o = align_up(o + sizeof(int) * (size_t)B);
    L.sums = o; o = align_up(o + sizeof(double) * 2 * (size_t)B);
    L.total = o;
    return L;
}

static int check_images(const eed4_image *im, int B, const eed4_params *p)
{
    if (!im || B < 1 || !p) return EED4_EINVAL;
    for (int i = 0; i < B; ++i) {
        if (!im[i].u || !im[i].mask || !im[i].known) return EED4_EINVAL;
        eed4_params q = *p;
        q.lambda = im[i].lambda;
        int rc = check_params(&q, 1, im[i].H, im[i].W);
        if (rc != EED4_OK) return rc;
    }
    return EED4_OK;
}

// Everything a batched run needs on the device, for one kernel shape.
struct BatchRun {
    int R, shape, grid, n, B;
    int iw, ih;                      // item size in pixels
    std::vector<BImage> himg;
    std::vector<int> slot0, nslot;   // residual slots per image
    std::vector<BItem> queue;        // items of the active images
    BImage *dimg;
    BItem *dqueue;
    int *dqlen, *dslot0, *dnslot;
    double *dpartials, *dsums;
    const eed4_params *p;
};

static void build_queue(BatchRun &r, const std::vector<char> &active)
{
    r.queue.clear();
    for (int i = 0; i < r.B; ++i) {
        if (!active[i]) continue;
        const int nx = (r.himg[i].W + r.iw - 1) / r.iw, ny = (r.himg[i].H + r.ih - 1) / r.ih;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) r.queue.push_back({i, y, x, r.slot0[i] + y * nx + x});
    }
}

static int upload_queue(BatchRun &r, hipStream_t s)
{
    int ql = (int)r.queue.size();
    hipError_t e = hipMemcpyAsync(r.dqueue, r.queue.data(), sizeof(BItem) * r.queue.size(),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(r.dqlen, &ql, sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // host buffers are stack/vector owned
    return e == hipSuccess ? EED4_OK : hip_fail(e, "queue upload");
}

static int prepare(BatchRun &r, const eed4_image *im, int B, const eed4_params *p, int shape,
                   char *base, const BatchLayout &L, hipStream_t s)
{
    r.R = eed4_radius(p->sigma);
    r.shape = shape;
    r.n = p->cycle_len;
    r.B = B;
    r.p = p;
    item_dims(shape, r.R, &r.iw, &r.ih);
    r.himg.resize(B);
    r.slot0.resize(B);
    r.nslot.resize(B);
    int slot = 0;
    for (int i = 0; i < B; ++i) {
        BImage d;
        d.buf[0] = im[i].u;
        d.buf[1] = (float *)(base + L.X[i]);
        d.buf[2] = (float *)(base + L.Y[i]);
        d.mask = im[i].mask;
        d.H = im[i].H;
        d.W = im[i].W;
        d.inv_lam2 = (float)(1.0 / ((double)im[i].lambda * (double)im[i].lambda));
        d.nx = (im[i].W + r.iw - 1) / r.iw;
        r.himg[i] = d;
        r.slot0[i] = slot;
        r.nslot[i] = tiles_per_image(shape, r.R, im[i].H, im[i].W);
        slot += r.nslot[i];
    }
    r.dimg = (BImage *)(base + L.imgs);
    r.dqueue = (BItem *)(base + L.queue);
    r.dqlen = (int *)(base + L.qlen);
    r.dslot0 = (int *)(base + L.slot0);
    r.dnslot = (int *)(base + L.nslot);
    r.dpartials = (double *)(base + L.partials);
    r.dsums = (double *)(base + L.sums);
    hipError_t e = hipMemcpyAsync(r.dimg, r.himg.data(), sizeof(BImage) * B,
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(r.dslot0, r.slot0.data(), sizeof(int) * B, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(r.dnslot, r.nslot.data(), sizeof(int) * B, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "descriptor upload");
    std::vector<char> active(B, 1);
    build_queue(r, active);
    // one wave (strip) or workgroup (tile) per item of the full queue; the
    // hardware dispatcher balances them.  Later cycles may have fewer items:
    // the waves past the queue length exit at once.
    const int ql = (int)r.queue.size();
    r.grid = std::max(1, is_strip(shape) ? (ql + 3) / 4 : ql);
    return upload_queue(r, s);
}

// Roles of S (0), X (1), Y (2) in step k of a cycle of n (as cycle_roles).
static void roles(int k, int n, int *sc, int *sp, int *so)
{
    if (k == 0) { *sc = 0; *sp = 0; *so = 1; }
    else {
        *sc = (k & 1) ? 1 : 2;
        *sp = (k == 1) ? 0 : ((k & 1) ? 2 : 1);
        *so = (k & 1) ? 2 : 1;
    }
    if (k == n - 1 && n > 1) *so = 0;
}

static int enqueue_bcycle(const BatchRun &r, hipStream_t s)
{
    hipError_t e;
    for (int k = 0; k < r.n; ++k) {
        int sc, sp, so;
        roles(k, r.n, &sc, &sp, &so);
        StepArgs a = make_args(r.p->sigma, r.R, r.p->tau, 1.0f, k, model_of_flags(r.p->flags));
        e = launch_bstep(r.R, r.shape, r.grid, r.dimg, r.dqueue, r.dqlen, sc, sp,
                         so, k == r.n - 1, a, r.dpartials, s);
        if (e != hipSuccess) return hip_fail(e, "batched step launch");
    }
    if (r.n == 1) {
        hipLaunchKernelGGL(bcopy_kernel, dim3(1024), dim3(256), 0, s, r.dimg, r.dqueue, r.dqlen,
                           r.iw, r.ih);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "batched copy");
    }
    hipLaunchKernelGGL(breduce_kernel, dim3(r.B), dim3(256), 0, s, r.dpartials, r.dslot0,
                       r.dnslot, r.dsums);
    e = hipGetLastError();
    return e == hipSuccess ? EED4_OK : hip_fail(e, "batched reduce");
}

// ---- autotuner (the choice cache is shared with the single-image path) ----
static std::string batch_tune_key(const eed4_image *im, int B, int R)
{
    double px = 0;
    int minside = 1 << 30, maxside = 0;
    for (int i = 0; i < B; ++i) {
        px += (double)im[i].H * im[i].W;
        minside = std::min(minside, std::min(im[i].H, im[i].W));
        maxside = std::max(maxside, std::max(im[i].H, im[i].W));
    }
    char buf[128];
    std::snprintf(buf, sizeof(buf), "batched_R%d_B%d_px2^%d_side2^%d-%d", R, B,
                  (int)std::lround(std::log2(px + 1)), (int)std::lround(std::log2(minside)),
                  (int)std::lround(std::log2(maxside)));
    return buf;
}

// Times one inner step (k = 0: S -> X, S unchanged) of every shape on the batch.
static int autotune(const eed4_image *im, int B, const eed4_params *p, char *base,
                    const BatchLayout &L, hipStream_t s, int *best_shape, float *best_ms)
{
    int order[kNumShapes];
    tune_order(kShapeStrip, order);
    BatchRun r;
    StepArgs a;
    return tune_pick(
        order, kNumShapes, s,
        [&](int sh) {
            r = BatchRun();
            const int rc = prepare(r, im, B, p, sh, base, L, s);
            a = make_args(p->sigma, r.R, p->tau, 1.0f, 0);
            return rc;
        },
        [&](int sh) {
            return launch_bstep(r.R, sh, r.grid, r.dimg, r.dqueue, r.dqlen, 0, 0, 1, false, a,
                                r.dpartials, s);
        },
        "autotune timing", best_shape, best_ms);
}

static int choose_shape(const eed4_image *im, int B, const eed4_params *p, char *base,
                        const BatchLayout &L, hipStream_t s, int *shape)
{
    if (model_of_flags(p->flags) != 0) {   // the tensor-variant kernel
        *shape = kShapeStripShort;
        return EED4_OK;
    }
    const int forced = (p->flags >> 8) & 0xff;
    if (forced) {
        if (forced > kNumShapes) return EED4_EINVAL;
        *shape = forced - 1;
        return EED4_OK;
    }
    const std::string key = batch_tune_key(im, B, eed4_radius(p->sigma));
    if (tune_lookup(key, shape)) return EED4_OK;
    float ms = 0.0f;
    int rc = autotune(im, B, p, base, L, s, shape, &ms);
    if (rc != EED4_OK) return rc;
    tune_remember(key, *shape);
    return EED4_OK;
}

}  // namespace eed4

using namespace eed4;

extern "C" size_t eed4_batched_workspace_size(const eed4_image *imgs, int B, const eed4_params *p)
{
    if (check_images(imgs, B, p) != EED4_OK) return 0;
    return batch_layout(imgs, B, p).total;
}

extern "C" int eed4_autotune_batched(const eed4_image *imgs, int B, const eed4_params *p,
                                     void *ws, size_t ws_bytes, void *stream)
{
    TraceRange range("eed4_autotune_batched %d images", B);
    int rc = check_images(imgs, B, p);
    if (rc != EED4_OK) return rc;
    BatchLayout L = batch_layout(imgs, B, p);
    if ((rc = check_ws(ws, ws_bytes, L.total)) != EED4_OK) return rc;
    if (model_of_flags(p->flags) != 0) return kShapeStripShort;   // one kernel for variants
    int shape = 0;
    float ms = 0.0f;
    rc = autotune(imgs, B, p, (char *)ws, L, (hipStream_t)stream, &shape, &ms);
    if (rc != EED4_OK) return rc;
    tune_remember(batch_tune_key(imgs, B, eed4_radius(p->sigma)), shape);
    return shape;
}

extern "C" int eed4_inpaint_batched(const eed4_image *imgs, int B, const eed4_params *p, void *ws,
                                    size_t ws_bytes, void *stream, eed4_stats *stats)
{
    TraceRange range("eed4_inpaint_batched %d images, up to %d cycles of %d", B,
                     p ? p->max_cycles : 0, p ? p->cycle_len : 0);
    int rc = check_images(imgs, B, p);
    if (rc != EED4_OK) return rc;
    BatchLayout L = batch_layout(imgs, B, p);
    if ((rc = check_ws(ws, ws_bytes, L.total)) != EED4_OK) return rc;
    char *base = (char *)ws;
    hipStream_t s = (hipStream_t)stream;

    for (int i = 0; i < B; ++i) {
        size_t n = (size_t)imgs[i].H * imgs[i].W;
        unsigned g = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
        hipLaunchKernelGGL(bhold_kernel, dim3(g), dim3(256), 0, s, imgs[i].u, imgs[i].mask,
                           imgs[i].known, n);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "hold launch");

    int shape = kShapeStrip;
    if ((rc = choose_shape(imgs, B, p, base, L, s, &shape)) != EED4_OK) return rc;
    BatchRun r;
    if ((rc = prepare(r, imgs, B, p, shape, base, L, s)) != EED4_OK) return rc;

    hipGraphExec_t exec = nullptr;
    if (!(p->flags & EED4_NO_GRAPH)) {
        rc = capture_graph([&](hipStream_t cs) { return enqueue_bcycle(r, cs); }, &exec);
        if (rc != EED4_OK) return rc;
    }

    const int M = p->max_cycles;
    std::vector<char> active(B, 1);
    std::vector<double> host(2 * (size_t)B);
    std::vector<eed4_stats> st(B);
    for (int i = 0; i < B; ++i) st[i] = {0, 0.0, 0.0};
    int nactive = B;
    bool diverged = false;
    for (int m = 0; m < M && nactive > 0 && rc == EED4_OK; ++m) {
        if (exec) {
            e = hipGraphLaunch(exec, s);
            if (e != hipSuccess) { rc = hip_fail(e, "graph launch"); break; }
        } else if ((rc = enqueue_bcycle(r, s)) != EED4_OK) {
            break;
        }
        const bool need = p->tol > 0.0f || m == M - 1;
        if (!need) {
            for (int i = 0; i < B; ++i)
                if (active[i]) st[i].cycles = m + 1;
            continue;
        }
        e = hipMemcpyAsync(host.data(), r.dsums, sizeof(double) * 2 * B, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { rc = hip_fail(e, "residual read-back"); break; }
        bool changed = false;
        for (int i = 0; i < B; ++i) {
            if (!active[i]) continue;
            const double res = std::sqrt(host[2 * i]), nn = std::sqrt(host[2 * i + 1]);
            st[i].cycles = m + 1;
            st[i].residual = res;
            st[i].rel_residual = nn > 0.0 ? res / nn : res;
            if (!std::isfinite(res) || !std::isfinite(nn)) diverged = true;
            const double crit = (p->flags & EED4_ABS_TOL) ? st[i].residual : st[i].rel_residual;
            if (p->tol > 0.0f && crit < (double)p->tol) {
                active[i] = 0;
                --nactive;
                changed = true;
            }
        }
        if (diverged) break;
        if (changed && nactive > 0) {
            build_queue(r, active);
            rc = upload_queue(r, s);
        }
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (rc != EED4_OK) return rc;
    if (stats)
        for (int i = 0; i < B; ++i) stats[i] = st[i];
    return diverged ? EED4_EDIVERGED : EED4_OK;
}
