// Host side of libeed4: argument checks, workspace layout, the FSI cycle
// driver (buffer rotation, hipGraph capture and replay, residual read-back
// and stop rule) and the C ABI entry points declared in include/eed4.h.
#include "eed4.h"
#include "eed4_internal.h"
#include "eed4_host.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

namespace eed4 {

thread_local std::string g_last_hip;

int hip_fail(hipError_t e, const char *where)
{
    g_last_hip = std::string(where) + ": " + hipGetErrorString(e);
    return EED4_EHIP;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int check_params(const eed4_params *p, int B, int H, int W)
{
    if (!p || B < 1 || H < 1 || W < 1) return EED4_EINVAL;
    // W bound: a strip addresses up to 169 rows of one plane with a 32-bit
    // byte offset that must stay below 2^31
    if (H > (1 << 24) || W > (1 << 21)) return EED4_EINVAL;
    if ((long long)H * W > (1LL << 31) || (long long)B * H * W > (1LL << 36)) return EED4_EINVAL;
    if (!(p->lambda > 0.0f) || !std::isfinite(p->lambda)) return EED4_EINVAL;
    if (eed4_radius(p->sigma) < 0) return EED4_EINVAL;
    if (!(p->tau > 0.0f) || !std::isfinite(p->tau)) return EED4_EINVAL;
    if (p->cycle_len < 1 || p->max_cycles < 1) return EED4_EINVAL;
    if (!(p->tol >= 0.0f) || !std::isfinite(p->tol)) return EED4_EINVAL;
    const int forced = (p->flags >> 8) & 0xff;
    if (forced > kNumShapes) return EED4_EINVAL;
    if (((p->flags >> 16) & 0xf) >= kNumDiffusivities || ((p->flags >> 20) & 0x3) >= kNumMu3Rules)
        return EED4_EINVAL;
    // a tensor variant runs one kernel shape (the 28-row strips)
    if (model_of_flags(p->flags) != 0 &&
        ((forced && forced - 1 != kShapeStripShort) || (p->flags & EED4_TILE_KERNEL)))
        return EED4_EINVAL;
    if (!(p->flags & EED4_ALLOW_LARGE_TAU) && (double)p->tau > 1.0 / 16.0) return EED4_EUNSTABLE;
    return EED4_OK;
}

StepArgs make_args(float sigma, int R, float tau, float lambda, int k, int model)
{
    StepArgs a;
    std::memset(&a, 0, sizeof(a));
    if (R == 0) {
        a.w[0] = 1.0f;
    } else {
        double s = (double)sigma, w[2 * kRMax + 1], sum = 0.0;
        for (int j = -R; j <= R; ++j) {
            w[j + R] = std::exp(-(double)(j * j) / (2.0 * s * s));
            sum += w[j + R];
        }
        for (int j = 0; j <= 2 * R; ++j) a.w[j] = (float)(w[j] / sum);
    }
    a.tau = tau;
    a.alpha = (float)((4.0 * k + 2.0) / (2.0 * k + 3.0));
    a.inv_lam2 = (float)(1.0 / ((double)lambda * (double)lambda));
    a.model = model;
    return a;
}

// One library-owned, non-blocking, default-priority stream per device and
// role (0: graph capture, 1: the backward's recompute).
static hipStream_t library_stream(int role)
{
    static std::mutex mu;
    static std::vector<hipStream_t> streams[2];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    std::vector<hipStream_t> &v = streams[role];
    if ((int)v.size() <= dev) v.resize(dev + 1, nullptr);
    if (!v[dev]) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
        v[dev] = s;
    }
    return v[dev];
}

hipStream_t capture_stream() { return library_stream(0); }
hipStream_t recompute_stream() { return library_stream(1); }

// Rotation of the three state buffers over one cycle: S (cycle start and
// result), X, Y.  Step k reads cur = u^k (with halo) and prev = u^{k-1}
// (pointwise) and writes out = u^{k+1}; out may alias prev because both are
// touched only at the thread's own pixel.  The last step writes S while
// reading S pointwise for the residual.
void cycle_roles(int k, int n, float *S, float *X, float *Y, float **cur, float **prev,
                 float **out)
{
    if (k == 0) {
        *cur = S; *prev = S; *out = X;
    } else {
        *cur = (k & 1) ? X : Y;
        *prev = (k == 1) ? S : ((k & 1) ? Y : X);
        *out = (k & 1) ? Y : X;
    }
    if (k == n - 1 && n > 1) *out = S;
}

int enqueue_cycle(const CycleJob &j, hipStream_t s)
{
    const int n = j.n;
    float *const dst = j.Out ? j.Out : j.S;
    for (int k = 0; k < n; ++k) {
        float *cur, *prev, *out;
        cycle_roles(k, n, j.S, j.X, j.Y, &cur, &prev, &out);
        const bool last = (k == n - 1);
        if (last && (n > 1 || dst != j.S)) out = dst;
        StepArgs a = make_args(j.sigma, j.R, j.tau, j.lambda, k, j.model);
        hipError_t e = launch_step(j.R, j.shape, cur, prev, out, last ? j.S : nullptr, j.mask,
                                   j.B, j.H, j.W, a, last ? j.partials : nullptr, s);
        if (e != hipSuccess) return hip_fail(e, "fsi step launch");
    }
    if (n == 1 && dst == j.S) {
        hipError_t e = hipMemcpyAsync(j.S, j.X, sizeof(float) * (size_t)j.B * j.H * j.W,
                                      hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "cycle copy");
    }
    hipError_t e = launch_reduce(j.partials, tiles_per_image(j.shape, j.R, j.H, j.W), j.B, j.sums, s);
    if (e != hipSuccess) return hip_fail(e, "residual reduce launch");
    return EED4_OK;
}

// Records what `enqueue` puts on the library's capture stream into an
// executable graph.  That stream is shared by all host threads of the process,
// so captures are serialised; a capture only records launches.
int capture_graph(const std::function<int(hipStream_t)> &enqueue, hipGraphExec_t *exec)
{
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    *exec = nullptr;
    hipStream_t cs = capture_stream();
    if (!cs) return hip_fail(hipErrorInvalidValue, "capture stream");
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "begin capture");
    int rc = enqueue(cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    if (rc != EED4_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "graph instantiate");
    return EED4_OK;
}

int capture_cycle(const CycleJob &j, hipGraphExec_t *exec, int nc)
{
    return capture_graph(
        [&](hipStream_t cs) {
            for (int c = 0; c < nc; ++c) {
                const int rc = enqueue_cycle(j, cs);
                if (rc != EED4_OK) return rc;
            }
            return (int)EED4_OK;
        },
        exec);
}

// Instantiated cycle graphs of eed4_inpaint, kept across calls.  A graph
// records only kernel launches and their arguments, so a later call whose job
// has the same device, buffers, sizes, shape and step parameters replays it
// without a new capture and instantiation.  The cache is bounded; beyond
// kMaxCachedGraphs jobs a call captures its own graph and destroys it at the
// end, as without the cache.  Entries are never evicted (a launch of an
// evicted graph might still be in flight on another stream).
constexpr size_t kMaxCachedGraphs = 64;
constexpr int kGraphCycles = 4;    // cycles per graph when no host work sits between cycles

struct CycleKey {
    int dev, nc;                   // device, cycles per graph
    const void *S, *X, *Y, *Out, *mask, *partials, *sums;
    int B, H, W, R, shape, n, model;
    float sigma, tau, lambda;      // finite (checked), so < is a strict order
    auto tie() const
    {
        return std::tie(dev, nc, S, X, Y, Out, mask, partials, sums, B, H, W, R, shape, n,
                        model, sigma, tau, lambda);
    }
    bool operator<(const CycleKey &o) const { return tie() < o.tie(); }
};

static std::mutex g_graph_mu;
static std::map<CycleKey, hipGraphExec_t> g_graphs;

// The executable graph of nc cycles of job j: from the cache, or captured now
// (and cached when there is room).  *owned tells the caller to destroy it
// after use.
int cycle_graph(const CycleJob &j, int nc, hipGraphExec_t *exec, bool *owned)
{
    CycleKey k;
    k.nc = nc;
    hipError_t e = hipGetDevice(&k.dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    k.S = j.S; k.X = j.X; k.Y = j.Y; k.Out = j.Out ? j.Out : j.S; k.mask = j.mask;
    k.partials = j.partials; k.sums = j.sums;
    k.B = j.B; k.H = j.H; k.W = j.W; k.R = j.R; k.shape = j.shape; k.n = j.n; k.model = j.model;
    k.sigma = j.sigma; k.tau = j.tau; k.lambda = j.lambda;
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        auto it = g_graphs.find(k);
        if (it != g_graphs.end()) {
            *exec = it->second;
            *owned = false;
            return EED4_OK;
        }
    }
    int rc = capture_cycle(j, exec, nc);
    if (rc != EED4_OK) return rc;
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(k);
    if (it != g_graphs.end()) {          // another thread cached the same job meanwhile
        *owned = true;
    } else if (g_graphs.size() < kMaxCachedGraphs) {
        g_graphs.emplace(k, *exec);
        *owned = false;
    } else {
        *owned = true;
    }
    return EED4_OK;
}

struct InpaintLayout {
    size_t X, Y, T, partials, sums, hist, total;
};

// residual partials: enough for the largest per-image count of any kernel shape
int max_partials_per_image(int R, int H, int W)
{
    int m = 0;
    for (int sh = 0; sh < kNumShapes; ++sh) {
        int t = tiles_per_image(sh, R, H, W);
        if (t > m) m = t;
    }
    return m;
}

InpaintLayout inpaint_layout(int op, int B, int H, int W, int R, int M)
{
    InpaintLayout L{};
    size_t N = (size_t)B * H * W;
    size_t tiles = (size_t)max_partials_per_image(R, H, W) * B;
    size_t o = 0;
    L.X = o; o = align_up(o + sizeof(float) * N);
    L.Y = o; o = align_up(o + sizeof(float) * N);
    L.partials = o; o = align_up(o + sizeof(double) * 2 * tiles);
    L.sums = o; o = align_up(o + sizeof(double) * 2 * (size_t)B);
    if (op == EED4_OP_INPAINT) {
        // the second state buffer of the run to a tolerance
        L.T = o; o = align_up(o + sizeof(float) * N);
    }
    L.hist = o;
    if (op == EED4_OP_INPAINT) o = align_up(o + sizeof(double) * 2 * (size_t)B * M);
    L.total = o;
    return L;
}

// ---- autotuner choice cache ----
static std::mutex g_tune_mu;
static std::map<std::string, int> g_tune;
static bool g_tune_loaded = false;

static void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("EED4_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char key[160];
    int shape;
    while (std::fscanf(f, "%159s %d", key, &shape) == 2)
        if (shape >= 0 && shape < kNumShapes) g_tune[key] = shape;
    std::fclose(f);
}

bool tune_lookup(const std::string &key, int *shape)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *shape = it->second;
    return true;
}

void tune_remember(const std::string &key, int shape)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    g_tune[key] = shape;
    const char *path = std::getenv("EED4_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "w");
    if (!f) return;
    for (auto &kv : g_tune) std::fprintf(f, "%s %d\n", kv.first.c_str(), kv.second);
    std::fclose(f);
}

std::string single_tune_key(int R, int B, int H, int W)
{
    char buf[96];
    std::snprintf(buf, sizeof(buf), "single_R%d_B%d_H%d_W%d", R, B, H, W);
    return buf;
}

// Fused step kernel of the single-image / equal-size-batch entry points:
// EED4_FORCE_SHAPE, else EED4_TILE_KERNEL, else the autotuned choice for this
// problem size, else tiles for problems too small for strips and strips
// otherwise.  All shapes give bitwise the same result (they share the
// per-pixel arithmetic of eed4_pointwise.h), so the choice changes only speed.
int step_shape(const eed4_params *p, int B, int H, int W)
{
    if (model_of_flags(p->flags) != 0) return kShapeStripShort;   // the variant kernel
    const int forced = (p->flags >> 8) & 0xff;
    if (forced >= 1 && forced <= kNumShapes) return forced - 1;
    if (p->flags & EED4_TILE_KERNEL) return 0;
    const int R = eed4_radius(p->sigma);
    int shape;
    if (tune_lookup(single_tune_key(R, B, H, W), &shape)) return shape;
    return default_step_shape(R, B, H, W);
}

int default_step_shape(int R, int B, int H, int W)
{
    const long long waves = (long long)tiles_per_image(kShapeStrip, R, H, W) * B;
    return waves < kMinStripWaves ? 2 : kShapeStrip;
}

// Times one inner step (k = 0, S -> X; S is not modified) of every candidate
// shape (tune_candidates) and remembers the fastest for this problem size.
int tune_single_step(const eed4_params *p, int B, int H, int W, float *S, float *X,
                     const uint8_t *mask, hipStream_t s, int *shape)
{
    TraceRange range("eed4 step-shape tuning %dx%dx%d", B, H, W);
    const int R = eed4_radius(p->sigma);
    const StepArgs a = make_args(p->sigma, R, p->tau, p->lambda, 0);
    int order[kNumShapes];
    const int first = default_step_shape(R, B, H, W);
    const int nc = tune_candidates(first, order);
    float margins[kNumShapes];
    for (int i = 0; i < nc; ++i) margins[i] = tune_margin(first, order[i]);
    const int rc = tune_pick(
        order, nc, s, [](int) { return (int)EED4_OK; },
        [&](int sh) { return launch_step(R, sh, S, S, X, nullptr, mask, B, H, W, a, nullptr, s); },
        "step autotune", shape, nullptr, margins);
    if (rc != EED4_OK) return rc;
    tune_remember(single_tune_key(R, B, H, W), *shape);
    return EED4_OK;
}

int check_ws(void *ws, size_t ws_bytes, size_t need)
{
    if (!ws || ((uintptr_t)ws & 255) != 0 || ws_bytes < need) return EED4_EWORKSPACE;
    return EED4_OK;
}

// Pinned, coherent host memory of at least `bytes` for the residual sums of
// the calling thread's runs to tolerance: the cycle's reduction kernel stores
// them straight into it over the bus, so no copy sits in the stream between
// two cycles.  Grows and is kept for the thread's lifetime (a cycle graph
// captured on a buffer that was since replaced is never launched again: the
// graph cache keys on the pointer).
static double *pinned_sums(size_t bytes)
{
    static thread_local double *buf = nullptr;
    static thread_local size_t cap = 0;
    if (cap < bytes) {
        if (buf) (void)hipHostFree(buf);
        buf = nullptr;
        cap = 0;
        void *q = nullptr;
        if (hipHostMalloc(&q, bytes, hipHostMallocCoherent) != hipSuccess) return nullptr;
        buf = (double *)q;
        cap = bytes;
    }
    return buf;
}

// Result of a run of FSI cycles: cycles run, the last cycle's largest plain
// and relative residual over the batch, and whether any was not finite.
struct RunResult {
    int cycles = 0;
    double worst_abs = 0.0, worst_rel = 0.0;
    bool diverged = false;
};

static void evaluate_residuals(const double *sums, int B, RunResult &r)
{
    r.worst_abs = r.worst_rel = 0.0;
    for (int b = 0; b < B; ++b) {
        const double res = std::sqrt(sums[2 * b]), nn = std::sqrt(sums[2 * b + 1]);
        if (!std::isfinite(res) || !std::isfinite(nn)) r.diverged = true;
        r.worst_abs = std::fmax(r.worst_abs, res);
        r.worst_rel = std::fmax(r.worst_rel, nn > 0.0 ? res / nn : res);
    }
}

// Cycles until the first whose residual is below tol (Sec. 3.3), or M, with
// the stop decision one cycle behind the GPU: cycle m+1 is queued before the
// host reads cycle m's residual, so the GPU never waits for the host.  The
// cycles alternate between the caller's u and T (even cycles read u and end
// in T, odd ones the reverse), so the cycle queued beyond the stop point
// writes only the buffer that does not hold the accepted result; at the end
// the result is copied into u when it lies in T.  That extra cycle also writes
// its checkpoint slot (when it exists) and history slot, which the caller does
// not read.  Each cycle's reduction stores its residual sums straight into
// slot m & 1 of a pinned host buffer, which the host reads once the event
// recorded after the cycle has completed.
static int run_to_tolerance(const CycleJob &j, float *T, const eed4_params *p,
                            float *ckpt, double *hist_dev, hipStream_t s, RunResult *out)
{
    const int M = p->max_cycles, B = j.B;
    const size_t N = (size_t)B * j.H * j.W;
    int rc = EED4_OK;
    hipError_t e = hipSuccess;
    // cycle m's sums land in slot m & 1 of the pinned buffer
    double *host = pinned_sums(sizeof(double) * 4 * (size_t)B);
    void *dev_host = nullptr;
    if (!host) rc = hip_fail(hipErrorOutOfMemory, "pinned host buffer");
    else if ((e = hipHostGetDevicePointer(&dev_host, host, 0)) != hipSuccess)
        rc = hip_fail(e, "pinned host buffer");
    CycleJob job[2] = {j, j};
    job[0].Out = T;                                   // even cycles: u -> T
    job[1].S = T; job[1].Out = j.S;                   // odd cycles: T -> u
    job[0].sums = (double *)dev_host;
    job[1].sums = (double *)dev_host + 2 * (size_t)B;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    bool own[2] = {false, false};
    for (int i = 0; i < 2 && rc == EED4_OK && !(p->flags & EED4_NO_GRAPH); ++i)
        rc = cycle_graph(job[i], 1, &exec[i], &own[i]);
    hipEvent_t ev[2] = {nullptr, nullptr};
    for (int i = 0; i < 2 && rc == EED4_OK; ++i) {
        e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
        if (e != hipSuccess) rc = hip_fail(e, "event");
    }
    auto issue = [&](int m) -> int {
        trace_mark("eed4 cycle %d queued", m);
        const CycleJob &c = job[m & 1];
        if (ckpt) {
            e = hipMemcpyAsync(ckpt + (size_t)m * N, c.S, sizeof(float) * N,
                               hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
        }
        if (exec[m & 1]) {
            e = hipGraphLaunch(exec[m & 1], s);
            if (e != hipSuccess) return hip_fail(e, "graph launch");
        } else {
            const int r = enqueue_cycle(c, s);
            if (r != EED4_OK) return r;
        }
        if (hist_dev) {
            e = hipMemcpyAsync(hist_dev + 2 * (size_t)B * m, c.sums, sizeof(double) * 2 * B,
                               hipMemcpyDefault, s);
            if (e != hipSuccess) return hip_fail(e, "history copy");
        }
        e = hipEventRecord(ev[m & 1], s);
        return e == hipSuccess ? (int)EED4_OK : hip_fail(e, "residual read-back");
    };
    // The residual decays about geometrically from cycle to cycle: when the last
    // two criteria predict that cycle m comes within 5 % of tol or below it,
    // m+1 is not queued before m's residual is read.  That saves the wasted
    // cycle at the stop; a wrong guess costs one host round trip of GPU idle
    // time, far less than a cycle, hence the generous margin.
    const double tol = (double)p->tol;
    double c1 = -1.0, c2 = -1.0;                     // criteria of cycles m-1, m-2
    int m = 0;
    if (rc == EED4_OK) rc = issue(0);
    for (; rc == EED4_OK; ++m) {
        const bool stop_likely = c1 > 0.0 && c2 > c1 && c1 * (c1 / c2) < 1.05 * tol;
        if (!stop_likely && m + 1 < M && (rc = issue(m + 1)) != EED4_OK) break;
        {
            TraceRange wait("eed4 wait for the residual of cycle %d", m);
            e = hipEventSynchronize(ev[m & 1]);
        }
        if (e != hipSuccess) { rc = hip_fail(e, "residual read-back"); break; }
        evaluate_residuals(host + 2 * (size_t)B * (m & 1), B, *out);
        const double crit = (p->flags & EED4_ABS_TOL) ? out->worst_abs : out->worst_rel;
        if (out->diverged || crit < tol || m == M - 1) break;
        if (stop_likely && (rc = issue(m + 1)) != EED4_OK) break;
        c2 = c1;
        c1 = crit;
    }
    out->cycles = m + 1;
    // wait for the cycle queued beyond the stop point, then bring the result home
    if (rc == EED4_OK && (e = hipStreamSynchronize(s)) != hipSuccess) rc = hip_fail(e, "sync");
    if (rc == EED4_OK && (m & 1) == 0) {
        e = hipMemcpyAsync(j.S, T, sizeof(float) * N, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = hip_fail(e, "result copy");
    }
    if (rc != EED4_OK) (void)hipStreamSynchronize(s);   // the pinned buffer outlives queued copies
    for (int i = 0; i < 2; ++i) {
        if (ev[i]) (void)hipEventDestroy(ev[i]);
        if (exec[i] && own[i]) (void)hipGraphExecDestroy(exec[i]);
    }
    return rc;
}

// M cycles in place on j.S with one stop-rule evaluation at the end (tol 0,
// or a single cycle).  Without checkpoints or history nothing is read between
// cycles: whole groups of kGraphCycles cycles run as one graph each (one
// launch, and one gap between launches, per group), the rest one by one.  The
// group size is fixed, so calls of any length share one cached graph.
static int run_fixed(const CycleJob &j, int M, const eed4_params *p, float *ckpt,
                     double *hist_dev, hipStream_t s, RunResult *out)
{
    const int B = j.B;
    const size_t N = (size_t)B * j.H * j.W;
    hipGraphExec_t exec = nullptr, multi = nullptr;
    bool own_exec = false, own_multi = false;
    int rc = EED4_OK;
    hipError_t e = hipSuccess;
    if (!(p->flags & EED4_NO_GRAPH)) rc = cycle_graph(j, 1, &exec, &own_exec);
    int m = 0;
    if (rc == EED4_OK && exec && !ckpt && !hist_dev && M >= kGraphCycles) {
        rc = cycle_graph(j, kGraphCycles, &multi, &own_multi);
        for (; rc == EED4_OK && m + kGraphCycles <= M; m += kGraphCycles) {
            trace_mark("eed4 cycles %d-%d queued", m, m + kGraphCycles - 1);
            e = hipGraphLaunch(multi, s);
            if (e != hipSuccess) rc = hip_fail(e, "graph launch");
        }
    }
    for (; rc == EED4_OK && m < M; ++m) {
        trace_mark("eed4 cycle %d queued", m);
        if (ckpt) {
            e = hipMemcpyAsync(ckpt + (size_t)m * N, j.S, sizeof(float) * N,
                               hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) { rc = hip_fail(e, "checkpoint copy"); break; }
        }
        if (exec) {
            e = hipGraphLaunch(exec, s);
            if (e != hipSuccess) { rc = hip_fail(e, "graph launch"); break; }
        } else if ((rc = enqueue_cycle(j, s)) != EED4_OK) {
            break;
        }
        if (hist_dev) {
            e = hipMemcpyAsync(hist_dev + 2 * (size_t)B * m, j.sums, sizeof(double) * 2 * B,
                               hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) { rc = hip_fail(e, "history copy"); break; }
        }
    }
    if (rc == EED4_OK) {       // the last cycle's residual: reported, and checked for divergence
        std::vector<double> host(2 * (size_t)B);
        e = hipMemcpyAsync(host.data(), j.sums, sizeof(double) * 2 * B, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = hip_fail(e, "residual read-back");
        else evaluate_residuals(host.data(), B, *out);
    }
    out->cycles = M;
    if (exec && own_exec) (void)hipGraphExecDestroy(exec);
    if (multi && own_multi) (void)hipGraphExecDestroy(multi);
    return rc;
}

// ---- static scratch of the allocation-free entry point ----
// In host code `scratch` is only a host-side stand-in for the device array:
// kernels and copies get the device address that hipGetSymbolAddress returns
// on each device (every device holds its own copy, at its own address).
static __device__ __align__(256) unsigned char scratch[EED4_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device, looked up on the first
// call per device and kept.
static int static_scratch(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "static scratch: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return hip_fail(hipErrorInvalidDevice, "static scratch");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "static scratch: hipGetSymbolAddress");
        if (!ptr || ((uintptr_t)ptr & 255) != 0)
            return hip_fail(hipErrorInvalidSymbol, "static scratch: address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return EED4_OK;
}

}  // namespace eed4

using namespace eed4;

extern "C" {

int eed4_step_shape(int B, int H, int W, const eed4_params *p)
{
    const int rc = check_params(p, B, H, W);
    return rc != EED4_OK ? rc : step_shape(p, B, H, W);
}

int eed4_radius(float sigma)
{
    if (!(sigma >= 0.0f) || !std::isfinite(sigma)) return -1;
    if (sigma == 0.0f) return 0;
    double r = std::ceil(3.0 * (double)sigma);
    return r <= (double)kRMax ? (int)r : -1;
}

size_t eed4_workspace_size(int op, int B, int H, int W, const eed4_params *p)
{
    if (check_params(p, B, H, W) == EED4_EINVAL) return 0;
    if (((p->flags >> 8) & 0xff) > kNumShapes) return 0;
    if (op == EED4_OP_INPAINT || op == EED4_OP_CYCLE)
        return inpaint_layout(op, B, H, W, eed4_radius(p->sigma), p->max_cycles).total;
    if (op == EED4_OP_BACKWARD) return backward_workspace(B, H, W, p);
    return 0;
}

int eed4_inpaint(float *u, const uint8_t *mask, const float *known, int B, int H, int W,
                 const eed4_params *p, float *ckpt, void *ws, size_t ws_bytes, void *stream,
                 eed4_stats *stats, double *hist)
{
    TraceRange range("eed4_inpaint %dx%dx%d, up to %d cycles of %d", B, H, W, p ? p->max_cycles : 0,
                     p ? p->cycle_len : 0);
    int rc = check_params(p, B, H, W);
    if (rc != EED4_OK) return rc;
    if (!u || !mask || !known) return EED4_EINVAL;
    const int M = p->max_cycles, R = eed4_radius(p->sigma);
    InpaintLayout L = inpaint_layout(EED4_OP_INPAINT, B, H, W, R, M);
    if ((rc = check_ws(ws, ws_bytes, L.total)) != EED4_OK) return rc;
    char *base = (char *)ws;
    hipStream_t s = (hipStream_t)stream;
    const size_t N = (size_t)B * H * W;

    CycleJob j;
    j.S = u; j.X = (float *)(base + L.X); j.Y = (float *)(base + L.Y);
    j.mask = mask; j.B = B; j.H = H; j.W = W; j.R = R; j.shape = step_shape(p, B, H, W); j.n = p->cycle_len;
    j.sigma = p->sigma; j.tau = p->tau; j.lambda = p->lambda; j.model = model_of_flags(p->flags);
    j.partials = (double *)(base + L.partials); j.sums = (double *)(base + L.sums);
    double *hist_dev = (double *)(base + L.hist);

    hipError_t e = launch_hold(u, mask, known, N, s);
    if (e != hipSuccess) return hip_fail(e, "hold launch");
    if (!((p->flags >> 8) & 0xff) && !(p->flags & EED4_TILE_KERNEL) && j.model == 0 &&
        !tune_lookup(single_tune_key(R, B, H, W), &j.shape)) {
        if ((rc = tune_single_step(p, B, H, W, u, j.X, mask, s, &j.shape)) != EED4_OK) return rc;
    }

    RunResult res;
    if (p->tol > 0.0f && M > 1) {
        rc = run_to_tolerance(j, (float *)(base + L.T), p, ckpt, hist ? hist_dev : nullptr, s,
                              &res);
    } else {
        rc = run_fixed(j, M, p, ckpt, hist ? hist_dev : nullptr, s, &res);
    }
    if (rc != EED4_OK) return rc;
    const int m = res.cycles;
    if (hist) {
        std::vector<double> hd(2 * (size_t)B * m);
        e = hipMemcpyAsync(hd.data(), hist_dev, sizeof(double) * hd.size(), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "history read-back");
        for (size_t i = 0; i < hd.size(); ++i) hist[i] = std::sqrt(hd[i]);
    }
    if (stats) {
        stats->cycles = m;
        stats->residual = res.worst_abs;
        stats->rel_residual = res.worst_rel;
    }
    return res.diverged ? EED4_EDIVERGED : EED4_OK;
}

int eed4_fsi_cycle(float *u, const uint8_t *mask, const float *known, int B, int H, int W,
                   const eed4_params *p, void *ws, size_t ws_bytes, void *stream, double *d_sums)
{
    TraceRange range("eed4_fsi_cycle %dx%dx%d", B, H, W);
    int rc = check_params(p, B, H, W);
    if (rc != EED4_OK) return rc;
    if (!u || !mask || !known || !d_sums) return EED4_EINVAL;
    InpaintLayout L = inpaint_layout(EED4_OP_CYCLE, B, H, W, eed4_radius(p->sigma), 1);
    if ((rc = check_ws(ws, ws_bytes, L.total)) != EED4_OK) return rc;
    char *base = (char *)ws;
    hipStream_t s = (hipStream_t)stream;
    CycleJob j;
    j.S = u; j.X = (float *)(base + L.X); j.Y = (float *)(base + L.Y);
    j.mask = mask; j.B = B; j.H = H; j.W = W; j.R = eed4_radius(p->sigma); j.shape = step_shape(p, B, H, W);
    j.n = p->cycle_len; j.sigma = p->sigma; j.tau = p->tau; j.lambda = p->lambda;
    j.model = model_of_flags(p->flags);
    j.partials = (double *)(base + L.partials); j.sums = d_sums;
    hipError_t e = launch_hold(u, mask, known, (size_t)B * H * W, s);
    if (e != hipSuccess) return hip_fail(e, "hold launch");
    return enqueue_cycle(j, s);
}

int eed4_fsi_cycle_static(float *u, const uint8_t *mask, const float *known, int B, int H,
                          int W, const eed4_params *p, void *stream, double *d_sums)
{
    int rc = check_params(p, B, H, W);
    if (rc != EED4_OK) return rc;
    if (!u || !mask || !known || !d_sums) return EED4_EINVAL;
    const size_t need =
        inpaint_layout(EED4_OP_CYCLE, B, H, W, eed4_radius(p->sigma), 1).total;
    if (need > EED4_STATIC_SCRATCH_BYTES) return EED4_ETOOLARGE;
    void *ws = nullptr;
    if ((rc = static_scratch(&ws)) != EED4_OK) return rc;
    return eed4_fsi_cycle(u, mask, known, B, H, W, p, ws, EED4_STATIC_SCRATCH_BYTES, stream,
                          d_sums);
}

int eed4_fsi_step(const float *ucur, const float *uprev, float *uout, const uint8_t *mask,
                  int B, int H, int W, const eed4_params *p, int k, void *stream)
{
    int rc = check_params(p, B, H, W);
    if (rc != EED4_OK) return rc;
    if (!ucur || !uprev || !uout || !mask || k < 0) return EED4_EINVAL;
    const size_t bytes = sizeof(float) * (size_t)B * H * W;
    const char *c0 = (const char *)ucur, *o0 = (const char *)uout;
    if (o0 < c0 + bytes && c0 < o0 + bytes) return EED4_EINVAL;
    const int R = eed4_radius(p->sigma);
    StepArgs a = make_args(p->sigma, R, p->tau, p->lambda, k, model_of_flags(p->flags));
    hipError_t e = launch_step(R, step_shape(p, B, H, W), ucur, uprev, uout, nullptr, mask, B, H, W, a, nullptr,
                               (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fsi step launch");
    return EED4_OK;
}

const char *eed4_strerror(int code)
{
    switch (code) {
    case EED4_OK: return "success";
    case EED4_EINVAL: return "invalid argument (size, pointer or parameter)";
    case EED4_EUNSTABLE: return "time step outside (0, 1/16] (set EED4_ALLOW_LARGE_TAU to force)";
    case EED4_EWORKSPACE: return "workspace missing, not 256-byte aligned or too small";
    case EED4_EHIP: {
        static thread_local std::string msg;
        msg = "HIP error: " + g_last_hip;
        return msg.c_str();
    }
    case EED4_EDIVERGED: return "non-finite cycle residual (diverged)";
    case EED4_ETOOLARGE:
        return "problem larger than the static scratch of eed4_fsi_cycle_static "
               "(EED4_STATIC_SCRATCH_BYTES)";
    default: return "unknown error code";
    }
}

}  // extern "C"
