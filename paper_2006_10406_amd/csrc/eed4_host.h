// Host-side helpers shared by the translation units of libeed4.
#pragma once

#include "eed4.h"
#include "eed4_internal.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <cmath>
#include <cstdio>
#include <functional>
#include <string>

namespace eed4 {

// Host-side roctx ranges and marks around the library's calls, cycles and
// waits (`rocprofv3 --marker-trace` shows them beside the kernel trace).  A
// range lasts for the lifetime of the object.  Without a tool attached each
// costs a formatted string and a call that returns at once.
class TraceRange {
public:
    template <typename... A>
    explicit TraceRange(const char *fmt, A... a)
    {
        char buf[160];
        std::snprintf(buf, sizeof(buf), fmt, a...);
        roctxRangePushA(buf);
    }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

template <typename... A>
inline void trace_mark(const char *fmt, A... a)
{
    char buf[160];
    std::snprintf(buf, sizeof(buf), fmt, a...);
    roctxMarkA(buf);
}

// One FSI cycle over a batch of B equal-size images.
struct CycleJob {
    float *S, *X, *Y;          // S: cycle start; X, Y: rotation buffers
    float *Out = nullptr;      // where the last step writes u^{m,n}: S (in place) when null
    const uint8_t *mask;
    int B, H, W, R, shape, n;
    float sigma, tau, lambda;
    int model;                 // tensor variant (0: FOEED)
    double *partials;          // per-tile residual partials
    double *sums;              // [B][2] residual sums
};

extern thread_local std::string g_last_hip;
int hip_fail(hipError_t e, const char *where);
size_t align_up(size_t x);
int check_params(const eed4_params *p, int B, int H, int W);
int check_ws(void *ws, size_t ws_bytes, size_t need);
int step_shape(const eed4_params *p, int B, int H, int W);

// Without a tuned choice, the single-image path uses workgroup tiles when
// the default strips would give fewer waves than this (too few to fill the
// chip), and strips otherwise.
constexpr long long kMinStripWaves = 2048;

// The autotuners keep the default shape unless another is faster by more than
// this factor, so shapes within timing noise of each other do not swap between
// runs.
constexpr float kTuneMargin = 0.98f;
// Candidate order for a tuner: `first`, then the other shapes in index order.
inline void tune_order(int first, int (&order)[kNumShapes])
{
    int n = 0;
    order[n++] = first;
    for (int sh = 0; sh < kNumShapes; ++sh)
        if (sh != first) order[n++] = sh;
}

// Candidates of the single-image tuner, `first` (the size rule's default)
// first; returns their count.  Where the default is a strip (enough work for
// the strips to fill the chip) the workgroup tiles are left out: they need
// 2-3x the instructions per pixel and lose by far more than the tuner's
// margin, and timing them would only load the GPU.  Where the default is a
// tile the 28- and 8-row strips are the strips that can compete.
inline int tune_candidates(int first, int (&order)[kNumShapes])
{
    int n = 0;
    order[n++] = first;
    for (int sh = 0; sh < kNumShapes; ++sh) {
        if (sh == first) continue;
        const bool keep = is_strip(first) ? is_strip(sh)
                                           : (!is_strip(sh) || sh == kShapeStripShort ||
                                              sh == kShapeStripTiny);
        if (keep) order[n++] = sh;
    }
    return n;
}
int default_step_shape(int R, int B, int H, int W);

// Margin a candidate of the single-image tuner must beat the current choice
// by.  Where the default is the 64-row strip (images large enough for it),
// the 28-row strips, which fetch the halo rows their neighbours share again
// (1.20x the algorithmic bytes against 1.006x for the 64-row strips, whose
// segments alternate direction), have to be clearly faster: in sustained
// runs at 4096^2 they are level with the 64-row strip or a few percent
// slower, and slower once the image leaves the Infinity Cache, while a short
// tuning burst has at times put them 2 % ahead.
constexpr float kTuneMarginRefetch = 0.95f;
inline float tune_margin(int first, int shape)
{
    const bool refetch = shape == kShapeStripShort || shape == kShapeStripWideShort;
    return first == kShapeStrip && refetch ? kTuneMarginRefetch : kTuneMargin;
}

// Chooses one of n candidate shapes (cands[0] the default) by timing on stream
// s.  prepare(shape) sets up a candidate outside the timed region (EED4 code);
// launch(shape) enqueues one launch of it.  Every candidate is sampled in two
// round-robin passes of one warm-up launch and two timed samples of
// kTuneLaunches back-to-back launches, and keeps its fastest sample, so the
// clock ramp at the start of tuning does not favour the candidates timed later
// and a fixed cost per launch (e.g. a profiler's) does not decide between
// shapes a few percent apart.  A candidate replaces the current choice only
// when it is faster by more than kTuneMargin (or its own entry of margins).
constexpr int kTuneLaunches = 4;
template <typename Prepare, typename Launch>
int tune_pick(const int *cands, int n, hipStream_t s, Prepare &&prepare, Launch &&launch,
              const char *where, int *best, float *best_ms, const float *margins = nullptr)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float tmin[kNumShapes];
    for (int i = 0; i < n; ++i) tmin[i] = 1e30f;
    int rc = EED4_OK;
    for (int pass = 0; pass < 2 && e == hipSuccess && rc == EED4_OK; ++pass)
        for (int i = 0; i < n && e == hipSuccess && rc == EED4_OK; ++i) {
            if ((rc = prepare(cands[i])) != EED4_OK) break;
            for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
                e = hipEventRecord(e0, s);
                for (int l = 0; l < (rep > 0 ? kTuneLaunches : 1) && e == hipSuccess; ++l)
                    e = launch(cands[i]);
                if (e == hipSuccess) e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e == hipSuccess && rep > 0) tmin[i] = std::fmin(tmin[i], ms);
            }
        }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc != EED4_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, where);
    int b = 0;
    for (int i = 1; i < n; ++i)
        if (tmin[i] < (margins ? margins[i] : kTuneMargin) * tmin[b]) b = i;
    *best = cands[b];
    if (best_ms) *best_ms = tmin[b];
    return EED4_OK;
}

// Autotuner choice cache (process-wide; persisted to the file named by
// EED4_AUTOTUNE_CACHE when set).
bool tune_lookup(const std::string &key, int *shape);
void tune_remember(const std::string &key, int shape);
std::string single_tune_key(int R, int B, int H, int W);
int tune_single_step(const eed4_params *p, int B, int H, int W, float *S, float *X,
                     const uint8_t *mask, hipStream_t s, int *shape);
StepArgs make_args(float sigma, int R, float tau, float lambda, int k, int model = 0);
hipStream_t capture_stream();
hipStream_t recompute_stream();
void cycle_roles(int k, int n, float *S, float *X, float *Y, float **cur, float **prev,
                 float **out);
int enqueue_cycle(const CycleJob &j, hipStream_t s);
int capture_graph(const std::function<int(hipStream_t)> &enqueue, hipGraphExec_t *exec);
int capture_cycle(const CycleJob &j, hipGraphExec_t *exec, int nc = 1);
size_t backward_workspace(int B, int H, int W, const eed4_params *p);

}  // namespace eed4
