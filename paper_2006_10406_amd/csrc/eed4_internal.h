// Internal declarations shared by the HIP translation units of libeed4.
// Not part of the public ABI (include/eed4.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace eed4 {

constexpr int kRMax = 8;        // largest Gaussian radius (sigma <= 8/3)
constexpr int kThreads = 256;   // threads per workgroup of the tile kernels

// Debug build (compiled with EED4_LDS_SENTINEL=1): every stencil kernel fills
// its LDS with NaN before each stage that writes it, so a read of a slot the
// stage did not write (an undersized halo, a missing barrier) turns the outputs
// it feeds into NaN or changes them.  Off (and compiled out) in the library.
#ifndef EED4_LDS_SENTINEL
#define EED4_LDS_SENTINEL 0
#endif
constexpr bool kLdsSentinel = EED4_LDS_SENTINEL != 0;

// NaN into p[0 .. n) by the whole workgroup, then a workgroup barrier.
__device__ __forceinline__ void sentinel_fill_block(float *p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = __builtin_nanf("");
    __syncthreads();
}

// NaN into p[0 .. n) by one wave (its own LDS region); the wave's later LDS
// accesses stay after these stores.
__device__ __forceinline__ void sentinel_fill_wave(float *p, int n)
{
    for (int i = threadIdx.x & 63; i < n; i += 64) p[i] = __builtin_nanf("");
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Per-launch constants of one inner FSI step.
struct StepArgs {
    float w[2 * kRMax + 1];  // sampled Gaussian, w[j + R], j = -R..R, sums to 1
    float tau;               // time step
    float alpha;             // FSI weight alpha_k = (4k+2)/(2k+3)
    float inv_lam2;          // 1 / lambda^2
    int model;               // tensor variant: diffusivity | mu3 rule << 4 (0: FOEED)
};

// Tensor variants (the public flags EED4_DIFFUSIVITY / EED4_MU3).
constexpr int kNumDiffusivities = 4;   // Charbonnier, Perona-Malik, exp. Perona-Malik, Geman-Reynolds
constexpr int kNumMu3Rules = 3;        // geometric mean, arithmetic mean, maximum
constexpr int kDiffPeronaMalik = 1, kDiffPeronaMalikExp = 2, kDiffGemanReynolds = 3;
constexpr int kMu3Arithmetic = 1, kMu3Max = 2;
inline int model_of_flags(int flags) { return ((flags >> 16) & 0xf) | (((flags >> 20) & 0x3) << 4); }

// Output tile of the fused step kernels.
struct TileShape {
    int tw, th;
};

// Threads of a tile workgroup: 512 for the 32 x 32 tile (one output per
// thread in the last stage, half the serial work per thread in each stage:
// 10 % faster on a 512^2 image, 6-7 % on 3 x 512^2 and 16 x 256^2, where tiles
// are chosen), 256 for the others.
constexpr int tile_threads(int tw, int th) { return tw == 32 && th == 32 ? 512 : kThreads; }

// Kernel shapes compiled into the library (index = config id): 0..2 and
// 9..10 are workgroup tiles (tw x th outputs per workgroup of tile_threads);
// 3..8 are wave strips (60 or 124 columns x a segment of rows per wave).  The
// small tiles (9, 10) give images of a few hundred pixels a side more
// workgroups than the chip has CUs.
constexpr int kNumTileShapes = 5;
constexpr TileShape kTileShapes[kNumTileShapes] = {{64, 32}, {64, 16}, {32, 32}, {32, 16}, {16, 16}};
constexpr int kShapeStrip = 3;       // wave strips of >= 64 output rows
constexpr int kShapeStripTall = 4;   // >= 136 rows
constexpr int kShapeStripShort = 5;  // >= 28 rows (more waves for small images)
constexpr int kShapeStripTiny = 6;   // >= 8 rows (shortest row pipeline per wave)
constexpr int kShapeStripWide = 7;       // two columns per lane (124 per wave), >= 64 rows
constexpr int kShapeStripWideShort = 8;  // two columns per lane, >= 28 rows
constexpr int kShapeTile32x16 = 9;
constexpr int kShapeTile16x16 = 10;
constexpr int kNumShapes = 11;
constexpr bool is_strip(int shape) { return shape >= kShapeStrip && shape <= kShapeStripWideShort; }
// index into kTileShapes of a tile shape
constexpr int tile_index(int shape) { return shape < kShapeStrip ? shape : shape - 6; }
constexpr int strip_target_rows(int shape)
{
    return shape == kShapeStripTall ? 136
         : shape == kShapeStripShort || shape == kShapeStripWideShort ? 28
         : shape == kShapeStripTiny  ? 8
                                     : 64;
}
constexpr int strip_cols_per_lane(int shape) { return shape >= kShapeStripWide ? 2 : 1; }
constexpr int strip_width(int shape) { return 64 * strip_cols_per_lane(shape) - 4; }

// ---- launchers (eed4_forward.hip) ----
hipError_t launch_hold(float *u, const uint8_t *mask, const float *known, size_t n,
                       hipStream_t s);
hipError_t launch_step(int R, int shape, const float *ucur, const float *uprev, float *uout,
                       const float *ref, const uint8_t *mask, int B, int H, int W,
                       const StepArgs &a, double *partials, hipStream_t s);
// A step of the adjoint's forward recompute on strips (the height follows the
// forward shape), which also writes K_sigma * u^k into vout.
hipError_t launch_step_keepv(int R, int shape, const float *ucur, const float *uprev,
                             float *uout, float *vout, const uint8_t *mask, int B, int H, int W,
                             const StepArgs &a, hipStream_t s);
// v = K_sigma * u, bitwise as a step from u computes it.
hipError_t launch_blur(int R, const float *u, float *v, int B, int H, int W, const StepArgs &a,
                       hipStream_t s);
hipError_t launch_reduce(const double *partials, int tiles_per_img, int B, double *sums,
                         hipStream_t s);
int tiles_per_image(int shape, int R, int H, int W);  // residual partials per image
int strip_rows(int R, int shape);                      // output rows per strip segment

}  // namespace eed4
