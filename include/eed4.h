/*
 * eed4.h -- C ABI of the MI355X (gfx950) implementation of fourth-order
 * edge-enhancing diffusion (FOEED) inpainting with the Fast Semi-Iterative
 * (FSI) scheme, after Jumakulyyev & Schultz, "Fourth-Order Anisotropic
 * Diffusion for Inpainting and Image Compression" (arXiv 2006.10406).
 *
 * The problem (Sec. 2.1, eq. inpaintingModel; Sec. 3.1, eq. genModel):
 *   du/dt = -d_ij [ D(J(u_sigma)) : H(u) ]_ij  on the unknown pixels,
 *   u = f on the known set K, homogeneous Neumann condition on the border,
 * with the fourth-order diffusion tensor D built from the Gaussian-presmoothed
 * gradient (eigenvalues g, 1, sqrt(g), 0; Charbonnier g, eq. CharDiff), solved
 * to steady state with FSI cycles (Sec. 3.3):
 *   u^{m,k+1} = alpha_k (I - tau P(u^{m,k})) u^{m,k} + (1 - alpha_k) u^{m,k-1},
 *   alpha_k = (4k+2)/(2k+3), u^{m,-1} := u^{m,0}, u^{m+1,0} := u^{m,n}.
 *
 * Conventions shared by every entry point
 *  - Images are row-major float32 [H][W] (x = column, fastest; y = row);
 *    a batch is [B][H][W] of equal-size images, contiguous.  Sizes:
 *    1 <= H <= 2^24, 1 <= W <= 2^21, H*W <= 2^31, B*H*W <= 2^36; anything
 *    else is EED4_EINVAL.
 *  - The mask is uint8 [B][H][W]; nonzero marks a known pixel.  known holds
 *    f and is read only where the mask is nonzero.
 *  - Every array pointer is a DEVICE pointer owned by the caller.  The library
 *    never frees or retains caller memory and allocates no device memory: the
 *    caller passes a workspace of at least eed4_workspace_size() bytes
 *    (256-byte aligned), used as scratch for the duration of the call.
 *  - stream is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is stream-ordered; only eed4_inpaint and eed4_inpaint_batched
 *    synchronise (once per cycle when a tolerance is set, else once at the
 *    end) to read residuals.
 *  - Return value: EED4_OK (0) or a negative EED4_E* code; no exception
 *    crosses the ABI.  eed4_strerror() gives a message (including the last
 *    HIP error for EED4_EHIP).
 *  - Numerics: FP32 arithmetic on the device; the cycle residual is
 *    accumulated in FP64.  Results are deterministic (no atomics in any sum).
 *  - Readings of the paper fixed by this ABI: half-sample mirror boundary,
 *    sampled Gaussian truncated at radius ceil(3 sigma) <= 8, central
 *    differences for the gradient, sign-corrected mixed difference u_xy
 *    (Sec. 3.3 prints four plus signs), tensor recomputed at every step.
 */
#ifndef EED4_H
#define EED4_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define EED4_OK          0
#define EED4_EINVAL     (-1)  /* bad size, pointer or parameter              */
#define EED4_EUNSTABLE  (-2)  /* tau outside (0, 1/16] without the override */
#define EED4_EWORKSPACE (-3)  /* workspace missing, misaligned or too small  */
#define EED4_EHIP       (-4)  /* a HIP runtime call or kernel launch failed  */
#define EED4_EDIVERGED  (-5)  /* non-finite cycle residual                   */
#define EED4_ETOOLARGE  (-6)  /* problem needs more than the static scratch of
                                 eed4_fsi_cycle_static                       */

/* ---- flags (eed4_params.flags) ---- */
/* Accept tau > 1/16.  The explicit step is L2-stable for tau <= 1/16 because
 * the largest eigenvalue of P is at most 32 (Sec. 3.3 gives the sufficient
 * bound 1/17 and reports 0.066 as usable in practice). */
#define EED4_ALLOW_LARGE_TAU 0x1
/* Stop on the plain residual ||u^{m,n} - u^{m,0}||_2 < tol (as in Sec. 3.3)
 * instead of the relative one ||u^{m,n} - u^{m,0}||_2 / ||u^{m,n}||_2. */
#define EED4_ABS_TOL         0x2
/* Launch each inner step directly instead of replaying a captured hipGraph
 * of the cycle (same results; for comparison). */
#define EED4_NO_GRAPH        0x4
/* Use the workgroup-tile step kernel (64 x 32 outputs per 256-thread
 * workgroup, stages separated by barriers) instead of the default wave-strip
 * kernel.  Both compute the same step with bitwise the same results. */
#define EED4_TILE_KERNEL     0x8

/* Use kernel shape s for the fused step instead of the automatic choice
 * (the autotuners of eed4_inpaint and eed4_inpaint_batched; eed4_fsi_cycle,
 * eed4_fsi_step and eed4_backward use the choice eed4_inpaint made for the
 * same problem size, else a work-size rule):
 * 0: 64x32 workgroup tiles, 1: 64x16 tiles, 2: 32x32 tiles, 3: wave strips of
 * 60 columns x >= 64 rows, 4: strips of >= 136 rows, 5: strips of >= 28 rows,
 * 6: strips of >= 8 rows, 7: strips of 124 columns (two per lane) x >= 64 rows,
 * 8: 124-column strips of >= 28 rows, 9: 32x16 tiles, 10: 16x16 tiles.
 * Every shape forms each value with the same operations in the same order, so
 * all shapes give bitwise the same results. */
#define EED4_FORCE_SHAPE(s)  ((((s) + 1) & 0xff) << 8)

/* Tensor variants.  The default (both fields 0) is the paper's FOEED tensor:
 * Charbonnier diffusivity and mu_3 = sqrt(mu_1 mu_2).  The others are the
 * alternatives the paper compares: the diffusivities of Table 7 and the
 * choices of mu_3 of Sec. 3.1 (Table 1).  With s = |grad u_sigma| and
 * x = (s/lambda)^2, the diffusivity g = mu_1 is
 *   EED4_CHARBONNIER       (1 + x)^(-1/2)   (eq. CharDiff)
 *   EED4_PERONA_MALIK      (1 + x)^(-1)
 *   EED4_PERONA_MALIK_EXP  exp(-x)
 *   EED4_GEMAN_REYNOLDS    (1 + x)^(-2): Table 7's 2 lambda^2/(s^2+lambda^2)^2
 *                          scaled to g(0) = 1 like the others
 * (Table 7's Aubert entry vanishes at s = 0 and is not offered), and mu_3 is
 *   EED4_MU3_GEOMETRIC     sqrt(mu_1 mu_2) = sqrt(g)
 *   EED4_MU3_ARITHMETIC    (mu_1 + mu_2)/2 = (1 + g)/2
 *   EED4_MU3_MAX           max(mu_1, mu_2) = 1.
 * Every eigenvalue stays in [0, 1], so the step bound tau <= 1/16 holds for
 * all of them.  A non-default variant runs the 60-column strip kernel of
 * shape 5 (EED4_FORCE_SHAPE may name only that shape; EED4_TILE_KERNEL is
 * EED4_EINVAL) in every entry point: eed4_inpaint, eed4_fsi_cycle,
 * eed4_fsi_step, the batched calls (no shape tuning) and, with the matching
 * reverse step, eed4_backward. */
#define EED4_CHARBONNIER       0
#define EED4_PERONA_MALIK      1
#define EED4_PERONA_MALIK_EXP  2
#define EED4_GEMAN_REYNOLDS    3
#define EED4_MU3_GEOMETRIC     0
#define EED4_MU3_ARITHMETIC    1
#define EED4_MU3_MAX           2
#define EED4_DIFFUSIVITY(d)  (((d) & 0xf) << 16)
#define EED4_MU3(r)          (((r) & 0x3) << 20)

/* ---- workspace sizing (eed4_workspace_size op) ---- */
#define EED4_OP_INPAINT  1
#define EED4_OP_CYCLE    2
#define EED4_OP_BACKWARD 3

typedef struct eed4_params {
    float lambda;    /* contrast lambda > 0 of the diffusivity; by default the
                        Charbonnier g(s^2) = 1/sqrt(1 + s^2/lambda^2) (eq. CharDiff) */
    float sigma;     /* presmoothing sigma >= 0 with ceil(3 sigma) <= 8; 0 disables
                        the presmoothing (Sec. 2.2)                            */
    float tau;       /* time step tau in (0, 1/16] (Sec. 3.3)                   */
    int   cycle_len; /* FSI cycle length n >= 1 (the paper uses 40)             */
    int   max_cycles;/* cycle count M >= 1 (upper bound when tol > 0)           */
    float tol;       /* >= 0; > 0 stops after the first cycle whose residual is
                        below tol for every image of the batch (Sec. 3.3)       */
    int   flags;     /* EED4_* flags                                           */
} eed4_params;

typedef struct eed4_stats {
    int    cycles;        /* cycles run                                         */
    double residual;      /* largest ||u^{m,n} - u^{m,0}||_2 over the batch,
                             last cycle                                         */
    double rel_residual;  /* largest relative residual over the batch           */
} eed4_stats;

/* One image of an uneven batch (eed4_inpaint_batched).  Device pointers. */
typedef struct eed4_image {
    float         *u;       /* [H][W] in: initial guess, out: result            */
    const uint8_t *mask;    /* [H][W] nonzero = known                           */
    const float   *known;   /* [H][W] f, read where mask != 0                   */
    int            H, W;    /* >= 1                                             */
    float          lambda;  /* per-image contrast (> 0)                         */
} eed4_image;

/* Gaussian truncation radius ceil(3 sigma), evaluated in double from the
 * float sigma, used by every entry point (0 for sigma == 0); -1 if sigma is
 * negative, not finite or the radius would exceed 8. */
int eed4_radius(float sigma);

/* Bytes of workspace needed by op (EED4_OP_*) for a batch of B images of
 * H x W; max_cycles of p matters for EED4_OP_INPAINT (residual history) and
 * cycle_len for EED4_OP_BACKWARD (recomputed states).  0 on invalid input. */
size_t eed4_workspace_size(int op, int B, int H, int W, const eed4_params *p);

/* Inpaint B equal-size images (Sec. 2.1 model with the tensor of Sec. 3.1,
 * solved by FSI, Sec. 3.3).
 *  u      [B][H][W] in: initial guess (any values off the mask); out: u^{m,0}
 *         after the last cycle run.  Known pixels are set to f first.
 *  ckpt   NULL, or [max_cycles][B][H][W]: receives the cycle-start state
 *         u^{m,0} of every cycle run (for eed4_backward).
 *  hist   NULL, or HOST [max_cycles][B][2]: per cycle and image, the residual
 *         ||u^{m,n}-u^{m,0}||_2 and ||u^{m,n}||_2 (FP64).
 *  stats  NULL or HOST output.
 * Errors: EED4_EINVAL, EED4_EUNSTABLE, EED4_EWORKSPACE, EED4_EHIP,
 * EED4_EDIVERGED (u then holds the diverged state). */
int eed4_inpaint(float *u, const uint8_t *mask, const float *known,
                 int B, int H, int W, const eed4_params *p, float *ckpt,
                 void *ws, size_t ws_bytes, void *stream,
                 eed4_stats *stats, double *hist);

/* One FSI cycle (n = p->cycle_len inner steps, Sec. 3.3) in place on u,
 * after setting the known pixels to f.  d_sums: DEVICE [B][2] receives
 * sum (u^{m,n}-u^{m,0})^2 and sum (u^{m,n})^2 per image (FP64).  No
 * synchronisation, no stop decision.  max_cycles and tol are ignored. */
int eed4_fsi_cycle(float *u, const uint8_t *mask, const float *known,
                   int B, int H, int W, const eed4_params *p,
                   void *ws, size_t ws_bytes, void *stream, double *d_sums);

/* Bytes of the static device scratch of eed4_fsi_cycle_static (per device). */
#define EED4_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/* eed4_fsi_cycle without a workspace, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  The cycle's scratch (the two rotation buffers and the
 * residual partials) lives in a static device array of
 * EED4_STATIC_SCRATCH_BYTES that every device the library runs on holds until
 * the process ends; the call itself allocates nothing.  Arguments, results and
 * errors are those of eed4_fsi_cycle, and so are the results, bitwise.
 * Limit: a problem fits when eed4_workspace_size(EED4_OP_CYCLE, B, H, W, p)
 * <= EED4_STATIC_SCRATCH_BYTES (B*H*W up to about 8 million pixels, e.g. one
 * 2048 x 2048 image or 16 images of 512 x 512); larger ones return
 * EED4_ETOOLARGE before any device work.  Every call on one device shares that
 * device's scratch: calls that overlap on one device (two host threads, or
 * two streams with no ordering between them) race and give undefined results.
 * The first call on a device looks up the array's address there (no
 * allocation); nothing in the scratch needs clearing between calls. */
int eed4_fsi_cycle_static(float *u, const uint8_t *mask, const float *known,
                          int B, int H, int W, const eed4_params *p,
                          void *stream, double *d_sums);

/* One FSI inner step (Sec. 3.3) of B equal-size images:
 *   uout = alpha_k (I - tau P(ucur)) ucur + (1 - alpha_k) uprev,
 * then uout = ucur on the known pixels (ucur must already hold f there).
 * alpha_k = (4k+2)/(2k+3) with k >= 0 the step index inside the cycle.
 * uout may equal uprev (each pixel is read before it is written) but must not
 * overlap ucur.  No workspace, no residual, no synchronisation. */
int eed4_fsi_step(const float *ucur, const float *uprev, float *uout,
                  const uint8_t *mask, int B, int H, int W,
                  const eed4_params *p, int k, void *stream);

/* Adjoint of eed4_inpaint run for exactly M cycles with tol == 0 (the FSI
 * evolution differentiated by hand; the paper gives the forward scheme only).
 * Each cycle is recomputed from its checkpoint (the states and, for the strip
 * reverse step, their presmoothed images: 2n - 1 planes of B x H x W floats
 * per cycle, two cycles' worth in the workspace), then reversed step by step;
 * the recompute of cycle m-1 runs on a library-owned stream (one per device,
 * default priority) while cycle m is reversed on `stream`, ordered by events,
 * and `stream` waits for all of it: work on `stream` after the call sees
 * every result, as for any stream-ordered call.  The first call for a problem
 * size times the reverse-step kernels once (cached per process).
 *  ckpt        [M][B][H][W] cycle-start states as written by eed4_inpaint.
 *  grad_u      [B][H][W] dL/du^{M,0}.
 *  grad_known  [B][H][W] out: dL/df (0 off the mask).
 *  grad_init   [B][H][W] out: dL/du_init (0 on the mask).
 *  grad_lambda [B] out: dL/dlambda contributed by each image (float).
 * max_cycles and tol of p are ignored; M is passed explicitly. */
int eed4_backward(const float *ckpt, const uint8_t *mask, const float *known,
                  int B, int H, int W, const eed4_params *p, int M,
                  const float *grad_u, float *grad_known, float *grad_init,
                  float *grad_lambda, void *ws, size_t ws_bytes, void *stream);

/* Bytes of workspace for eed4_inpaint_batched over the given images. */
size_t eed4_batched_workspace_size(const eed4_image *imgs, int B,
                                   const eed4_params *p);

/* Inpaint B images of uneven sizes with one launch per inner step over a
 * work queue of tiles or strip segments spanning all images; the cycle is
 * replayed as a captured hipGraph.  sigma, tau, n, M, tol and flags come from p; lambda
 * from each image.  imgs is a HOST array.  stats: NULL or HOST [B]; an image
 * whose residual falls below tol stops and leaves the queue (per-image stop).
 * Results equal eed4_inpaint on each image alone. */
int eed4_inpaint_batched(const eed4_image *imgs, int B, const eed4_params *p,
                         void *ws, size_t ws_bytes, void *stream,
                         eed4_stats *stats);

/* Autotuner of eed4_inpaint_batched: times one inner step of every kernel
 * shape on this batch (the caller's u is not modified), remembers the fastest
 * for batches of this kind (radius, image count, size classes) and returns
 * its id (>= 0), or a negative EED4_E* code.  eed4_inpaint_batched runs it by
 * itself on the first call for a kind of batch; with the environment variable
 * EED4_AUTOTUNE_CACHE naming a file, choices persist across processes. */
int eed4_autotune_batched(const eed4_image *imgs, int B, const eed4_params *p,
                          void *ws, size_t ws_bytes, void *stream);

/* Fused-step kernel shape (EED4_FORCE_SHAPE index) that eed4_inpaint,
 * eed4_fsi_cycle and eed4_fsi_step use for B equal-size H x W images with
 * parameters p: the forced shape, else the one the autotuner chose for this
 * problem size in this process (eed4_inpaint tunes on first use), else the
 * size rule used before any tuning.  No device work.  Returns the shape
 * (>= 0) or EED4_EINVAL. */
int eed4_step_shape(int B, int H, int W, const eed4_params *p);

/* Message for a return code (static or thread-local storage; not freed). */
const char *eed4_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* EED4_H */
