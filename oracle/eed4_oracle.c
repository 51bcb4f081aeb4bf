/*
 * eed4_oracle.c -- plain FP64 reference of fourth-order edge-enhancing
 * diffusion (FOEED) inpainting with the Fast Semi-Iterative (FSI) scheme,
 * after Jumakulyyev & Schultz, "Fourth-Order Anisotropic Diffusion for
 * Inpainting and Image Compression" (arXiv 2006.10406).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct checker
 * of the HIP implementation.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.  It
 * shares no code, header or table with the HIP library.
 *
 * Conventions: images are row-major [H][W]; x is the column index (fastest),
 * y the row index; grid spacing is 1.  Every routine works in double.
 *
 * Readings of the paper taken here (where it is silent or garbled):
 *  - the mixed difference u_xy uses signs (++ and -- positive, +- and -+
 *    negative); the printed stencil (Sec. 3.3) shows four plus signs, which
 *    would not be a derivative;
 *  - the homogeneous Neumann condition (Sec. 2.1) is realised by a half-sample
 *    mirror extension of u, and every intermediate (presmoothed image,
 *    gradient, Hessian, contracted tensor) is evaluated on the extended image;
 *  - the Gaussian presmoothing (Sec. 2.2) is a sampled, normalised,
 *    separable kernel truncated at radius ceil(3 sigma);
 *  - the gradient of u_sigma uses central differences;
 *  - the diffusion tensor is recomputed at every inner FSI step (Sec. 3.3
 *    writes P(u^{m,k}));
 *  - the cycle residual may be taken relative to ||u^{m,n}||_2;
 *  - Table 7's Geman-Reynolds diffusivity is scaled to g(0) = 1 (see
 *    diffusivity_x); its Aubert entry, which vanishes at s = 0, is left out.
 * Adjoint: derived here from the forward recursion (Sec. 3.3) by the chain
 * rule; it is not in the paper.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* basic helpers                                                             */
/* ------------------------------------------------------------------------ */

/* Half-sample mirror index: ... 1 0 | 0 1 ... N-1 | N-1 N-2 ..., repeated
 * reflection for indices farther away than N (period 2N). */
static int refl(int i, int N)
{
    int p = 2 * N;
    int m = i % p;
    if (m < 0) m += p;
    return m < N ? m : p - 1 - m;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following calls (timing of the oracle on n host cores). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Gaussian truncation radius used throughout: ceil(3 sigma), 0 for sigma<=0. */
int oracle_radius(double sigma)
{
    if (!(sigma > 0.0)) return 0;
    return (int)ceil(3.0 * sigma);
}

/* Sampled Gaussian exp(-j^2 / (2 sigma^2)), j = -R..R, normalised to sum 1
 * (presmoothing of Sec. 2.2).  w has 2R+1 entries. */
void oracle_gauss(double sigma, int R, double *w)
{
    if (R == 0) { w[0] = 1.0; return; }
    double s = 0.0;
    for (int j = -R; j <= R; ++j) {
        w[j + R] = exp(-(double)(j * j) / (2.0 * sigma * sigma));
        s += w[j + R];
    }
    for (int j = 0; j < 2 * R + 1; ++j) w[j] /= s;
}

/* Charbonnier diffusivity g(s^2) = 1/sqrt(1 + s^2/lambda^2) (Sec. 2.2). */
double oracle_charbonnier(double s2, double lam)
{
    return 1.0 / sqrt(1.0 + s2 / (lam * lam));
}

/* The diffusivities compared in Table 7, as functions of x = (s/lambda)^2,
 * and their derivatives dg/dx:
 *   0 Charbonnier              (1 + x)^(-1/2)            (eq. CharDiff)
 *   1 Perona-Malik             (1 + x)^(-1)
 *   2 Perona-Malik exponential exp(-x)
 *   3 Geman-Reynolds           (1 + x)^(-2)
 * Table 7 prints the Geman-Reynolds function as 2 lambda^2 / (s^2 +
 * lambda^2)^2, which is (2 / lambda^2) (1 + x)^(-2); it is used here scaled
 * to g(0) = 1 like the other three, so that every eigenvalue of the tensor
 * stays in [0, 1] and the step bound tau <= 1/16 holds for all of them.
 * (The Aubert entry of the table vanishes at s = 0 and is left out.) */
static double diffusivity_x(double x, int diff, double *dgdx)
{
    double g;
    switch (diff) {
    case 1: g = 1.0 / (1.0 + x); *dgdx = -g * g; break;
    case 2: g = exp(-x); *dgdx = -g; break;
    case 3: g = 1.0 / ((1.0 + x) * (1.0 + x)); *dgdx = -2.0 * g / (1.0 + x); break;
    default: g = 1.0 / sqrt(1.0 + x); *dgdx = -0.5 * g * g * g; break;
    }
    return g;
}

double oracle_diffusivity(double s2, double lam, int diff)
{
    double d;
    return diffusivity_x(s2 / (lam * lam), diff, &d);
}

/* mu_3 from mu_1 = g and mu_2 = 1 (Sec. 3.1, Table 1):
 *   0 geometric mean sqrt(mu_1 mu_2)  (the paper's choice for FOEED)
 *   1 arithmetic mean (mu_1 + mu_2)/2
 *   2 maximum of mu_1 and mu_2 (= 1)
 * and d mu_3 / d g. */
static double mu3_of(double g, int rule, double *dmdg)
{
    switch (rule) {
    case 1: *dmdg = 0.5; return 0.5 * (g + 1.0);
    case 2: *dmdg = 0.0; return g > 1.0 ? g : 1.0;
    default:   /* g = 0 only where g underflows; there d sqrt(g)/ds -> 0 */
        *dmdg = g > 0.0 ? 0.5 / sqrt(g) : 0.0;
        return sqrt(g);
    }
}

/* ------------------------------------------------------------------------ */
/* the fourth-order diffusion tensor (Sec. 3.1)                              */
/* ------------------------------------------------------------------------ */

/* 2x2 matrices are stored row-major: [xx, xy, yx, yy]. */
static void outer2(const double a[2], const double b[2], double M[4])
{
    M[0] = a[0] * b[0]; M[1] = a[0] * b[1];
    M[2] = a[1] * b[0]; M[3] = a[1] * b[1];
}

/* A:B = trace(B^T A). */
static double ddot2(const double A[4], const double B[4])
{
    return A[0] * B[0] + A[1] * B[1] + A[2] * B[2] + A[3] * B[3];
}

/* Eigen-directions of the structure tensor J = grad u_s grad u_s^T:
 * v1 along the gradient, v2 orthogonal.  Where the gradient vanishes the
 * direction is arbitrary; (1,0) is used (every mu_i is 1 there, so the tensor
 * does not depend on it). */
static void directions(double gx, double gy, double v1[2], double v2[2])
{
    double s = sqrt(gx * gx + gy * gy);
    if (s > 0.0) { v1[0] = gx / s; v1[1] = gy / s; }
    else { v1[0] = 1.0; v1[1] = 0.0; }
    v2[0] = -v1[1]; v2[1] = v1[0];
}

/* Eigentensors E1..E4 of eq. (foad_diffTensor_entries) and their derivative
 * with respect to the gradient angle theta (v1 = (cos t, sin t)). */
static void eigentensors(const double v1[2], const double v2[2],
                         double E[4][4], double dE[4][4])
{
    const double r2 = 1.0 / sqrt(2.0);
    double a[4], b[4], c[4], d[4];
    outer2(v1, v1, a);          /* v1 v1^T */
    outer2(v2, v2, b);          /* v2 v2^T */
    outer2(v1, v2, c);          /* v1 v2^T */
    outer2(v2, v1, d);          /* v2 v1^T */
    for (int i = 0; i < 4; ++i) {
        E[0][i] = a[i];
        E[1][i] = b[i];
        E[2][i] = r2 * (c[i] + d[i]);
        E[3][i] = r2 * (c[i] - d[i]);
    }
    /* d v1/dt = v2, d v2/dt = -v1 */
    for (int i = 0; i < 4; ++i) {
        dE[0][i] = c[i] + d[i];            /* v2 v1^T + v1 v2^T */
        dE[1][i] = -(c[i] + d[i]);         /* -v1 v2^T - v2 v1^T */
        dE[2][i] = r2 * (2.0 * b[i] - 2.0 * a[i]);
        dE[3][i] = 0.0;
    }
}

/* Eigenvalues mu_1..mu_4 = g, 1, mu_3(g), 0 (eq. foad_diffTensor_entries)
 * for diffusivity diff and mu_3 rule mu3 (diff = mu3 = 0 is the paper's
 * FOEED: Charbonnier, geometric mean), with their derivatives with respect
 * to s = |grad u_sigma| and to lambda (used by the adjoint). */
static void eigenvalues(double s2, double lam, int diff, int mu3, double mu[4],
                        double dmu_ds[4], double dmu_dl[4])
{
    double l2 = lam * lam, x = s2 / l2, dgdx, dmdg;
    double g = diffusivity_x(x, diff, &dgdx);
    double m3 = mu3_of(g, mu3, &dmdg);
    /* dx/ds = 2 s / lambda^2, dx/dlambda = -2 s^2 / lambda^3 */
    double gs = dgdx * 2.0 * sqrt(s2) / l2, gl = dgdx * (-2.0 * s2 / (l2 * lam));
    mu[0] = g; mu[1] = 1.0; mu[2] = m3; mu[3] = 0.0;
    dmu_ds[0] = gs; dmu_ds[1] = 0.0; dmu_ds[2] = dmdg * gs; dmu_ds[3] = 0.0;
    dmu_dl[0] = gl; dmu_dl[1] = 0.0; dmu_dl[2] = dmdg * gl; dmu_dl[3] = 0.0;
}

/* Full 16-coefficient tensor d_ijkl = sum_n mu_n (E_n)_ij (E_n)_kl
 * (eq. faod_diffTensor); d[(2i+j)*4 + (2k+l)]. */
void oracle_tensor(double gx, double gy, double lam, int diff, int mu3, double d[16])
{
    double v1[2], v2[2], E[4][4], dE[4][4], mu[4], ds[4], dl[4];
    directions(gx, gy, v1, v2);
    eigentensors(v1, v2, E, dE);
    eigenvalues(gx * gx + gy * gy, lam, diff, mu3, mu, ds, dl);
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            double s = 0.0;
            for (int n = 0; n < 4; ++n) s += mu[n] * E[n][a] * E[n][b];
            d[a * 4 + b] = s;
        }
}

/* T_ij = d_ijkl H_kl (eq. double-dot). */
static void contract(const double d[16], const double Hm[4], double T[4])
{
    for (int a = 0; a < 4; ++a) {
        double s = 0.0;
        for (int b = 0; b < 4; ++b) s += d[a * 4 + b] * Hm[b];
        T[a] = s;
    }
}

/* Pointwise bilinear form e = A : D(G) : H and its derivatives with respect
 * to the regularised gradient G = (gx, gy) and to the contrast lambda.  Used
 * by the adjoint.  G is written in polar form s (cos t, sin t); the mu_n
 * depend on s, the eigentensors on t. */
void oracle_e_grad(double gx, double gy, const double A[4], const double Hm[4],
                   double lam, int diff, int mu3, double *e, double q[2], double *dedlam)
{
    double v1[2], v2[2], E[4][4], dE[4][4], mu[4], dmu_ds[4], dmu_dl[4];
    double s2 = gx * gx + gy * gy, s = sqrt(s2);
    directions(gx, gy, v1, v2);
    eigentensors(v1, v2, E, dE);
    eigenvalues(s2, lam, diff, mu3, mu, dmu_ds, dmu_dl);
    double ee = 0.0, de_ds = 0.0, de_dt = 0.0, de_dl = 0.0;
    for (int n = 0; n < 4; ++n) {
        double aE = ddot2(A, E[n]), hE = ddot2(E[n], Hm);
        ee += mu[n] * aE * hE;
        de_ds += dmu_ds[n] * aE * hE;
        de_dl += dmu_dl[n] * aE * hE;
        de_dt += mu[n] * (ddot2(A, dE[n]) * hE + aE * ddot2(dE[n], Hm));
    }
    *e = ee;
    *dedlam = de_dl;
    if (s > 0.0) {
        /* d/dgx = cos t d/ds - sin t / s d/dt ; d/dgy = sin t d/ds + cos t / s d/dt */
        q[0] = v1[0] * de_ds - v1[1] * de_dt / s;
        q[1] = v1[1] * de_ds + v1[0] * de_dt / s;
    } else {
        q[0] = 0.0; q[1] = 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* forward operator, evaluated on the mirror-extended image                  */
/* ------------------------------------------------------------------------ */

static void extend(const double *a, int H, int W, int h, double *e)
{
    int We = W + 2 * h, He = H + 2 * h;
    for (int y = 0; y < He; ++y)
        for (int x = 0; x < We; ++x)
            e[(size_t)y * We + x] = a[(size_t)refl(y - h, H) * W + refl(x - h, W)];
}

/* out = P(ut) x: the diffusion tensor is built from the presmoothed gradient
 * of ut; the Hessian, the contraction and the outer divergence act on x
 * (eq. genModel; P(u)u is the right-hand side with the sign flipped). */
void oracle_apply_P(const double *ut, const double *x, int H, int W,
                    double lam, double sigma, int diff, int mu3, double *out)
{
    int R = oracle_radius(sigma), h = R + 2;
    int He = H + 2 * h, We = W + 2 * h;
    size_t ne = (size_t)He * We;
    double *w = malloc(sizeof(double) * (2 * R + 1));
    double *ue = malloc(sizeof(double) * ne);
    double *xe = malloc(sizeof(double) * ne);
    double *vx = calloc(ne, sizeof(double));
    double *v = calloc(ne, sizeof(double));
    int Hp = H + 2, Wp = W + 2;                /* T on domain rows/cols -1..H/W */
    double *T = malloc(sizeof(double) * 4 * (size_t)Hp * Wp);
    oracle_gauss(sigma, R, w);
    extend(ut, H, W, h, ue);
    extend(x, H, W, h, xe);

    /* separable presmoothing: x pass, then y pass */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < He; ++y)
        for (int xx = R; xx < We - R; ++xx) {
            double s = 0.0;
            for (int j = -R; j <= R; ++j) s += w[j + R] * ue[(size_t)y * We + xx + j];
            vx[(size_t)y * We + xx] = s;
        }
#pragma omp parallel for schedule(static)
    for (int y = R; y < He - R; ++y)
        for (int xx = R; xx < We - R; ++xx) {
            double s = 0.0;
            for (int j = -R; j <= R; ++j) s += w[j + R] * vx[(size_t)(y + j) * We + xx];
            v[(size_t)y * We + xx] = s;
        }

    /* gradient, tensor, Hessian and contraction on domain points -1..H, -1..W */
#pragma omp parallel for schedule(static)
    for (int py = 0; py < Hp; ++py)
        for (int px = 0; px < Wp; ++px) {
            int ey = py - 1 + h, ex = px - 1 + h;
#define V(yy, xx) v[(size_t)(yy) * We + (xx)]
#define X(yy, xx) xe[(size_t)(yy) * We + (xx)]
            double gx = 0.5 * (V(ey, ex + 1) - V(ey, ex - 1));
            double gy = 0.5 * (V(ey + 1, ex) - V(ey - 1, ex));
            double hxx = X(ey, ex - 1) - 2.0 * X(ey, ex) + X(ey, ex + 1);
            double hyy = X(ey - 1, ex) - 2.0 * X(ey, ex) + X(ey + 1, ex);
            double hxy = 0.25 * (X(ey + 1, ex + 1) + X(ey - 1, ex - 1)
                                 - X(ey + 1, ex - 1) - X(ey - 1, ex + 1));
#undef V
#undef X
            double d[16], Hm[4] = { hxx, hxy, hxy, hyy }, Tm[4];
            oracle_tensor(gx, gy, lam, diff, mu3, d);
            contract(d, Hm, Tm);
            for (int c = 0; c < 4; ++c) T[((size_t)c * Hp + py) * Wp + px] = Tm[c];
        }

    /* outer derivatives: dxx T_xx + dyx T_xy + dxy T_yx + dyy T_yy */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int xx = 0; xx < W; ++xx) {
            int py = y + 1, px = xx + 1;
#define TT(c, yy, x2) T[((size_t)(c) * Hp + (yy)) * Wp + (x2)]
            double dxx = TT(0, py, px - 1) - 2.0 * TT(0, py, px) + TT(0, py, px + 1);
            double dyy = TT(3, py - 1, px) - 2.0 * TT(3, py, px) + TT(3, py + 1, px);
            double dxy1 = 0.25 * (TT(1, py + 1, px + 1) + TT(1, py - 1, px - 1)
                                  - TT(1, py + 1, px - 1) - TT(1, py - 1, px + 1));
            double dxy2 = 0.25 * (TT(2, py + 1, px + 1) + TT(2, py - 1, px - 1)
                                  - TT(2, py + 1, px - 1) - TT(2, py - 1, px + 1));
#undef TT
            out[(size_t)y * W + xx] = dxx + dxy1 + dxy2 + dyy;
        }
    free(w); free(ue); free(xe); free(vx); free(v); free(T);
}

/* Hessian (h_xx, h_xy, h_yy) of u at the domain points, mirror boundary. */
void oracle_hessian(const double *u, int H, int W, double *hxx, double *hxy, double *hyy)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
#define U(yy, x2) u[(size_t)refl(yy, H) * W + refl(x2, W)]
            size_t i = (size_t)y * W + x;
            hxx[i] = U(y, x - 1) - 2.0 * U(y, x) + U(y, x + 1);
            hyy[i] = U(y - 1, x) - 2.0 * U(y, x) + U(y + 1, x);
            hxy[i] = 0.25 * (U(y + 1, x + 1) + U(y - 1, x - 1) - U(y + 1, x - 1) - U(y - 1, x + 1));
#undef U
        }
}

/* Regularised gradient grad(K_sigma * u) at the domain points. */
void oracle_gradient(const double *u, int H, int W, double sigma, double *gx, double *gy)
{
    int R = oracle_radius(sigma);
    double *w = malloc(sizeof(double) * (2 * R + 1));
    double *t = malloc(sizeof(double) * (size_t)H * W);
    double *v = malloc(sizeof(double) * (size_t)H * W);
    oracle_gauss(sigma, R, w);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double s = 0.0;
            for (int j = -R; j <= R; ++j) s += w[j + R] * u[(size_t)y * W + refl(x + j, W)];
            t[(size_t)y * W + x] = s;
        }
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double s = 0.0;
            for (int j = -R; j <= R; ++j) s += w[j + R] * t[(size_t)refl(y + j, H) * W + x];
            v[(size_t)y * W + x] = s;
        }
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            gx[(size_t)y * W + x] = 0.5 * (v[(size_t)y * W + refl(x + 1, W)] - v[(size_t)y * W + refl(x - 1, W)]);
            gy[(size_t)y * W + x] = 0.5 * (v[(size_t)refl(y + 1, H) * W + x] - v[(size_t)refl(y - 1, H) * W + x]);
        }
    free(w); free(t); free(v);
}

/* ------------------------------------------------------------------------ */
/* FSI (Sec. 3.3)                                                            */
/* ------------------------------------------------------------------------ */

/* alpha_k = (4k+2)/(2k+3) */
double oracle_alpha(int k)
{
    return (4.0 * k + 2.0) / (2.0 * k + 3.0);
}

/* One FSI inner step:
 *   u^{k+1} = alpha_k (I - tau P(u^k)) u^k + (1 - alpha_k) u^{k-1},
 * followed by the Dirichlet condition u = f on the known set K. */
void oracle_step(const double *u, const double *uprev, const uint8_t *mask,
                 const double *f, int H, int W, double lam, double sigma,
                 int diff, int mu3, double tau, int k, double *out)
{
    size_t N = (size_t)H * W;
    double *Pu = malloc(sizeof(double) * N);
    double a = oracle_alpha(k);
    oracle_apply_P(u, u, H, W, lam, sigma, diff, mu3, Pu);
    for (size_t i = 0; i < N; ++i) {
        double v = a * (u[i] - tau * Pu[i]) + (1.0 - a) * uprev[i];
        out[i] = (mask && mask[i]) ? f[i] : v;
    }
    free(Pu);
}

/* Inpainting of B equal-size images.  u holds the initial guess on entry and
 * the result on exit ([B][H][W]); known pixels are first set to f.  Each
 * cycle runs n FSI steps starting with u^{m,-1} := u^{m,0}.  After the cycle
 * the residual ||u^{m,n} - u^{m,0}||_2 and ||u^{m,n}||_2 are recorded per
 * image in hist[m][b][0..1].  With tol > 0 the run stops after the first
 * cycle whose residual (relative unless abs_tol) is below tol for every image;
 * otherwise after M cycles.  ckpt (may be NULL) receives u^{m,0} per cycle,
 * [M][B][H][W].  Returns the number of cycles run. */
int oracle_inpaint(double *u, const uint8_t *mask, const double *f,
                   int B, int H, int W, double lam, double sigma, int diff, int mu3,
                   double tau, int n, int M, double tol, int abs_tol,
                   double *ckpt, double *hist)
{
    size_t N = (size_t)H * W;
    double *S = malloc(sizeof(double) * N);
    double *prev = malloc(sizeof(double) * N);
    double *cur = malloc(sizeof(double) * N);
    double *nxt = malloc(sizeof(double) * N);
    for (int b = 0; b < B; ++b)
        for (size_t i = 0; i < N; ++i)
            if (mask[b * N + i]) u[b * N + i] = f[b * N + i];
    int m;
    for (m = 0; m < M; ++m) {
        double worst = 0.0;
        if (ckpt) memcpy(ckpt + (size_t)m * B * N, u, sizeof(double) * B * N);
        for (int b = 0; b < B; ++b) {
            double *ub = u + b * N;
            memcpy(S, ub, sizeof(double) * N);
            memcpy(prev, ub, sizeof(double) * N);
            memcpy(cur, ub, sizeof(double) * N);
            for (int k = 0; k < n; ++k) {
                oracle_step(cur, prev, mask + b * N, f + b * N, H, W, lam, sigma, diff, mu3,
                            tau, k, nxt);
                double *t = prev; prev = cur; cur = nxt; nxt = t;
            }
            memcpy(ub, cur, sizeof(double) * N);
            double r = 0.0, nn = 0.0;
            for (size_t i = 0; i < N; ++i) {
                double d = ub[i] - S[i];
                r += d * d;
                nn += ub[i] * ub[i];
            }
            r = sqrt(r); nn = sqrt(nn);
            if (hist) { hist[((size_t)m * B + b) * 2] = r; hist[((size_t)m * B + b) * 2 + 1] = nn; }
            double crit = abs_tol ? r : (nn > 0.0 ? r / nn : r);
            if (crit > worst) worst = crit;
        }
        if (tol > 0.0 && worst < tol) { ++m; break; }
    }
    free(S); free(prev); free(cur); free(nxt);
    return m;
}

/* ------------------------------------------------------------------------ */
/* adjoint (derived from the forward recursion; not in the paper)            */
/* ------------------------------------------------------------------------ */
/* Here the operator is written with gathers over the domain points (mirror
 * indices), and every transpose is the matching scatter.                    */

static void blur_gather(const double *u, int H, int W, const double *w, int R, double *v)
{
    double *t = malloc(sizeof(double) * (size_t)H * W);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double s = 0.0;
            for (int j = -R; j <= R; ++j) s += w[j + R] * u[(size_t)y * W + refl(x + j, W)];
            t[(size_t)y * W + x] = s;
        }
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double s = 0.0;
            for (int j = -R; j <= R; ++j) s += w[j + R] * t[(size_t)refl(y + j, H) * W + x];
            v[(size_t)y * W + x] = s;
        }
    free(t);
}

static void blur_scatter(const double *vb, int H, int W, const double *w, int R, double *ub)
{
    double *tb = calloc((size_t)H * W, sizeof(double));
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int j = -R; j <= R; ++j)
                tb[(size_t)refl(y + j, H) * W + x] += w[j + R] * vb[(size_t)y * W + x];
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int j = -R; j <= R; ++j)
                ub[(size_t)y * W + refl(x + j, W)] += w[j + R] * tb[(size_t)y * W + x];
    free(tb);
}

/* 2x2 Hessian per domain point: Hm[i*4 + (xx, xy, yx, yy)] */
static void hess_gather(const double *u, int H, int W, double *Hm)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
#define U(yy, x2) u[(size_t)refl(yy, H) * W + refl(x2, W)]
            double *o = Hm + 4 * ((size_t)y * W + x);
            o[0] = U(y, x - 1) - 2.0 * U(y, x) + U(y, x + 1);
            o[3] = U(y - 1, x) - 2.0 * U(y, x) + U(y + 1, x);
            o[1] = o[2] = 0.25 * (U(y + 1, x + 1) + U(y - 1, x - 1) - U(y + 1, x - 1) - U(y - 1, x + 1));
#undef U
        }
}

static void hess_scatter(const double *T, int H, int W, double *out)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const double *t = T + 4 * ((size_t)y * W + x);
#define O(yy, x2) out[(size_t)refl(yy, H) * W + refl(x2, W)]
            O(y, x - 1) += t[0]; O(y, x) += -2.0 * t[0]; O(y, x + 1) += t[0];
            O(y - 1, x) += t[3]; O(y, x) += -2.0 * t[3]; O(y + 1, x) += t[3];
            double c = 0.25 * (t[1] + t[2]);
            O(y + 1, x + 1) += c; O(y - 1, x - 1) += c;
            O(y + 1, x - 1) -= c; O(y - 1, x + 1) -= c;
#undef O
        }
}

/* J_F(u)^T w for F(u) = P(u) u, and <dF/dlambda, w>.  Since
 * <w, F(u)> = sum_p (B w)_p : D(G_p) : (B u)_p with G = grad K_sigma u, the
 * gradient with respect to u is B^T (D : B w) + C^T q, q_p = de_p/dG_p. */
void oracle_jtv(const double *u, const double *wv, int H, int W, double lam,
                double sigma, int diff, int mu3, double *out, double *dlam)
{
    int R = oracle_radius(sigma);
    size_t N = (size_t)H * W;
    double *wg = malloc(sizeof(double) * (2 * R + 1));
    double *v = malloc(sizeof(double) * N);
    double *Hu = malloc(sizeof(double) * 4 * N);
    double *Aw = malloc(sizeof(double) * 4 * N);
    double *T = malloc(sizeof(double) * 4 * N);
    double *qx = malloc(sizeof(double) * N), *qy = malloc(sizeof(double) * N);
    double *vb = calloc(N, sizeof(double));
    oracle_gauss(sigma, R, wg);
    blur_gather(u, H, W, wg, R, v);
    hess_gather(u, H, W, Hu);
    hess_gather(wv, H, W, Aw);
    double dl = 0.0;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t i = (size_t)y * W + x;
            double gx = 0.5 * (v[(size_t)y * W + refl(x + 1, W)] - v[(size_t)y * W + refl(x - 1, W)]);
            double gy = 0.5 * (v[(size_t)refl(y + 1, H) * W + x] - v[(size_t)refl(y - 1, H) * W + x]);
            double d[16], e, q[2], de;
            oracle_tensor(gx, gy, lam, diff, mu3, d);
            contract(d, Aw + 4 * i, T + 4 * i);        /* D is major-symmetric */
            oracle_e_grad(gx, gy, Aw + 4 * i, Hu + 4 * i, lam, diff, mu3, &e, q, &de);
            qx[i] = q[0]; qy[i] = q[1];
            dl += de;
        }
    memset(out, 0, sizeof(double) * N);
    hess_scatter(T, H, W, out);
    /* C^T q = K^T D^T q */
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t i = (size_t)y * W + x;
            vb[(size_t)y * W + refl(x + 1, W)] += 0.5 * qx[i];
            vb[(size_t)y * W + refl(x - 1, W)] -= 0.5 * qx[i];
            vb[(size_t)refl(y + 1, H) * W + x] += 0.5 * qy[i];
            vb[(size_t)refl(y - 1, H) * W + x] -= 0.5 * qy[i];
        }
    blur_scatter(vb, H, W, wg, R, out);
    *dlam = dl;
    free(wg); free(v); free(Hu); free(Aw); free(T); free(qx); free(qy); free(vb);
}

/* Reverse pass of oracle_inpaint run for exactly M cycles (no early stop),
 * for B equal-size images.  ckpt holds u^{m,0} for m = 0..M-1 ([M][B][H][W],
 * as written by oracle_inpaint).  gu = dL/du^{M,0} ([B][H][W]).  Outputs:
 * gf = dL/df (zero off the mask), ginit = dL/du_init (zero on the mask),
 * glam[b] = dL/dlambda contributed by image b. */
void oracle_backward(const double *ckpt, const uint8_t *mask, const double *f,
                     int B, int H, int W, double lam, double sigma, int diff, int mu3,
                     double tau, int n, int M, const double *gu, double *gf, double *ginit,
                     double *glam)
{
    size_t N = (size_t)H * W;
    double *U = malloc(sizeof(double) * N * (size_t)(n + 1));   /* u^{m,0..n} */
    double *abar = malloc(sizeof(double) * N * (size_t)(n + 2)); /* ubar^{m,-1..n} */
    double *r = malloc(sizeof(double) * N);
    double *jt = malloc(sizeof(double) * N);
    for (int b = 0; b < B; ++b) {
        const uint8_t *mb = mask + b * N;
        const double *fb = f + b * N;
        double *gfb = gf + b * N;
        double gl = 0.0;
        memset(gfb, 0, sizeof(double) * N);
        double *cyc = malloc(sizeof(double) * N);
        memcpy(cyc, gu + b * N, sizeof(double) * N);       /* ubar^{M,0} */
        for (int m = M - 1; m >= 0; --m) {
            /* recompute the cycle from its checkpoint */
            memcpy(U, ckpt + ((size_t)m * B + b) * N, sizeof(double) * N);
            for (int k = 0; k < n; ++k)
                oracle_step(U + (size_t)k * N, U + (size_t)(k > 0 ? k - 1 : 0) * N, mb, fb,
                            H, W, lam, sigma, diff, mu3, tau, k, U + (size_t)(k + 1) * N);
            /* abar index j holds ubar^{m, j-1} */
            memset(abar, 0, sizeof(double) * N * (size_t)(n + 2));
            memcpy(abar + (size_t)(n + 1) * N, cyc, sizeof(double) * N);
            for (int k = n - 1; k >= 0; --k) {
                double *an = abar + (size_t)(k + 2) * N;   /* ubar^{k+1} */
                double *ac = abar + (size_t)(k + 1) * N;   /* ubar^{k}   */
                double *ap = abar + (size_t)k * N;         /* ubar^{k-1} */
                double a = oracle_alpha(k), dl;
                for (size_t i = 0; i < N; ++i) {
                    if (mb[i]) { gfb[i] += an[i]; r[i] = 0.0; }
                    else r[i] = an[i];
                }
                oracle_jtv(U + (size_t)k * N, r, H, W, lam, sigma, diff, mu3, jt, &dl);
                for (size_t i = 0; i < N; ++i) {
                    ac[i] += a * r[i] - tau * a * jt[i];
                    ap[i] += (1.0 - a) * r[i];
                }
                gl += -tau * a * dl;
            }
            /* u^{m,-1} := u^{m,0} */
            for (size_t i = 0; i < N; ++i) cyc[i] = abar[N + i] + abar[i];
        }
        for (size_t i = 0; i < N; ++i) {
            if (mb[i]) { gfb[i] += cyc[i]; ginit[b * N + i] = 0.0; }
            else ginit[b * N + i] = cyc[i];
        }
        glam[b] = gl;
        free(cyc);
    }
    free(U); free(abar); free(r); free(jt);
}
