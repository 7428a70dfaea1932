/*
 * FP64 CPU oracle for learning-free feature uplifting (LUDVIG, arXiv
 * 2410.14462).  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the
 * CPU-baseline leg of the benchmark are its only callers.  It shares no code,
 * header or constant table with the GPU library; it is written from the
 * paper's definitions:
 *
 *   - Sec. 3.1, Eq. (1): pixel p of view d blends the ordered set S_{d,p};
 *     w_i(d,p) = alpha_i(d,p) * prod_{j<i} (1 - alpha_j(d,p)), with alpha_i the
 *     opacity times the projected 2D Gaussian density at p.
 *   - Sec. 3.2, Eq. (3) / Eq. (5): f_i = sum_{(d,p) in S_i} w_i(d,p) F_{d,p}
 *     / sum_{(d,p) in S_i} w_i(d,p), i.e. f = diag(beta)^-1 W^T F with beta the
 *     column sums of W (Gaussian filtering paragraph: beta_i = sum w_i).
 *   - Sec. 3.2, Eq. (4): the forward render F^ = W g (used for the adjoint pin).
 *
 * Conventions the paper leaves open (the projection, the tile support, the
 * clamp/skip/stop constants) follow the 3D Gaussian Splatting rasteriser the
 * paper relies on (Sec. 5); every choice is spelled out below.
 *
 * Evaluation is brute force: every pixel of every view walks, in order, every
 * Gaussian whose tile rectangle contains the pixel's tile.
 *
 *   - Structure (visibility, depth key, tile rectangle, hence each tile's
 *     ordered list) is discrete and decided by a fixed sequence of IEEE FP32
 *     operations ("S32") from the FP32 inputs, so that any two correct
 *     implementations of the convention agree bit for bit.
 *   - Everything else is FP64 from the same FP32 inputs: the projected centre
 *     and conic, alpha, the transmittance, the alpha >= 1/255 skip, the
 *     T < 1e-4 stop and every sum.  The skip and the stop are decided on the
 *     FP64 values, straight from the definition.
 *   - Decision margins: every skip decision has the relative margin
 *     |alpha - 1/255| / (1/255), every stop decision |T' - 1e-4| / 1e-4.  A
 *     pixel with a margin below a threshold (1e-5 by default) is ambiguous:
 *     an FP32 evaluation of the same definition may decide it the other way.
 *     Its Gaussians whose weight at the pixel depends on that decision (from
 *     the first ambiguous decision on: every candidate with alpha within the
 *     threshold of 1/255 or above, up to the stop and two beyond it) are
 *     flagged, so that comparisons can exclude them and count them.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fopenmp -fPIC -shared
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TILE 16

/* FP32 constants, exactly as FP32 literals (also promoted to FP64 for values). */
static const float K_ALPHA_MAX = 0x1.fae148p-1f;   /* 0.99f   */
static const float K_ALPHA_MIN = 0x1.010102p-8f;   /* 1/255.f */
static const float K_T_EPS = 0x1.a36e2ep-14f;      /* 1e-4f   */
static const float K_DILATE = 0x1.333334p-2f;      /* 0.3f    */
static const float K_CLAMP = 0x1.4cccccp+0f;       /* 1.3f    */

/* ----------------------------------------------------------------------- */
/* Camera: 17 floats = R[9] (world->camera, row-major), t[3], fx, fy, cx, cy,
 * znear; x_c = R x_w + t; x right, y down, z forward; pixel (i,j) is the unit
 * square [i,i+1) x [j,j+1), its centre (i+0.5, j+0.5).                       */
typedef struct { const float* c; int W, H; } orc_cam;

/* Per-Gaussian, per-view quantities. */
typedef struct {
    int vis;
    uint32_t depth;                 /* bits of FP32 z_c (z_c > 0 orders as unsigned) */
    int x0, y0, x1, y1;             /* tile rectangle [x0,x1) x [y0,y1)              */
    float ux, uy;                   /* S32 projected centre (decides the rectangle)   */
    double ux64, uy64;              /* FP64 projected centre                          */
    double A64, B64, C64, op64;     /* power = A dx^2 + B dx dy + C dy^2 (FP64)       */
} orc_proj;

/* Sec. 3.1: covariance from scale and rotation, Sigma = R diag(s)^2 R^T =
 * M M^T with M = R diag(s), R the rotation of the normalised quaternion
 * (w,x,y,z).  S32 keeps the factor M (row-major): the 2D covariance is then
 * formed from V = T M, which avoids the cancellation that a stored Sigma
 * suffers for thin Gaussians.                                                */
static void orc_factor32(const float* s, const float* q, float M[9])
{
    float n2 = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
    float w = 1.0f, x = 0.0f, y = 0.0f, z = 0.0f;
    if (n2 > 0.0f) {
        float nr = sqrtf(n2);
        w = q[0] / nr; x = q[1] / nr; y = q[2] / nr; z = q[3] / nr;
    }
    float R[9];
    R[0] = 1.0f - 2.0f * (y * y + z * z);
    R[1] = 2.0f * (x * y - w * z);
    R[2] = 2.0f * (x * z + w * y);
    R[3] = 2.0f * (x * y + w * z);
    R[4] = 1.0f - 2.0f * (x * x + z * z);
    R[5] = 2.0f * (y * z - w * x);
    R[6] = 2.0f * (x * z - w * y);
    R[7] = 2.0f * (y * z + w * x);
    R[8] = 1.0f - 2.0f * (x * x + y * y);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) M[3 * i + j] = R[3 * i + j] * s[j];
}

/* a*b - c*d to within ~1.5 ulp (Kahan's algorithm with fmaf). */
static float orc_diff_prod(float a, float b, float c, float d)
{
    float w = c * d;
    float e = fmaf(-c, d, w);
    return fmaf(a, b, -w) + e;
}

static void orc_cov64(const float* s, const float* q, double out[6])
{
    double q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
    double n2 = q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3;
    double w = 1, x = 0, y = 0, z = 0;
    if (n2 > 0) { double nr = sqrt(n2); w = q0 / nr; x = q1 / nr; y = q2 / nr; z = q3 / nr; }
    double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                   2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                   2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
    double M[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) M[3 * i + j] = R[3 * i + j] * (double)s[j];
    static const int I[6] = {0, 0, 0, 1, 1, 2}, J[6] = {0, 1, 2, 1, 2, 2};
    for (int e = 0; e < 6; e++) {
        const double* a = M + 3 * I[e];
        const double* b = M + 3 * J[e];
        out[e] = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    }
}

/* S32 centre, which places the tile rectangle: the centre u = f x_c / z_c + c
 * is formed as the correctly rounded value of an unevaluated sum of two
 * floats, built with error-free transformations: Knuth's TwoSum, TwoProduct
 * by fmaf, the compensated dot product Dot2 of Ogita, Rump and Oishi (SIAM
 * J. Sci. Comput. 26(6), 2005) for x_c = R x_w + t, one Newton-style
 * correction of the quotient x_c / z_c, and a compensated affine map
 * u = f i + c.  The FP32 result is therefore (almost always) the FP32 value
 * nearest the exact centre, whichever implementation computes it.          */
static void orc_two_sum(float a, float b, float* s, float* e)
{
    float x = a + b, bb = x - a;
    *s = x;
    *e = (a - (x - bb)) + (b - bb);
}

static void orc_two_prod(float a, float b, float* p, float* e)
{
    float x = a * b;
    *p = x;
    *e = fmaf(a, b, -x);
}

/* hi + lo = r0 m0 + r1 m1 + r2 m2 + t (Dot2 with the extra addend t). */
static void orc_dot3(const float* r, const float* m, float t, float* hi, float* lo)
{
    float p, s, h, q, e;
    orc_two_prod(r[0], m[0], &p, &s);
    orc_two_prod(r[1], m[1], &h, &q);
    orc_two_sum(p, h, &p, &e);
    s = s + (q + e);
    orc_two_prod(r[2], m[2], &h, &q);
    orc_two_sum(p, h, &p, &e);
    s = s + (q + e);
    orc_two_sum(p, t, &p, &e);
    s = s + e;
    *hi = p + s;
    *lo = s - (*hi - p);
}

/* hi = fl(f (xh + xl) / (zh + zl) + c) */
static float orc_center(float f, float c, float xh, float xl, float zh, float zl)
{
    float q = xh / zh;
    float r = fmaf(-q, zh, xh);
    r = (r + xl) - q * zl;
    float ql = r / zh;
    float p, e, s, g;
    orc_two_prod(f, q, &p, &e);
    e = fmaf(f, ql, e);
    orc_two_sum(p, c, &s, &g);
    g = g + e;
    return s + g;
}

/* Projection of one Gaussian into one view: EWA local-affine approximation
 * of the perspective map (Jacobian with x/z, y/z clamped to 1.3x the half-FoV
 * tangent), 2D covariance plus 0.3 px^2, conic = inverse, radius
 * ceil(3 sqrt(lambda_max)), 16x16 tile rectangle.  Values in FP64 from the
 * same FP32 inputs, as the textbook formulas.  Structure in S32: x_c, y_c,
 * z_c by Dot2 and the centre as above (the depth key is the FP32 z_c); the
 * 2D covariance [[a, b], [b, c]] = V V^T + 0.3 I from V = T M (T = J R_cam),
 * its determinant by Lagrange's identity |v0|^2 |v1|^2 - (v0.v1)^2 =
 * |v0 x v1|^2 (a sum of squares, no cancellation), lambda_max, the radius
 * and the rectangle.                                                        */
static void orc_project(const float* mu, const float* M, const double* cov64, float op,
                        const orc_cam* cam, orc_proj* g)
{
    const float* c = cam->c;
    const float *Rc = c, *t = c + 9;
    float fx = c[12], fy = c[13], cx = c[14], cy = c[15], zn = c[16];
    int TX = (cam->W + ORC_TILE - 1) / ORC_TILE, TY = (cam->H + ORC_TILE - 1) / ORC_TILE;
    memset(g, 0, sizeof(*g));

    /* ---- S32 ---- */
    float xc, xl, yc, yl, zc, zl;
    orc_dot3(Rc, mu, t[0], &xc, &xl);
    orc_dot3(Rc + 3, mu, t[1], &yc, &yl);
    orc_dot3(Rc + 6, mu, t[2], &zc, &zl);
    if (!(zc > zn)) return;
    float ix = xc / zc, iy = yc / zc;
    float ux = orc_center(fx, cx, xc, xl, zc, zl);
    float uy = orc_center(fy, cy, yc, yl, zc, zl);
    float limx = K_CLAMP * ((0.5f * (float)cam->W) / fx);
    float limy = K_CLAMP * ((0.5f * (float)cam->H) / fy);
    float tx = fminf(limx, fmaxf(-limx, ix));
    float ty = fminf(limy, fmaxf(-limy, iy));
    float j00 = fx / zc, j11 = fy / zc;
    float j02 = -(j00 * tx), j12 = -(j11 * ty);
    float T[6];
    for (int k = 0; k < 3; k++) {
        T[k] = j00 * Rc[k] + j02 * Rc[6 + k];
        T[3 + k] = j11 * Rc[3 + k] + j12 * Rc[6 + k];
    }
    float V[6];
    for (int i = 0; i < 2; i++)
        for (int k = 0; k < 3; k++)
            V[3 * i + k] = (T[3 * i] * M[k] + T[3 * i + 1] * M[3 + k]) + T[3 * i + 2] * M[6 + k];
    float n0 = (V[0] * V[0] + V[1] * V[1]) + V[2] * V[2];
    float n1 = (V[3] * V[3] + V[4] * V[4]) + V[5] * V[5];
    float b = (V[0] * V[3] + V[1] * V[4]) + V[2] * V[5];
    float a = n0 + K_DILATE, cc = n1 + K_DILATE;
    float k0 = orc_diff_prod(V[1], V[5], V[2], V[4]);
    float k1 = orc_diff_prod(V[2], V[3], V[0], V[5]);
    float k2 = orc_diff_prod(V[0], V[4], V[1], V[3]);
    float det = (((k0 * k0 + k1 * k1) + k2 * k2) + K_DILATE * (n0 + n1)) + K_DILATE * K_DILATE;
    if (!(det > 0.0f)) return;
    float h = 0.5f * (a + cc), dd = 0.5f * (a - cc);
    float lam = h + sqrtf(dd * dd + b * b);
    float r = ceilf(3.0f * sqrtf(lam));
    float fx0 = floorf((ux - r) / (float)ORC_TILE);
    float fx1 = floorf((ux + r) / (float)ORC_TILE) + 1.0f;
    float fy0 = floorf((uy - r) / (float)ORC_TILE);
    float fy1 = floorf((uy + r) / (float)ORC_TILE) + 1.0f;
    int x0 = (int)fminf(fmaxf(fx0, 0.0f), (float)TX), x1 = (int)fminf(fmaxf(fx1, 0.0f), (float)TX);
    int y0 = (int)fminf(fmaxf(fy0, 0.0f), (float)TY), y1 = (int)fminf(fmaxf(fy1, 0.0f), (float)TY);
    if (x1 <= x0 || y1 <= y0) return;
    g->vis = 1;
    memcpy(&g->depth, &zc, 4);
    g->x0 = x0; g->x1 = x1; g->y0 = y0; g->y1 = y1;
    g->ux = ux; g->uy = uy;

    /* ---- FP64 values ---- */
    double X = (double)Rc[0] * mu[0] + (double)Rc[1] * mu[1] + (double)Rc[2] * mu[2] + t[0];
    double Y = (double)Rc[3] * mu[0] + (double)Rc[4] * mu[1] + (double)Rc[5] * mu[2] + t[1];
    double Z = (double)Rc[6] * mu[0] + (double)Rc[7] * mu[1] + (double)Rc[8] * mu[2] + t[2];
    double IX = X / Z, IY = Y / Z;
    g->ux64 = (double)fx * IX + cx;
    g->uy64 = (double)fy * IY + cy;
    double LX = (double)K_CLAMP * (0.5 * cam->W / (double)fx);
    double LY = (double)K_CLAMP * (0.5 * cam->H / (double)fy);
    double TXc = fmin(LX, fmax(-LX, IX)), TYc = fmin(LY, fmax(-LY, IY));
    double J00 = fx / Z, J11 = fy / Z, J02 = -J00 * TXc, J12 = -J11 * TYc;
    double TT[6];
    for (int k = 0; k < 3; k++) {
        TT[k] = J00 * Rc[k] + J02 * Rc[6 + k];
        TT[3 + k] = J11 * Rc[3 + k] + J12 * Rc[6 + k];
    }
    double SS[9] = {cov64[0], cov64[1], cov64[2], cov64[1], cov64[3], cov64[4],
                    cov64[2], cov64[4], cov64[5]};
    double VV[6];
    for (int i = 0; i < 2; i++)
        for (int k = 0; k < 3; k++)
            VV[3 * i + k] = TT[3 * i] * SS[k] + TT[3 * i + 1] * SS[3 + k] + TT[3 * i + 2] * SS[6 + k];
    double A2 = VV[0] * TT[0] + VV[1] * TT[1] + VV[2] * TT[2] + (double)K_DILATE;
    double B2 = VV[0] * TT[3] + VV[1] * TT[4] + VV[2] * TT[5];
    double C2 = VV[3] * TT[3] + VV[4] * TT[4] + VV[5] * TT[5] + (double)K_DILATE;
    double DET = A2 * C2 - B2 * B2;
    g->A64 = -0.5 * C2 / DET;
    g->B64 = B2 / DET;
    g->C64 = -0.5 * A2 / DET;
    g->op64 = op;
}

/* ----------------------------------------------------------------------- */
/* Scene: precomputed FP32 covariance factors and FP64 covariances.         */
typedef struct {
    int64_t n;
    const float *mu, *op;
    float* fac32;
    double* cov64;
} orc_scene;

static int orc_scene_init(orc_scene* sc, int64_t n, const float* mu, const float* s,
                          const float* q, const float* op)
{
    sc->n = n; sc->mu = mu; sc->op = op;
    sc->fac32 = (float*)malloc(sizeof(float) * 9 * (size_t)(n ? n : 1));
    sc->cov64 = (double*)malloc(sizeof(double) * 6 * (size_t)(n ? n : 1));
    if (!sc->fac32 || !sc->cov64) return -1;
    for (int64_t i = 0; i < n; i++) {
        orc_factor32(s + 3 * i, q + 4 * i, sc->fac32 + 9 * i);
        orc_cov64(s + 3 * i, q + 4 * i, sc->cov64 + 6 * i);
    }
    return 0;
}

static void orc_scene_free(orc_scene* sc) { free(sc->fac32); free(sc->cov64); }

/* Per-view structure: projections and, per tile, the Gaussians whose tile
 * rectangle contains it, sorted by (depth key, Gaussian index) -- the ordered
 * set S_{d,p} of Sec. 3.1 shared by all pixels of the tile.                  */
typedef struct {
    orc_proj* g;
    int TX, TY;
    int64_t* start;   /* [TX*TY + 1] */
    int32_t* ids;     /* [P]         */
    int64_t P, nvis;
} orc_view;

static const orc_proj* g_sort_base;
static int orc_cmp(const void* a, const void* b)
{
    int32_t i = *(const int32_t*)a, j = *(const int32_t*)b;
    uint32_t di = g_sort_base[i].depth, dj = g_sort_base[j].depth;
    if (di != dj) return di < dj ? -1 : 1;
    return (i > j) - (i < j);
}

static int orc_view_build(const orc_scene* sc, const orc_cam* cam, orc_view* v)
{
    int64_t n = sc->n;
    v->TX = (cam->W + ORC_TILE - 1) / ORC_TILE;
    v->TY = (cam->H + ORC_TILE - 1) / ORC_TILE;
    int64_t nt = (int64_t)v->TX * v->TY;
    v->g = (orc_proj*)malloc(sizeof(orc_proj) * (size_t)(n ? n : 1));
    v->start = (int64_t*)calloc((size_t)nt + 1, sizeof(int64_t));
    if (!v->g || !v->start) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++)
        orc_project(sc->mu + 3 * i, sc->fac32 + 9 * i, sc->cov64 + 6 * i, sc->op[i], cam, v->g + i);
    v->nvis = 0;
    for (int64_t i = 0; i < n; i++) {
        const orc_proj* g = v->g + i;
        if (!g->vis) continue;
        v->nvis++;
        for (int y = g->y0; y < g->y1; y++)
            for (int x = g->x0; x < g->x1; x++) v->start[(int64_t)y * v->TX + x + 1]++;
    }
    for (int64_t t = 0; t < nt; t++) v->start[t + 1] += v->start[t];
    v->P = v->start[nt];
    v->ids = (int32_t*)malloc(sizeof(int32_t) * (size_t)(v->P ? v->P : 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nt ? nt : 1));
    if (!v->ids || !fill) return -1;
    memcpy(fill, v->start, sizeof(int64_t) * (size_t)nt);
    for (int64_t i = 0; i < n; i++) {
        const orc_proj* g = v->g + i;
        if (!g->vis) continue;
        for (int y = g->y0; y < g->y1; y++)
            for (int x = g->x0; x < g->x1; x++) v->ids[fill[(int64_t)y * v->TX + x]++] = (int32_t)i;
    }
    free(fill);
    g_sort_base = v->g;
    for (int64_t t = 0; t < nt; t++)
        qsort(v->ids + v->start[t], (size_t)(v->start[t + 1] - v->start[t]), sizeof(int32_t), orc_cmp);
    return 0;
}

static void orc_view_free(orc_view* v) { free(v->g); free(v->start); free(v->ids); }

/* alpha_i(p) of Sec. 3.1 in FP64: min(0.99, opacity * exp(power)), power =
 * -d^T Sigma2^-1 d / 2 clamped to <= 0 (it is <= 0 in exact arithmetic). */
static double orc_alpha(const orc_proj* g, double pxd, double pyd)
{
    double ex = pxd - g->ux64, ey = pyd - g->uy64;
    double p = fmin(0.0, g->A64 * ex * ex + g->B64 * ex * ey + g->C64 * ey * ey);
    return fmin((double)K_ALPHA_MAX, g->op64 * exp(p));
}

/* Decision log of one thread: smallest relative margins seen, ambiguous
 * pixels, and per Gaussian the number of ambiguous pixels at which it is
 * flagged (nullable). */
typedef struct {
    double thr;
    double min_skip, min_stop;
    int64_t amb_px;
    int32_t* flag;
} orc_dec;

/* One pixel's front-to-back walk (Eq. 1), every decision in FP64: a Gaussian
 * with alpha < 1/255 is skipped; the walk stops at the Gaussian that would
 * take T below 1e-4, which is not counted.  Calls `emit(i, w)` for every
 * counted Gaussian, in order, and returns the final transmittance.  With a
 * decision log, logs the margins and, if the pixel is ambiguous, flags the
 * Gaussians whose weight here depends on the ambiguous decision: a
 * different skip changes T for everything behind it, a different stop adds
 * or removes the stopping Gaussian, and a transmittance off by a factor
 * (1 - alpha) of a Gaussian near 1/255 can move the stop by at most the next
 * two candidates (each of which multiplies T by at most 1 - 1/255).       */
typedef void (*orc_emit_fn)(void* ctx, int32_t i, double w);

static double orc_walk(const orc_view* v, int64_t tile, int px, int py, orc_emit_fn emit,
                       void* ctx, orc_dec* dec, int* ambiguous)
{
    const double pxd = px + 0.5, pyd = py + 0.5;
    const double amin = K_ALPHA_MIN, teps = K_T_EPS;
    const int64_t k0 = v->start[tile], k1 = v->start[tile + 1];
    const double thr = dec ? dec->thr : -1.0;
    double T = 1.0;
    int64_t first = -1, k;
    for (k = k0; k < k1; k++) {
        const int32_t i = v->ids[k];
        const double a = orc_alpha(v->g + i, pxd, pyd);
        if (dec) {
            const double ms = fabs(a - amin) / amin;
            if (ms < dec->min_skip) dec->min_skip = ms;
            if (ms < thr && first < 0) first = k;
        }
        if (a < amin) continue;
        const double Tn = T * (1.0 - a);
        if (dec) {
            const double mt = fabs(Tn - teps) / teps;
            if (mt < dec->min_stop) dec->min_stop = mt;
            if (mt < thr && first < 0) first = k;
        }
        if (Tn < teps) break;
        emit(ctx, i, a * T);
        T = Tn;
    }
    if (ambiguous) *ambiguous = first >= 0;
    if (first >= 0) {
        dec->amb_px++;
        if (dec->flag) {
            int beyond = 0;
            for (int64_t j = first; j < k1; j++) {
                const int32_t i = v->ids[j];
                if (orc_alpha(v->g + i, pxd, pyd) < amin * (1.0 - thr)) continue;
                if (j > k && beyond++ == 2) break;
                dec->flag[i]++;
            }
        }
    }
    return T;
}

/* ----------------------------------------------------------------------- */
/* Accumulation context: U_r += w F_p, a_r += w |F_p| for accumulated rows r,
 * beta_i += w and count_i += 1 for every Gaussian.                           */
typedef struct {
    const float* F;    /* current pixel's D features */
    int D;
    const int32_t* row;  /* Gaussian -> accumulated row or -1; NULL = identity */
    double *U, *A, *beta;
    int64_t* cnt;
    int64_t nnz;
} orc_acc;

static void orc_emit_acc(void* vctx, int32_t i, double w)
{
    orc_acc* c = (orc_acc*)vctx;
    c->beta[i] += w;
    c->cnt[i] += 1;
    c->nnz++;
    int64_t r = c->row ? c->row[i] : i;
    if (r < 0) return;
    double* u = c->U + r * c->D;
    double* a = c->A + r * c->D;
    for (int k = 0; k < c->D; k++) {
        double f = c->F[k];
        u[k] += w * f;
        a[k] += w * fabs(f);
    }
}

static int orc_threads(int req)
{
#ifdef _OPENMP
    return req > 0 ? req : omp_get_max_threads();
#else
    (void)req;
    return 1;
#endif
}

/* Uplift one view (Eq. 3 numerator and denominator), ADDING into the
 * caller's FP64 accumulators:
 *   U[nrows][D] += sum_p w_i(p) F_p,   A[nrows][D] += sum_p w_i(p) |F_p|,
 *   beta[n] += sum_p w_i(p),           cnt[n] += #{p : i counted at p}.
 * F is [H][W][D] FP32 (HWC).  row[n] maps Gaussian -> accumulated row (or -1);
 * NULL means every Gaussian, nrows = n.  tfinal (nullable) gets the FP64 final
 * transmittance per pixel [H][W].
 * Decision log (see the header): amb_thr is the margin threshold; amb_px
 * (nullable, [H][W]) gets 1 at ambiguous pixels, 0 elsewhere; amb_flag
 * (nullable, [n]) += the number of ambiguous pixels at which each Gaussian is
 * flagged; margins[0..1] = min(margins, smallest skip / stop margin).
 * stats[0..3] += nnz, P, n_visible, ambiguous pixels.
 * Returns 0, or -1 on allocation failure.                                    */
int orc_uplift_view(int64_t n, const float* mu, const float* s, const float* q, const float* op,
                    const float* cam17, int W, int H, const float* F, int D, const int32_t* row,
                    int64_t nrows, double* U, double* A, double* beta, int64_t* cnt,
                    double* tfinal, uint8_t* amb_px, int32_t* amb_flag, double amb_thr,
                    double* margins, int64_t* stats, int nthreads)
{
    orc_scene sc;
    orc_view v;
    orc_cam cam = {cam17, W, H};
    memset(&v, 0, sizeof(v));
    if (orc_scene_init(&sc, n, mu, s, q, op) || orc_view_build(&sc, &cam, &v)) {
        orc_scene_free(&sc); orc_view_free(&v);
        return -1;
    }
    int nth = orc_threads(nthreads);
    int64_t nt = (int64_t)v.TX * v.TY;
    size_t rs = (size_t)nrows * (size_t)D;
    size_t nn = (size_t)(n ? n : 1);
    double** pu = (double**)calloc((size_t)nth, sizeof(double*));
    double** pa = (double**)calloc((size_t)nth, sizeof(double*));
    double** pb = (double**)calloc((size_t)nth, sizeof(double*));
    int64_t** pc = (int64_t**)calloc((size_t)nth, sizeof(int64_t*));
    int64_t* pn = (int64_t*)calloc((size_t)nth, sizeof(int64_t));
    orc_dec* pd = (orc_dec*)calloc((size_t)nth, sizeof(orc_dec));
    int fail = !pu || !pa || !pb || !pc || !pn || !pd;
    for (int t = 0; t < nth && !fail; t++) {
        pu[t] = (double*)calloc(rs ? rs : 1, sizeof(double));
        pa[t] = (double*)calloc(rs ? rs : 1, sizeof(double));
        pb[t] = (double*)calloc(nn, sizeof(double));
        pc[t] = (int64_t*)calloc(nn, sizeof(int64_t));
        pd[t].thr = amb_thr;
        pd[t].min_skip = pd[t].min_stop = INFINITY;
        pd[t].flag = amb_flag ? (int32_t*)calloc(nn, sizeof(int32_t)) : NULL;
        fail |= !pu[t] || !pa[t] || !pb[t] || !pc[t] || (amb_flag && !pd[t].flag);
    }
    if (!fail) {
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth)
        for (int64_t tile = 0; tile < nt; tile++) {
#ifdef _OPENMP
            int th = omp_get_thread_num();
#else
            int th = 0;
#endif
            orc_acc ctx = {0, D, row, pu[th], pa[th], pb[th], pc[th], 0};
            int tx = (int)(tile % v.TX), ty = (int)(tile / v.TX);
            for (int py = ty * ORC_TILE; py < (ty + 1) * ORC_TILE && py < H; py++)
                for (int px = tx * ORC_TILE; px < (tx + 1) * ORC_TILE && px < W; px++) {
                    int amb = 0;
                    ctx.F = F + ((int64_t)py * W + px) * D;
                    double T = orc_walk(&v, tile, px, py, orc_emit_acc, &ctx, pd + th, &amb);
                    if (tfinal) tfinal[(int64_t)py * W + px] = T;
                    if (amb_px) amb_px[(int64_t)py * W + px] = (uint8_t)amb;
                }
            pn[th] += ctx.nnz;
        }
        for (int t = 0; t < nth; t++) {
            for (size_t k = 0; k < rs; k++) { U[k] += pu[t][k]; A[k] += pa[t][k]; }
            for (int64_t i = 0; i < n; i++) { beta[i] += pb[t][i]; cnt[i] += pc[t][i]; }
            if (amb_flag)
                for (int64_t i = 0; i < n; i++) amb_flag[i] += pd[t].flag[i];
            if (margins) {
                margins[0] = fmin(margins[0], pd[t].min_skip);
                margins[1] = fmin(margins[1], pd[t].min_stop);
            }
            stats[0] += pn[t];
            stats[3] += pd[t].amb_px;
        }
        stats[1] += v.P;
        stats[2] += v.nvis;
    }
    for (int t = 0; t < nth; t++) {
        if (pu) free(pu[t]);
        if (pa) free(pa[t]);
        if (pb) free(pb[t]);
        if (pc) free(pc[t]);
        if (pd) free(pd[t].flag);
    }
    free(pu); free(pa); free(pb); free(pc); free(pn); free(pd);
    orc_view_free(&v);
    orc_scene_free(&sc);
    return fail ? -1 : 0;
}

/* ----------------------------------------------------------------------- */
/* Forward render of one view, Eq. (4): out[H][W][D] = sum_i w_i(p) g_i
 * (FP64 g [n][D]); alpha[H][W] (nullable) = sum_i w_i(p); amb_px[H][W]
 * (nullable) = 1 where the pixel is ambiguous at threshold amb_thr.       */
typedef struct { const double* g; double* out; double asum; int D; } orc_rctx;

static void orc_emit_render(void* vctx, int32_t i, double w)
{
    orc_rctx* c = (orc_rctx*)vctx;
    for (int k = 0; k < c->D; k++) c->out[k] += w * c->g[(int64_t)i * c->D + k];
    c->asum += w;
}

int orc_render_view(int64_t n, const float* mu, const float* s, const float* q, const float* op,
                    const float* cam17, int W, int H, const double* g, int D, double* out,
                    double* alpha, uint8_t* amb_px, double amb_thr, int nthreads)
{
    orc_scene sc;
    orc_view v;
    orc_cam cam = {cam17, W, H};
    memset(&v, 0, sizeof(v));
    if (orc_scene_init(&sc, n, mu, s, q, op) || orc_view_build(&sc, &cam, &v)) {
        orc_scene_free(&sc); orc_view_free(&v);
        return -1;
    }
    int nth = orc_threads(nthreads);
    int64_t nt = (int64_t)v.TX * v.TY;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth)
    for (int64_t tile = 0; tile < nt; tile++) {
        orc_dec dec = {amb_thr, INFINITY, INFINITY, 0, NULL};
        int tx = (int)(tile % v.TX), ty = (int)(tile / v.TX);
        for (int py = ty * ORC_TILE; py < (ty + 1) * ORC_TILE && py < H; py++)
            for (int px = tx * ORC_TILE; px < (tx + 1) * ORC_TILE && px < W; px++) {
                int amb = 0;
                orc_rctx c = {g, out + ((int64_t)py * W + px) * D, 0.0, D};
                for (int k = 0; k < D; k++) c.out[k] = 0.0;
                orc_walk(&v, tile, px, py, orc_emit_render, &c, &dec, &amb);
                if (alpha) alpha[(int64_t)py * W + px] = c.asum;
                if (amb_px) amb_px[(int64_t)py * W + px] = (uint8_t)amb;
            }
    }
    orc_view_free(&v);
    orc_scene_free(&sc);
    return 0;
}

/* ----------------------------------------------------------------------- */
/* Structure of one view, for bit-exact comparison.  Call with ids == NULL to
 * get P (returned); then with ids[P] and tile_start[TX*TY+1].  visible[n],
 * depth[n], rect[n][4] = (x0,y0,x1,y1) and center[n][2] (the S32 centre that
 * places the rectangle) are filled when non-NULL.  Returns P, or -1 on
 * allocation failure.                                                       */
int64_t orc_view_structure(int64_t n, const float* mu, const float* s, const float* q,
                           const float* op, const float* cam17, int W, int H, uint8_t* visible,
                           uint32_t* depth, int32_t* rect, float* center, int64_t* tile_start,
                           int32_t* ids)
{
    orc_scene sc;
    orc_view v;
    orc_cam cam = {cam17, W, H};
    memset(&v, 0, sizeof(v));
    if (orc_scene_init(&sc, n, mu, s, q, op) || orc_view_build(&sc, &cam, &v)) {
        orc_scene_free(&sc); orc_view_free(&v);
        return -1;
    }
    for (int64_t i = 0; i < n; i++) {
        const orc_proj* g = v.g + i;
        if (visible) visible[i] = (uint8_t)g->vis;
        if (depth) depth[i] = g->depth;
        if (rect) { rect[4 * i] = g->x0; rect[4 * i + 1] = g->y0; rect[4 * i + 2] = g->x1; rect[4 * i + 3] = g->y1; }
        if (center) { center[2 * i] = g->ux; center[2 * i + 1] = g->uy; }
    }
    int64_t nt = (int64_t)v.TX * v.TY;
    if (tile_start) memcpy(tile_start, v.start, sizeof(int64_t) * (size_t)(nt + 1));
    if (ids) memcpy(ids, v.ids, sizeof(int32_t) * (size_t)v.P);
    int64_t P = v.P;
    orc_view_free(&v);
    orc_scene_free(&sc);
    return P;
}

/* FP32 covariance factor M = R diag(s) of the S32 convention, [n][3][3]. */
void orc_factor32_array(int64_t n, const float* s, const float* q, float* out)
{
    for (int64_t i = 0; i < n; i++) orc_factor32(s + 3 * i, q + 4 * i, out + 9 * i);
}

/* Threads an oracle call uses by default. */
int orc_num_threads(void) { return orc_threads(0); }
