/* Host driver that runs the C oracle's entry points on small synthetic
 * inputs, built with AddressSanitizer and UndefinedBehaviorSanitizer by
 * test_oracle_sanitizers.py.  It checks memory safety and defined behaviour
 * of the oracle code paths (projection, tile lists, the walk with its
 * decision log, accumulation, render, structure); numerical results are
 * pinned by the Python tests.  Inputs come from a fixed linear congruential
 * generator; nothing here does any of the method's arithmetic. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_uplift_view(int64_t n, const float* mu, const float* s, const float* q, const float* op,
                    const float* cam17, int W, int H, const float* F, int D, const int32_t* row,
                    int64_t nrows, double* U, double* A, double* beta, int64_t* cnt,
                    double* tfinal, uint8_t* amb_px, int32_t* amb_flag, double amb_thr,
                    double* margins, int64_t* stats, int nthreads);
int orc_render_view(int64_t n, const float* mu, const float* s, const float* q, const float* op,
                    const float* cam17, int W, int H, const double* g, int D, double* out,
                    double* alpha, uint8_t* amb_px, double amb_thr, int nthreads);
int64_t orc_view_structure(int64_t n, const float* mu, const float* s, const float* q,
                           const float* op, const float* cam17, int W, int H, uint8_t* visible,
                           uint32_t* depth, int32_t* rect, float* center, int64_t* tile_start,
                           int32_t* ids);
void orc_factor32_array(int64_t n, const float* s, const float* q, float* out);

static uint64_t st = 88172645463325252ull;
static float u01(void) {
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    return (float)((st >> 40) & 0xFFFFFF) / 16777216.0f;
}

int main(void) {
    const int64_t n = 1500;
    const int W = 61, H = 47, D = 3;  /* ragged tiles */
    float* mu = malloc(sizeof(float) * 3 * n);
    float* s = malloc(sizeof(float) * 3 * n);
    float* q = malloc(sizeof(float) * 4 * n);
    float* op = malloc(sizeof(float) * n);
    for (int64_t i = 0; i < n; i++) {
        for (int k = 0; k < 3; k++) {
            mu[3 * i + k] = 2.0f * u01() - 1.0f;
            s[3 * i + k] = 0.005f + 0.08f * u01();
        }
        for (int k = 0; k < 4; k++) q[4 * i + k] = u01() - 0.5f;
        op[i] = 0.05f + 0.94f * u01();
    }
    /* camera on the z axis looking at the origin (R = I), one inside the cloud */
    float cams[2][17] = {{1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 4.0f, 60, 60, 30.5f, 23.5f, 0.01f},
                         {1, 0, 0, 0, 1, 0, 0, 0, 1, 0.1f, 0, 0.3f, 30, 30, 30.5f, 23.5f, 0.01f}};
    float* F = malloc(sizeof(float) * W * H * D);
    for (int i = 0; i < W * H * D; i++) F[i] = u01();
    double* U = calloc((size_t)n * D, sizeof(double));
    double* A = calloc((size_t)n * D, sizeof(double));
    double* beta = calloc((size_t)n, sizeof(double));
    int64_t* cnt = calloc((size_t)n, sizeof(int64_t));
    double* tf = calloc((size_t)W * H, sizeof(double));
    uint8_t* amb = calloc((size_t)W * H, 1);
    int32_t* flag = calloc((size_t)n, sizeof(int32_t));
    double margins[2] = {INFINITY, INFINITY};
    int64_t stats[4] = {0, 0, 0, 0};
    int32_t rows[1500];
    for (int64_t i = 0; i < n; i++) rows[i] = (i % 3 == 0) ? (int32_t)(i / 3) : -1;
    for (int c = 0; c < 2; c++) {
        if (orc_uplift_view(n, mu, s, q, op, cams[c], W, H, F, D, NULL, n, U, A, beta, cnt, tf, amb,
                            flag, 1e-5, margins, stats, 2))
            return 2;
        memset(U, 0, sizeof(double) * n * D);
        if (orc_uplift_view(n, mu, s, q, op, cams[c], W, H, F, D, rows, 500, U, A, beta, cnt, NULL,
                            NULL, NULL, 1e-5, NULL, stats, 1))
            return 3;
        double* g = calloc((size_t)n * D, sizeof(double));
        double* out = calloc((size_t)W * H * D, sizeof(double));
        double* al = calloc((size_t)W * H, sizeof(double));
        for (int64_t i = 0; i < n * D; i++) g[i] = u01();
        if (orc_render_view(n, mu, s, q, op, cams[c], W, H, g, D, out, al, amb, 1e-5, 2)) return 4;
        int64_t P = orc_view_structure(n, mu, s, q, op, cams[c], W, H, NULL, NULL, NULL, NULL, NULL, NULL);
        if (P < 0) return 5;
        uint8_t* vis = calloc((size_t)n, 1);
        uint32_t* dep = calloc((size_t)n, 4);
        int32_t* rect = calloc((size_t)n * 4, 4);
        float* ctr = calloc((size_t)n * 2, 4);
        int64_t* ts = calloc((size_t)(((W + 15) / 16) * ((H + 15) / 16) + 1), 8);
        int32_t* ids = calloc((size_t)(P > 0 ? P : 1), 4);
        if (orc_view_structure(n, mu, s, q, op, cams[c], W, H, vis, dep, rect, ctr, ts, ids) != P) return 6;
        free(g); free(out); free(al); free(vis); free(dep); free(rect); free(ctr); free(ts); free(ids);
    }
    /* empty scene */
    if (orc_uplift_view(0, mu, s, q, op, cams[0], W, H, F, D, NULL, 0, U, A, beta, cnt, NULL, NULL,
                        NULL, 1e-5, margins, stats, 1))
        return 7;
    float* fac = malloc(sizeof(float) * 9 * n);
    orc_factor32_array(n, s, q, fac);
    printf("ok nnz=%lld P=%lld ambiguous=%lld\n", (long long)stats[0], (long long)stats[1],
           (long long)stats[3]);
    free(mu); free(s); free(q); free(op); free(F); free(U); free(A); free(beta); free(cnt); free(tf);
    free(amb); free(flag); free(fac);
    return 0;
}
