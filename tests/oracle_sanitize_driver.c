/* oracle_sanitize_driver.c -- runs every entry point of the CPU oracle on
 * small random clouds, for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py).  Inputs come
 * from a fixed-seed xorshift generator; the driver checks return codes and a
 * few invariants, and prints "ok" when every call succeeded. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "vicp_oracle.h"

static uint64_t g_state = 0x9E3779B97F4A7C15ull;

static double uniform(void)
{
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return (double)(g_state >> 11) * (1.0 / 9007199254740992.0);
}

static void cloud(float* x, float* y, float* z, int64_t k, float scale, float shift)
{
    for (int64_t i = 0; i < k; ++i) {
        x[i] = (float)((2.0 * uniform() - 1.0) * scale) + shift;
        y[i] = (float)((2.0 * uniform() - 1.0) * scale);
        z[i] = (float)((2.0 * uniform() - 1.0) * scale);
    }
}

#define CHECK(expr)                                                            \
    do {                                                                       \
        int rc_ = (expr);                                                      \
        if (rc_ != VICPO_OK) {                                                 \
            fprintf(stderr, "%s:%d: %s returned %d\n", __FILE__, __LINE__, #expr, rc_); \
            return 1;                                                          \
        }                                                                      \
    } while (0)

static int one_case(int64_t n, int64_t m, float voxel, int32_t rings, float src_scale, int64_t cap)
{
    float* q = (float*)malloc(sizeof(float) * 3 * (size_t)n);
    float* p = (float*)malloc(sizeof(float) * 3 * (size_t)m);
    float *qx = q, *qy = q + n, *qz = q + 2 * n, *px = p, *py = p + m, *pz = p + 2 * m;
    cloud(qx, qy, qz, n, 1.0f, 0.0f);
    if (n > 8)   /* exact duplicates: ties go to the lower index */
        for (int a = 0; a < 4; ++a) {
            qx[n - 1 - a] = qx[a];
            qy[n - 1 - a] = qy[a];
            qz[n - 1 - a] = qz[a];
        }
    cloud(px, py, pz, m, src_scale, 0.05f);
    float origin[3], inv;
    int32_t dims[3];
    int64_t V;
    CHECK(vicpo_grid_spec(qx, qy, qz, n, voxel, rings, origin, &inv, dims, &V));
    uint32_t* hist = (uint32_t*)calloc((size_t)V, sizeof(uint32_t));
    uint32_t* off = (uint32_t*)calloc((size_t)V + 1, sizeof(uint32_t));
    uint32_t* vm = (uint32_t*)calloc((size_t)(n + 2 * V), sizeof(uint32_t));
    uint32_t* roots = (uint32_t*)calloc((size_t)V, sizeof(uint32_t));
    int64_t* vid = (int64_t*)calloc((size_t)m, sizeof(int64_t));
    int32_t* idx = (int32_t*)calloc((size_t)m, sizeof(int32_t));
    float* d2 = (float*)calloc((size_t)m, sizeof(float));
    CHECK(vicpo_voxel_ids(px, py, pz, m, origin, inv, dims, vid));
    CHECK(vicpo_build(qx, qy, qz, n, origin, inv, dims, V, hist, off, vm));
    if (off[V] != (uint32_t)(n + 2 * V)) return 1;
    CHECK(vicpo_dilate(dims, V, hist, off, rings, vm, roots));
    const float Rt[12] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 0.01f, -0.02f, 0.0f};
    int64_t F = 0, Ct = 0, Dl = 0;
    CHECK(vicpo_nns(qx, qy, qz, n, origin, inv, dims, off, vm, px, py, pz, m, Rt, idx, d2, &F, &Ct, &Dl));
    CHECK(vicpo_nns_cap(qx, qy, qz, n, origin, inv, dims, off, vm, px, py, pz, m, Rt, cap, idx, d2, &F, &Ct, &Dl));
    for (int64_t i = 0; i < m; ++i)
        if (idx[i] < 0 || idx[i] >= n) return 1;
    double prev[12] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0}, out[12], sv[3];
    int32_t deg = 0;
    CHECK(vicpo_solve(px, py, pz, qx, qy, qz, idx, m, prev, out, sv, &deg));
    const int32_t K = 5;
    double Rt_io[12] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0};
    double rmse[5];
    int64_t fb[5];
    int32_t iters = 0, dh[5];
    CHECK(vicpo_register(qx, qy, qz, n, px, py, pz, m, voxel, rings, K, 1e-5, 1, Rt_io, rmse, fb, &iters, dh, idx,
                         d2));
    if (iters < 1 || iters > K) return 1;
    memcpy(Rt_io, prev, sizeof prev);
    CHECK(vicpo_register_cap(qx, qy, qz, n, px, py, pz, m, origin, inv, dims, V, rings, cap, K, 1e-5, 0, Rt_io, rmse,
                             fb, &iters, dh, idx, d2));
    double xi[6] = {0.01, -0.02, 0.005, 0.03, -0.01, 0.02}, R[9], t[3], J[36];
    vicpo_se3_exp(xi, R, t, J);
    double* p64 = (double*)malloc(sizeof(double) * 3 * (size_t)m);
    for (int64_t i = 0; i < 3 * m; ++i) p64[i] = (double)p[i];
    double* dp = (double*)calloc(3 * (size_t)m, sizeof(double));
    double loss = 0.0, dxi[6];
    CHECK(vicpo_p2p(qx, qy, qz, n, origin, inv, dims, off, vm, px, py, pz, m, xi, &loss, dp, dp + m, dp + 2 * m, dxi,
                    idx));
    const double lf = vicpo_p2p_loss_fixed(qx, qy, qz, p64, p64 + m, p64 + 2 * m, m, idx, xi);
    if (!(fabs(lf - loss) <= 1e-9 * (1.0 + fabs(loss)))) return 1;
    free(q);
    free(p);
    free(hist);
    free(off);
    free(vm);
    free(roots);
    free(vid);
    free(idx);
    free(d2);
    free(p64);
    free(dp);
    return 0;
}

int main(void)
{
    /* a regular case, a one-voxel grid, a coarse grid with capacity overflow,
     * sources far outside (every query global), and a single target point */
    if (one_case(600, 400, 0.2f, 2, 1.2f, 0)) return 1;
    if (one_case(300, 200, 10.0f, 0, 0.5f, 0)) return 1;
    if (one_case(900, 300, 0.5f, 3, 1.1f, 16)) return 1;
    if (one_case(200, 150, 0.1f, 1, 30.0f, 0)) return 1;
    if (one_case(1, 50, 0.3f, 2, 1.0f, 0)) return 1;
    /* error paths */
    float x = 0.0f, o[3];
    float inv;
    int32_t d[3];
    int64_t V;
    if (vicpo_grid_spec(&x, &x, &x, 1, 0.0f, 1, o, &inv, d, &V) == VICPO_OK) return 1;
    if (vicpo_grid_spec(&x, &x, &x, 1, 1e-9f, 1, o, &inv, d, &V) == VICPO_OK) {
        /* a tiny voxel around one point is a small grid: fine either way */
    }
    printf("ok\n");
    return 0;
}
