/*
 * vicp_oracle.c -- plain, slow CPU oracle of dilation-based ICP with the
 * segmented (offset-addressed) dilation memory of Chang, Wang, Zhong and
 * Miyazaki, "A dynamic memory assignment strategy for dilation-based ICP
 * algorithm on embedded GPUs" (arXiv 2512.04996).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU path is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, table or helper
 * with the HIP library, and the HIP library never calls it.
 *
 * Every step runs in the order the paper states it, with no blocking or
 * fusion, single-threaded by default.  The one exception is optional: the
 * per-query loop of Alg. 4 may run on several threads (vicpo_set_threads,
 * OpenMP), because each query's search reads only the grid and writes only
 * its own result slot; the counters are integer sums, so every output is the
 * same for any thread count.  Build with -ffp-contract=off so that every float32
 * expression rounds exactly as written: the voxel quantisation and the
 * float32 distances decide integers (voxel ids, nearest-neighbour indices),
 * so they are evaluated in float32, the precision the GPU kernels use.
 * Everything else (moments, the rigid-transform solve, RMSE, the
 * differentiable loss and its gradients) is float64.
 *
 * Readings of the paper where it is silent, ambiguous or garbled (each is
 * marked "reading:" below):
 *  - grid: the target's axis-aligned box padded by L voxels; voxel index
 *    floor((x - origin) * (1/s)), x fastest (Alg. 1 "Quantize"/"Concat" and
 *    the neighbour offsets of Alg. 3);
 *  - offsets: exclusive scan of count + 2 for every voxel (Alg. 1, CPU part;
 *    both arms of its branch equal count + 2), one extra entry = total;
 *  - segments: [lock = 0, count, point indices ascending] (Alg. 2 and Fig. 3;
 *    the paper's lock order is nondeterministic, ascending is canonical; the
 *    indices start two words after the segment head as Alg. 2 writes them);
 *  - dilation: exactly L synchronous rings over the six in-bounds face
 *    neighbours, each empty voxel takes the lowest root id among its
 *    neighbours' previous-ring roots, root = the occupied voxel, stored as
 *    Mask(root) = root | 2^31 in the count slot (Alg. 3);
 *  - NNS: the voxel of the transformed source point, its own segment when it
 *    holds points, its root's segment when dilated, otherwise (empty and
 *    undilated, or outside the grid) an exact search over every target point
 *    (Alg. 4); ties go to the lowest target index;
 *  - solve: the closed-form least-squares rigid transform of Eq. 1 on the
 *    original source points, computed here with Horn's unit-quaternion method;
 *    when the cross-covariance has rank below two the previous pose is kept.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "vicp_oracle.h"

#ifdef _OPENMP
#include <omp.h>
#endif

#define MASK_BIT 0x80000000u
#define NONE_ROOT 0xFFFFFFFFu

static int g_threads = 1;

/* Threads of the per-query loop of Alg. 4 (1 = single-threaded, the
 * default); returns the count in force (always 1 without OpenMP). */
int vicpo_set_threads(int32_t k)
{
#ifdef _OPENMP
    g_threads = k < 1 ? 1 : k;
#else
    (void)k;
    g_threads = 1;
#endif
    return g_threads;
}

/* ------------------------------------------------------------------------ */
/* grid specification (Sec. II.A Step 1; Alg. 1 "Quantize")                  */
/* ------------------------------------------------------------------------ */

int vicpo_grid_spec(const float* qx, const float* qy, const float* qz, int64_t n,
                    float voxel, int32_t rings, float origin[3], float* inv,
                    int32_t dims[3], int64_t* V)
{
    if (n <= 0 || !(voxel > 0.0f) || !isfinite(voxel) || rings < 0)
        return VICPO_ERR_ARG;
    const float* c[3] = {qx, qy, qz};
    float lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = c[a][0];
        hi[a] = c[a][0];
        for (int64_t i = 0; i < n; ++i) {
            float x = c[a][i];
            if (!isfinite(x)) return VICPO_ERR_NONFINITE;
            if (x < lo[a]) lo[a] = x;
            if (x > hi[a]) hi[a] = x;
        }
    }
    /* reading: one reciprocal rounded once, the origin is the box corner
     * moved out by L voxels, each a separate float32 rounding. */
    float iv = 1.0f / voxel;
    float pad = (float)rings * voxel;
    int64_t VV = 1;
    for (int a = 0; a < 3; ++a) {
        origin[a] = lo[a] - pad;
        float f = (hi[a] - origin[a]) * iv;
        if (!(f < 1073741824.0f)) return VICPO_ERR_TOO_LARGE;
        int64_t d = (int64_t)floorf(f) + 1 + rings;
        if (d > 2147483647LL) return VICPO_ERR_TOO_LARGE;
        dims[a] = (int32_t)d;
        VV *= d;
        if (VV >= 2147483648LL) return VICPO_ERR_TOO_LARGE;
    }
    if (n + 2 * VV >= 4294967296LL) return VICPO_ERR_TOO_LARGE;
    *inv = iv;
    *V = VV;
    return VICPO_OK;
}

/* Voxel of a point; returns 1 and sets *v when inside the grid, else 0.
 * reading: inside means 0 <= f_a < D_a for each axis, compared as floats
 * before any integer conversion. */
static int voxel_of(const float origin[3], float inv, const int32_t dims[3],
                    float x, float y, float z, int64_t* v)
{
    float f[3];
    f[0] = (x - origin[0]) * inv;
    f[1] = (y - origin[1]) * inv;
    f[2] = (z - origin[2]) * inv;
    for (int a = 0; a < 3; ++a)
        if (!(f[a] >= 0.0f && f[a] < (float)dims[a])) return 0;
    int64_t ix = (int64_t)floorf(f[0]);
    int64_t iy = (int64_t)floorf(f[1]);
    int64_t iz = (int64_t)floorf(f[2]);
    *v = ix + (int64_t)dims[0] * (iy + (int64_t)dims[1] * iz);
    return 1;
}

int vicpo_voxel_ids(const float* x, const float* y, const float* z, int64_t k,
                    const float origin[3], float inv, const int32_t dims[3], int64_t* out)
{
    for (int64_t i = 0; i < k; ++i) {
        int64_t v;
        out[i] = voxel_of(origin, inv, dims, x[i], y[i], z[i], &v) ? v : -1;
    }
    return VICPO_OK;
}

/* ------------------------------------------------------------------------ */
/* counts, offsets, segments (Alg. 1 and Alg. 2)                             */
/* ------------------------------------------------------------------------ */

int vicpo_build(const float* qx, const float* qy, const float* qz, int64_t n,
                const float origin[3], float inv, const int32_t dims[3], int64_t V,
                uint32_t* hist, uint32_t* off, uint32_t* vm)
{
    int64_t* vid = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!vid) return VICPO_ERR_OOM;
    /* Alg. 1, GPU part: histogram of target points per voxel. */
    for (int64_t v = 0; v < V; ++v) hist[v] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t v;
        if (!voxel_of(origin, inv, dims, qx[i], qy[i], qz[i], &v)) {
            free(vid);
            return VICPO_ERR_INTERNAL; /* a target outside its own grid */
        }
        vid[i] = v;
        hist[v] += 1;
    }
    /* Alg. 1, CPU part: running head address, count + 2 words per voxel. */
    uint64_t head = 0;
    for (int64_t v = 0; v < V; ++v) {
        off[v] = (uint32_t)head;
        head += (uint64_t)hist[v] + 2;
    }
    off[V] = (uint32_t)head;
    /* Alg. 2: each voxel's segment holds [lock, count, indices...]; walking
     * the points in index order appends them in ascending order. */
    for (int64_t v = 0; v < V; ++v) {
        vm[off[v]] = 0;
        vm[off[v] + 1] = 0;
    }
    for (int64_t i = 0; i < n; ++i) {
        uint32_t a = off[vid[i]];
        uint32_t cnt = vm[a + 1];
        vm[a + 2 + cnt] = (uint32_t)i;
        vm[a + 1] = cnt + 1;
    }
    free(vid);
    return VICPO_OK;
}

/* ------------------------------------------------------------------------ */
/* dilation (Alg. 3): L synchronous rings, six face neighbours, no wrap      */
/* ------------------------------------------------------------------------ */

int vicpo_dilate(const int32_t dims[3], int64_t V, const uint32_t* hist,
                 const uint32_t* off, int32_t rings, uint32_t* vm, uint32_t* roots_out)
{
    if (rings < 0) return VICPO_ERR_ARG;
    uint32_t* cur = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)V);
    uint32_t* nxt = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)V);
    if (!cur || !nxt) {
        free(cur);
        free(nxt);
        return VICPO_ERR_OOM;
    }
    for (int64_t v = 0; v < V; ++v) cur[v] = hist[v] > 0 ? (uint32_t)v : NONE_ROOT;
    const int64_t Dx = dims[0], Dy = dims[1], Dz = dims[2];
    for (int32_t r = 1; r <= rings; ++r) {
        for (int64_t v = 0; v < V; ++v) {
            if (cur[v] != NONE_ROOT) {
                nxt[v] = cur[v];
                continue;
            }
            int64_t x = v % Dx, y = (v / Dx) % Dy, z = v / (Dx * Dy);
            uint32_t best = NONE_ROOT;
            int64_t nb[6];
            int k = 0;
            if (x > 0) nb[k++] = v - 1;
            if (x + 1 < Dx) nb[k++] = v + 1;
            if (y > 0) nb[k++] = v - Dx;
            if (y + 1 < Dy) nb[k++] = v + Dx;
            if (z > 0) nb[k++] = v - Dx * Dy;
            if (z + 1 < Dz) nb[k++] = v + Dx * Dy;
            for (int j = 0; j < k; ++j)
                if (cur[nb[j]] < best) best = cur[nb[j]];
            nxt[v] = best;
        }
        uint32_t* t = cur;
        cur = nxt;
        nxt = t;
    }
    for (int64_t v = 0; v < V; ++v) {
        if (hist[v] == 0 && cur[v] != NONE_ROOT) vm[off[v] + 1] = cur[v] | MASK_BIT;
        if (roots_out) roots_out[v] = cur[v];
    }
    free(cur);
    free(nxt);
    return VICPO_OK;
}

/* ------------------------------------------------------------------------ */
/* nearest-neighbour search (Alg. 4)                                         */
/* ------------------------------------------------------------------------ */

/* float32 squared distance with a fixed operation order:
 * dx*dx, then fma(dy, dy, .), then fma(dz, dz, .). */
static float dist2(float sx, float sy, float sz, float qx, float qy, float qz)
{
    float dx = sx - qx, dy = sy - qy, dz = sz - qz;
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

static void transform_f32(const float Rt[12], float px, float py, float pz, float s[3])
{
    /* reading: R row-major then t; each row as fma(R0, x, fma(R1, y, fma(R2, z, t))). */
    s[0] = fmaf(Rt[0], px, fmaf(Rt[1], py, fmaf(Rt[2], pz, Rt[9])));
    s[1] = fmaf(Rt[3], px, fmaf(Rt[4], py, fmaf(Rt[5], pz, Rt[10])));
    s[2] = fmaf(Rt[6], px, fmaf(Rt[7], py, fmaf(Rt[8], pz, Rt[11])));
}

int vicpo_nns(const float* qx, const float* qy, const float* qz, int64_t n,
              const float origin[3], float inv, const int32_t dims[3],
              const uint32_t* off, const uint32_t* vm,
              const float* px, const float* py, const float* pz, int64_t m,
              const float Rt[12], int32_t* nn_idx, float* nn_d2, int64_t* n_fallback,
              int64_t* cand_total, int64_t* dilated_total)
{
    return vicpo_nns_cap(qx, qy, qz, n, origin, inv, dims, off, vm, px, py, pz, m, Rt, 0, nn_idx, nn_d2,
                         n_fallback, cand_total, dilated_total);
}

/* Alg. 4 under a per-voxel capacity (VANICP's fixed memory block per voxel,
 * Sec. II.B): when the points a query would search (its own voxel's, or its
 * root's for a dilated voxel) number more than `capacity`, they do not fit a
 * block, and the query takes the global search instead (Sec. IV.B: points
 * beyond a voxel's capacity force the global search).  capacity <= 0: no
 * limit, which is Alg. 4 itself.  A query counts as dilated only when it is
 * resolved through its root's points. */
int vicpo_nns_cap(const float* qx, const float* qy, const float* qz, int64_t n,
                  const float origin[3], float inv, const int32_t dims[3],
                  const uint32_t* off, const uint32_t* vm,
                  const float* px, const float* py, const float* pz, int64_t m,
                  const float Rt[12], int64_t capacity, int32_t* nn_idx, float* nn_d2,
                  int64_t* n_fallback, int64_t* cand_total, int64_t* dilated_total)
{
    int64_t F = 0, C = 0, Dl = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : F, C, Dl) num_threads(g_threads) if (g_threads > 1)
#endif
    for (int64_t i = 0; i < m; ++i) {
        float s[3];
        transform_f32(Rt, px[i], py[i], pz[i], s);
        /* Alg. 4: voxel of the source point, then its count-or-mask word. */
        int64_t v;
        int local = 0;
        uint32_t seg_head = 0, count = 0;
        if (voxel_of(origin, inv, dims, s[0], s[1], s[2], &v)) {
            uint32_t h = vm[off[v] + 1];
            int dilated = (h & MASK_BIT) != 0;
            if (dilated) {
                /* a dilated voxel: its Mask(root) word sends the search to the root */
                uint32_t root = h & ~MASK_BIT;
                seg_head = off[root];
                count = vm[seg_head + 1];
            } else {
                seg_head = off[v];
                count = h;
            }
            local = count > 0 && (capacity <= 0 || (int64_t)count <= capacity);
            if (local && dilated) Dl += 1;
        }
        float bd = INFINITY;
        int64_t bj = -1;
        if (local) {
            for (uint32_t k = 0; k < count; ++k) {
                int64_t j = vm[seg_head + 2 + k];
                float d = dist2(s[0], s[1], s[2], qx[j], qy[j], qz[j]);
                if (bj < 0 || d < bd || (d == bd && j < bj)) {
                    bd = d;
                    bj = j;
                }
            }
            C += count;
        } else {
            for (int64_t j = 0; j < n; ++j) {
                float d = dist2(s[0], s[1], s[2], qx[j], qy[j], qz[j]);
                if (bj < 0 || d < bd || (d == bd && j < bj)) {
                    bd = d;
                    bj = j;
                }
            }
            F += 1;
            C += n;
        }
        nn_idx[i] = (int32_t)bj;
        nn_d2[i] = bd;
    }
    if (n_fallback) *n_fallback = F;
    if (cand_total) *cand_total = C;
    if (dilated_total) *dilated_total = Dl;
    return VICPO_OK;
}

/* ------------------------------------------------------------------------ */
/* rigid-transform solve for Eq. 1 (Horn's unit quaternion, float64)         */
/* ------------------------------------------------------------------------ */

/* Cyclic Jacobi eigen-decomposition of a symmetric k x k matrix (k <= 4).
 * A is destroyed; evals[i] and column i of evec are an eigenpair. */
static void jacobi_eig(int k, double A[4][4], double evals[4], double evec[4][4])
{
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) evec[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 64; ++sweep) {
        double offd = 0.0, diag = 0.0;
        for (int i = 0; i < k; ++i) {
            diag += A[i][i] * A[i][i];
            for (int j = i + 1; j < k; ++j) offd += A[i][j] * A[i][j];
        }
        if (offd == 0.0 || offd <= 1e-36 * diag) break;
        for (int p = 0; p < k; ++p) {
            for (int q = p + 1; q < k; ++q) {
                if (A[p][q] == 0.0) continue;
                /* rotation in the (p, q) plane that zeroes A[p][q] */
                double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                for (int r = 0; r < k; ++r) {
                    double arp = A[r][p], arq = A[r][q];
                    A[r][p] = c * arp - s * arq;
                    A[r][q] = s * arp + c * arq;
                }
                for (int r = 0; r < k; ++r) {
                    double apr = A[p][r], aqr = A[q][r];
                    A[p][r] = c * apr - s * aqr;
                    A[q][r] = s * apr + c * aqr;
                }
                for (int r = 0; r < k; ++r) {
                    double vrp = evec[r][p], vrq = evec[r][q];
                    evec[r][p] = c * vrp - s * vrq;
                    evec[r][q] = s * vrp + c * vrq;
                }
            }
        }
    }
    for (int i = 0; i < k; ++i) evals[i] = A[i][i];
}

int vicpo_solve(const float* px, const float* py, const float* pz,
                const float* qx, const float* qy, const float* qz,
                const int32_t* idx, int64_t m, const double Rt_prev[12],
                double Rt_out[12], double sv_out[3], int32_t* degenerate)
{
    memcpy(Rt_out, Rt_prev, sizeof(double) * 12);
    *degenerate = 0;
    if (m <= 0) {
        *degenerate = 1;
        return VICPO_OK;
    }
    /* centroids, summed in index order */
    double pb[3] = {0, 0, 0}, qb[3] = {0, 0, 0};
    for (int64_t i = 0; i < m; ++i) {
        int64_t j = idx[i];
        pb[0] += px[i];
        pb[1] += py[i];
        pb[2] += pz[i];
        qb[0] += qx[j];
        qb[1] += qy[j];
        qb[2] += qz[j];
    }
    for (int a = 0; a < 3; ++a) {
        pb[a] /= (double)m;
        qb[a] /= (double)m;
    }
    /* cross-covariance S[a][b] = sum (p - pbar)_a (q - qbar)_b */
    double S[3][3] = {{0}};
    for (int64_t i = 0; i < m; ++i) {
        int64_t j = idx[i];
        double pc[3] = {px[i] - pb[0], py[i] - pb[1], pz[i] - pb[2]};
        double qc[3] = {qx[j] - qb[0], qy[j] - qb[1], qz[j] - qb[2]};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) S[a][b] += pc[a] * qc[b];
    }
    /* rank test on the singular values of S (eigenvalues of S^T S) */
    double G[4][4] = {{0}}, gev[4], gvec[4][4];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int r = 0; r < 3; ++r) acc += S[r][a] * S[r][b];
            G[a][b] = acc;
        }
    jacobi_eig(3, G, gev, gvec);
    double sv[3];
    for (int a = 0; a < 3; ++a) sv[a] = sqrt(gev[a] > 0.0 ? gev[a] : 0.0);
    /* sort descending */
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            if (sv[b] > sv[a]) {
                double t = sv[a];
                sv[a] = sv[b];
                sv[b] = t;
            }
    if (sv_out) memcpy(sv_out, sv, sizeof sv);
    if (!(sv[0] > 0.0) || sv[1] <= 1e-12 * sv[0]) {
        *degenerate = 1;
        return VICPO_OK;
    }
    /* Horn's symmetric 4x4 matrix; its top eigenvector is the quaternion of
     * the rotation taking the centred source onto the centred target. */
    double Sxx = S[0][0], Sxy = S[0][1], Sxz = S[0][2];
    double Syx = S[1][0], Syy = S[1][1], Syz = S[1][2];
    double Szx = S[2][0], Szy = S[2][1], Szz = S[2][2];
    double N[4][4] = {
        {Sxx + Syy + Szz, Syz - Szy, Szx - Sxz, Sxy - Syx},
        {Syz - Szy, Sxx - Syy - Szz, Sxy + Syx, Szx + Sxz},
        {Szx - Sxz, Sxy + Syx, -Sxx + Syy - Szz, Syz + Szy},
        {Sxy - Syx, Szx + Sxz, Syz + Szy, -Sxx - Syy + Szz},
    };
    double ev[4], vec[4][4];
    jacobi_eig(4, N, ev, vec);
    int top = 0;
    for (int i = 1; i < 4; ++i)
        if (ev[i] > ev[top]) top = i;
    double w = vec[0][top], x = vec[1][top], y = vec[2][top], z = vec[3][top];
    double nrm = sqrt(w * w + x * x + y * y + z * z);
    w /= nrm;
    x /= nrm;
    y /= nrm;
    z /= nrm;
    double R[9] = {
        w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (y * x + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x),
        2 * (z * x - w * y), 2 * (z * y + w * x), w * w - x * x - y * y + z * z,
    };
    for (int a = 0; a < 9; ++a) Rt_out[a] = R[a];
    for (int a = 0; a < 3; ++a)
        Rt_out[9 + a] = qb[a] - (R[3 * a] * pb[0] + R[3 * a + 1] * pb[1] + R[3 * a + 2] * pb[2]);
    return VICPO_OK;
}

/* ------------------------------------------------------------------------ */
/* ICP iteration (Sec. II.A; stop rule of Sec. IV.A)                         */
/* ------------------------------------------------------------------------ */

int vicpo_register(const float* qx, const float* qy, const float* qz, int64_t n,
                   const float* px, const float* py, const float* pz, int64_t m,
                   float voxel, int32_t rings, int32_t max_iter, double rmse_eps,
                   int32_t early_stop, double Rt_io[12], double* rmse_hist,
                   int64_t* fb_hist, int32_t* iters_done, int32_t* degenerate_hist,
                   int32_t* nn_idx, float* nn_d2)
{
    *iters_done = 0;
    if (m == 0) return VICPO_OK;
    if (m < 0 || max_iter < 0) return VICPO_ERR_ARG;
    float origin[3], inv;
    int32_t dims[3];
    int64_t V;
    int rc = vicpo_grid_spec(qx, qy, qz, n, voxel, rings, origin, &inv, dims, &V);
    if (rc) return rc;
    return vicpo_register_spec(qx, qy, qz, n, px, py, pz, m, origin, inv, dims, V, rings, max_iter, rmse_eps,
                               early_stop, Rt_io, rmse_hist, fb_hist, iters_done, degenerate_hist, nn_idx, nn_d2);
}

/* The same on a given grid (origin, 1/voxel, dims), e.g. the fixed 2^N grid
 * over the unit sphere's cube of Sec. IV.A. */
int vicpo_register_spec(const float* qx, const float* qy, const float* qz, int64_t n,
                        const float* px, const float* py, const float* pz, int64_t m,
                        const float origin[3], float inv, const int32_t dims[3], int64_t V,
                        int32_t rings, int32_t max_iter, double rmse_eps,
                        int32_t early_stop, double Rt_io[12], double* rmse_hist,
                        int64_t* fb_hist, int32_t* iters_done, int32_t* degenerate_hist,
                        int32_t* nn_idx, float* nn_d2)
{
    return vicpo_register_cap(qx, qy, qz, n, px, py, pz, m, origin, inv, dims, V, rings, 0, max_iter, rmse_eps,
                              early_stop, Rt_io, rmse_hist, fb_hist, iters_done, degenerate_hist, nn_idx, nn_d2);
}

/* The same with the per-voxel capacity of vicpo_nns_cap (VANICP's fixed
 * blocks; capacity <= 0: no limit). */
int vicpo_register_cap(const float* qx, const float* qy, const float* qz, int64_t n,
                       const float* px, const float* py, const float* pz, int64_t m,
                       const float origin[3], float inv, const int32_t dims[3], int64_t V,
                       int32_t rings, int64_t capacity, int32_t max_iter, double rmse_eps,
                       int32_t early_stop, double Rt_io[12], double* rmse_hist,
                       int64_t* fb_hist, int32_t* iters_done, int32_t* degenerate_hist,
                       int32_t* nn_idx, float* nn_d2)
{
    *iters_done = 0;
    if (m == 0) return VICPO_OK;
    if (m < 0 || max_iter < 0 || rings < 0) return VICPO_ERR_ARG;
    int rc = VICPO_OK;
    uint32_t* hist = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)V);
    uint32_t* off = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(V + 1));
    uint32_t* vm = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n + 2 * V));
    int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
    float* d2 = (float*)malloc(sizeof(float) * (size_t)m);
    if (!hist || !off || !vm || !idx || !d2) {
        rc = VICPO_ERR_OOM;
        goto done;
    }
    rc = vicpo_build(qx, qy, qz, n, origin, inv, dims, V, hist, off, vm);
    if (rc) goto done;
    rc = vicpo_dilate(dims, V, hist, off, rings, vm, NULL);
    if (rc) goto done;
    double prev_rmse = 0.0;
    for (int32_t k = 0; k < max_iter; ++k) {
        float Rtf[12];
        for (int a = 0; a < 12; ++a) Rtf[a] = (float)Rt_io[a];
        int64_t F = 0;
        vicpo_nns_cap(qx, qy, qz, n, origin, inv, dims, off, vm, px, py, pz, m, Rtf, capacity, idx, d2, &F, NULL,
                      NULL);
        double acc = 0.0;
        for (int64_t i = 0; i < m; ++i) acc += (double)d2[i];
        double rmse = sqrt(acc / (double)m);
        double next[12];
        int32_t deg = 0;
        vicpo_solve(px, py, pz, qx, qy, qz, idx, m, Rt_io, next, NULL, &deg);
        memcpy(Rt_io, next, sizeof next);
        if (rmse_hist) rmse_hist[k] = rmse;
        if (fb_hist) fb_hist[k] = F;
        if (degenerate_hist) degenerate_hist[k] = deg;
        *iters_done = k + 1;
        if (early_stop && k >= 1 && fabs(rmse - prev_rmse) < rmse_eps) break;
        prev_rmse = rmse;
    }
    if (nn_idx) memcpy(nn_idx, idx, sizeof(int32_t) * (size_t)m);
    if (nn_d2) memcpy(nn_d2, d2, sizeof(float) * (size_t)m);
done:
    free(hist);
    free(off);
    free(vm);
    free(idx);
    free(d2);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* differentiable point-to-point loss (float64)                              */
/* ------------------------------------------------------------------------ */

static void hat(const double w[3], double W[3][3])
{
    W[0][0] = 0;     W[0][1] = -w[2]; W[0][2] = w[1];
    W[1][0] = w[2];  W[1][1] = 0;     W[1][2] = -w[0];
    W[2][0] = -w[1]; W[2][1] = w[0];  W[2][2] = 0;
}

static void mm3(double A[3][3], double B[3][3], double C[3][3])
{
    double T[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += A[i][k] * B[k][j];
            T[i][j] = acc;
        }
    memcpy(C, T, sizeof T);
}

/* SE(3) exponential with xi = (rho, phi): R = Exp(phi) (Rodrigues),
 * t = J(phi) rho with J the SO(3) left Jacobian.  Also returns J and the
 * 6x6 SE(3) left Jacobian [[J, Qm], [0, J]] when asked. */
void vicpo_se3_exp(const double xi[6], double R[9], double t[3], double Jl6[36])
{
    const double* rho = xi;
    const double* phi = xi + 3;
    double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    double th = sqrt(th2);
    double A, B, C, c3, c4;
    if (th < 0.05) {
        double t4 = th2 * th2;
        A = 1.0 - th2 / 6.0 + t4 / 120.0;
        B = 0.5 - th2 / 24.0 + t4 / 720.0;
        C = 1.0 / 6.0 - th2 / 120.0 + t4 / 5040.0;
        c3 = 1.0 / 24.0 - th2 / 720.0 + t4 / 40320.0;
        c4 = 1.0 / 120.0 - th2 / 2520.0 + t4 / 120960.0;
    } else {
        double s = sin(th), c = cos(th);
        A = s / th;
        B = (1.0 - c) / th2;
        C = (th - s) / (th2 * th);
        c3 = (th2 + 2.0 * c - 2.0) / (2.0 * th2 * th2);
        c4 = (2.0 * th - 3.0 * s + th * c) / (2.0 * th2 * th2 * th);
    }
    double P[3][3], P2[3][3], J[3][3];
    hat(phi, P);
    mm3(P, P, P2);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double I = (i == j) ? 1.0 : 0.0;
            R[3 * i + j] = I + A * P[i][j] + B * P2[i][j];
            J[i][j] = I + B * P[i][j] + C * P2[i][j];
        }
    for (int i = 0; i < 3; ++i) t[i] = J[i][0] * rho[0] + J[i][1] * rho[1] + J[i][2] * rho[2];
    if (!Jl6) return;
    /* Q(rho, phi) of the SE(3) left Jacobian (Barfoot's closed form) */
    double Rh[3][3], Q[3][3];
    hat(rho, Rh);
    double PR[3][3], RP[3][3], PRP[3][3], PPR[3][3], RPP[3][3], PRPP[3][3], PPRP[3][3];
    mm3(P, Rh, PR);
    mm3(Rh, P, RP);
    mm3(PR, P, PRP);
    mm3(P, PR, PPR);
    mm3(RP, P, RPP);
    mm3(PRP, P, PRPP);
    mm3(P, PRP, PPRP);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            Q[i][j] = 0.5 * Rh[i][j] + C * (PR[i][j] + RP[i][j] + PRP[i][j]) +
                      c3 * (PPR[i][j] + RPP[i][j] - 3.0 * PRP[i][j]) +
                      c4 * (PRPP[i][j] + PPRP[i][j]);
    for (int i = 0; i < 36; ++i) Jl6[i] = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            Jl6[6 * i + j] = J[i][j];
            Jl6[6 * i + 3 + j] = Q[i][j];
            Jl6[6 * (i + 3) + 3 + j] = J[i][j];
        }
}

double vicpo_p2p_loss_fixed(const float* qx, const float* qy, const float* qz,
                            const double* px, const double* py, const double* pz, int64_t m,
                            const int32_t* idx, const double xi[6])
{
    double R[9], t[3];
    vicpo_se3_exp(xi, R, t, NULL);
    double acc = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        int64_t j = idx[i];
        double s[3];
        for (int a = 0; a < 3; ++a)
            s[a] = R[3 * a] * px[i] + R[3 * a + 1] * py[i] + R[3 * a + 2] * pz[i] + t[a];
        double r0 = s[0] - qx[j], r1 = s[1] - qy[j], r2 = s[2] - qz[j];
        acc += r0 * r0 + r1 * r1 + r2 * r2;
    }
    return m > 0 ? acc / (double)m : 0.0;
}

int vicpo_p2p(const float* qx, const float* qy, const float* qz, int64_t n,
              const float origin[3], float inv, const int32_t dims[3],
              const uint32_t* off, const uint32_t* vm,
              const float* px, const float* py, const float* pz, int64_t m,
              const double xi[6], double* loss, double* dpx, double* dpy, double* dpz,
              double dxi[6], int32_t* nn_idx)
{
    double R[9], t[3], Jl6[36];
    vicpo_se3_exp(xi, R, t, Jl6);
    float Rtf[12];
    for (int a = 0; a < 9; ++a) Rtf[a] = (float)R[a];
    for (int a = 0; a < 3; ++a) Rtf[9 + a] = (float)t[a];
    float* d2 = (float*)malloc(sizeof(float) * (size_t)(m > 0 ? m : 1));
    if (!d2) return VICPO_ERR_OOM;
    vicpo_nns(qx, qy, qz, n, origin, inv, dims, off, vm, px, py, pz, m, Rtf, nn_idx, d2, NULL, NULL, NULL);
    free(d2);
    double acc = 0.0, g[6] = {0, 0, 0, 0, 0, 0};
    double sc = m > 0 ? 2.0 / (double)m : 0.0;
    for (int64_t i = 0; i < m; ++i) {
        int64_t j = nn_idx[i];
        double p[3] = {px[i], py[i], pz[i]};
        double s[3], r[3];
        for (int a = 0; a < 3; ++a) s[a] = R[3 * a] * p[0] + R[3 * a + 1] * p[1] + R[3 * a + 2] * p[2] + t[a];
        r[0] = s[0] - qx[j];
        r[1] = s[1] - qy[j];
        r[2] = s[2] - qz[j];
        acc += r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        /* dL/dp = (2/m) R^T r */
        dpx[i] = sc * (R[0] * r[0] + R[3] * r[1] + R[6] * r[2]);
        dpy[i] = sc * (R[1] * r[0] + R[4] * r[1] + R[7] * r[2]);
        dpz[i] = sc * (R[2] * r[0] + R[5] * r[1] + R[8] * r[2]);
        /* left-perturbation gradient: translation part r, rotation part s x r */
        g[0] += r[0];
        g[1] += r[1];
        g[2] += r[2];
        g[3] += s[1] * r[2] - s[2] * r[1];
        g[4] += s[2] * r[0] - s[0] * r[2];
        g[5] += s[0] * r[1] - s[1] * r[0];
    }
    for (int a = 0; a < 6; ++a) g[a] *= sc;
    *loss = m > 0 ? acc / (double)m : 0.0;
    /* dL/dxi = Jl6^T g */
    for (int a = 0; a < 6; ++a) {
        double v = 0.0;
        for (int b = 0; b < 6; ++b) v += Jl6[6 * b + a] * g[b];
        dxi[a] = v;
    }
    return VICPO_OK;
}
