// k_solve.hip -- the closed-form rigid transform of Eq. 1 per pair, in
// float64, and the ICP iteration bookkeeping (Sec. II.A; stop rule of
// Sec. IV.A).  One block per pair reduces that pair's per-block moment
// partials in a fixed order, then one lane forms the cross-covariance
// H = sum (p - pbar)(q - qbar)^T = sum p q^T - m pbar qbar^T, takes its SVD
// H = U S V^T by one-sided Jacobi, and sets R = V diag(1, 1, det(V U^T)) U^T,
// t = qbar - R pbar; when det H is clearly positive the same R is taken as
// the orthogonal polar factor of H^T by a few Newton steps instead.  When the second singular value is below 1e-12 times the
// first, the rotation is not determined and the previous pose is kept.
#include <math.h>

#include "vicp_internal.hpp"

namespace vicp {

namespace {

constexpr int kThreads = 256;

__host__ __device__ void svd3(double A[3][3], double U[3][3], double sig[3], double V[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
    // one-sided Jacobi: rotate column pairs of A until they are orthogonal
    for (int sweep = 0; sweep < 16; ++sweep) {
        double worst = 0.0;
        for (int p = 0; p < 2; ++p) {
            for (int q = p + 1; q < 3; ++q) {
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int r = 0; r < 3; ++r) {
                    al += A[r][p] * A[r][p];
                    be += A[r][q] * A[r][q];
                    ga += A[r][p] * A[r][q];
                }
                if (ga == 0.0) continue;
                const double rel = fabs(ga) / sqrt(al * be);
                worst = fmax(worst, rel);
                if (!(rel > 1e-15)) continue;
                const double zeta = (be - al) / (2.0 * ga);
                const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                for (int r = 0; r < 3; ++r) {
                    const double ap = A[r][p], aq = A[r][q];
                    A[r][p] = c * ap - s * aq;
                    A[r][q] = s * ap + c * aq;
                    const double vp = V[r][p], vq = V[r][q];
                    V[r][p] = c * vp - s * vq;
                    V[r][q] = s * vp + c * vq;
                }
            }
        }
        if (!(worst > 1e-15)) break;
    }
    for (int j = 0; j < 3; ++j) {
        double nrm = 0.0;
        for (int r = 0; r < 3; ++r) nrm += A[r][j] * A[r][j];
        sig[j] = sqrt(nrm);
    }
    // order by decreasing singular value (columns of A and V move together)
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            if (sig[b] > sig[a]) {
                const double ts = sig[a];
                sig[a] = sig[b];
                sig[b] = ts;
                for (int r = 0; r < 3; ++r) {
                    double t = A[r][a];
                    A[r][a] = A[r][b];
                    A[r][b] = t;
                    t = V[r][a];
                    V[r][a] = V[r][b];
                    V[r][b] = t;
                }
            }
    for (int j = 0; j < 2; ++j)
        for (int r = 0; r < 3; ++r) U[r][j] = sig[j] > 0.0 ? A[r][j] / sig[j] : 0.0;
    if (sig[2] > 1e-13 * sig[0]) {
        for (int r = 0; r < 3; ++r) U[r][2] = A[r][2] / sig[2];
    } else {
        // complete the basis: the third left vector of a rank-2 H is free
        U[0][2] = U[1][0] * U[2][1] - U[2][0] * U[1][1];
        U[1][2] = U[2][0] * U[0][1] - U[0][0] * U[2][1];
        U[2][2] = U[0][0] * U[1][1] - U[1][0] * U[0][1];
    }
}

__host__ __device__ double det3(const double M[3][3])
{
    return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
           M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
}

// Orthogonal polar factor of a well-conditioned 3x3 matrix by the scaled
// Newton iteration X <- (g X + X^{-T} / g) / 2 (Frobenius-norm scaling while
// far from convergence).  Returns false when X becomes singular or the
// iteration does not settle; the caller then uses the SVD.
__host__ __device__ bool polar3(const double A[3][3], double Q[3][3])
{
    double X[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) X[i][j] = A[i][j];
    bool scale = true;
    for (int it = 0; it < 24; ++it) {
        double C[3][3];   // cofactors: X^{-T} = C / det
        C[0][0] = X[1][1] * X[2][2] - X[1][2] * X[2][1];
        C[0][1] = X[1][2] * X[2][0] - X[1][0] * X[2][2];
        C[0][2] = X[1][0] * X[2][1] - X[1][1] * X[2][0];
        C[1][0] = X[0][2] * X[2][1] - X[0][1] * X[2][2];
        C[1][1] = X[0][0] * X[2][2] - X[0][2] * X[2][0];
        C[1][2] = X[0][1] * X[2][0] - X[0][0] * X[2][1];
        C[2][0] = X[0][1] * X[1][2] - X[0][2] * X[1][1];
        C[2][1] = X[0][2] * X[1][0] - X[0][0] * X[1][2];
        C[2][2] = X[0][0] * X[1][1] - X[0][1] * X[1][0];
        const double det = X[0][0] * C[0][0] + X[0][1] * C[0][1] + X[0][2] * C[0][2];
        if (!(det > 0.0)) return false;
        double nx = 0.0, nc = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                nx += X[i][j] * X[i][j];
                nc += C[i][j] * C[i][j];
            }
        const double g = scale ? sqrt(sqrt(nc) / (det * sqrt(nx))) : 1.0;
        const double a = 0.5 * g, b = 0.5 / (g * det);
        double diff = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                const double v = a * X[i][j] + b * C[i][j];
                diff += (v - X[i][j]) * (v - X[i][j]);
                X[i][j] = v;
            }
        if (diff < 1e-4) scale = false;
        if (diff < 1e-24) {   // quadratic convergence: the step just taken is accurate to rounding
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) Q[i][j] = X[i][j];
            return true;
        }
    }
    return false;
}

// Moments about the centre c (see k_moments); returns false (pose untouched)
// when H has rank < 2: its second singular value is below 1e-12 of the first
// or below the rounding floor of the one-pass sums, 1e-13 sqrt(sum|p|^2 sum|q|^2)
// (taken about c), so that a cross-covariance made of rounding noise (e.g.
// every correspondence on one target point) never yields a rotation.
__host__ __device__ bool kabsch(const double* mom, const double c[3], double Rt[12])
{
    const double m = mom[18];
    if (!(m > 0.0)) return false;
    double pb[3], qb[3], H[3][3];
    for (int a = 0; a < 3; ++a) {
        pb[a] = mom[a] / m;
        qb[a] = mom[3 + a] / m;
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) H[a][b] = mom[6 + 3 * a + b] - m * pb[a] * qb[b];
    const double floor_ = 1e-13 * sqrt(mom[15] * mom[16]);
    double R[3][3];
    // R = V U^T is the orthogonal polar factor of H^T (H^T = V S U^T =
    // (V U^T)(U S U^T)); when H is far above the rounding floor and det H is
    // clearly positive, no reflection fix is needed and the Newton polar
    // iteration gives it directly
    double Ht[3][3], nh = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            Ht[i][j] = H[j][i];
            nh += H[i][j] * H[i][j];
        }
    const double fro = sqrt(nh);
    const bool fast = fro > 1e6 * floor_ && det3(Ht) > 1e-6 * nh * fro && polar3(Ht, R);
    if (!fast) {
        double U[3][3], sig[3], V[3][3];
        svd3(H, U, sig, V);
        if (!(sig[0] > 0.0) || sig[1] <= 1e-12 * sig[0] || sig[1] <= floor_) return false;
        const double d = (det3(U) * det3(V) < 0.0) ? -1.0 : 1.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) R[i][j] = V[i][0] * U[j][0] + V[i][1] * U[j][1] + d * V[i][2] * U[j][2];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Rt[3 * i + j] = R[i][j];
    // t = qbar - R pbar with the means taken back from c
    for (int i = 0; i < 3; ++i) {
        const double rp = R[i][0] * (pb[0] + c[0]) + R[i][1] * (pb[1] + c[1]) + R[i][2] * (pb[2] + c[2]);
        Rt[9 + i] = (qb[i] + c[i]) - rp;
    }
    return true;
}

constexpr int kWave = 64;
constexpr int kMomItems = 4;   // correspondences per lane

__device__ __forceinline__ double wave_sum(double v) { return wave_sum_f64(v); }

// Moments of the correspondences in float64 (sum p, sum q, sum p q^T,
// sum d, count): each lane adds kMomItems correspondences in a fixed order,
// the block reduces in a fixed order and writes one partial.
__global__ __launch_bounds__(kThreads) void k_moments(
    const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
    const float* __restrict__ px, const float* __restrict__ py, const float* __restrict__ pz,
    const float* __restrict__ qx, const float* __restrict__ qy, const float* __restrict__ qz,
    const PairState* __restrict__ st, const unsigned long long* __restrict__ fb_key, int32_t* __restrict__ nn_idx,
    float* __restrict__ nn_d2, double* __restrict__ part, int32_t* __restrict__ flags,
    const int32_t* __restrict__ mom_begin, const int32_t* __restrict__ nns_begin,
    const unsigned long long* __restrict__ ctr, unsigned long long* __restrict__ ctr_part)
{
    __shared__ double red[kMoments][kThreads / kWave];
    __shared__ unsigned long long cred[2][kThreads / kWave];
    const BlockJob job = jobs[blockIdx.x];
    const int pair = job.pair;
    const PairDev& P = pd[pair];
    const PairState& S = st[pair];
    if (S.done) return;   // uniform over the block
    // this block's share of the pair's search-block counters: the blocks of
    // the search split evenly over the pair's moment blocks
    const int32_t mb0 = mom_begin[pair], nmb = mom_begin[pair + 1] - mb0;
    const int32_t nb0 = nns_begin[pair], nbn = nns_begin[pair + 1] - nb0;
    const int32_t chunk = (nbn + nmb - 1) / nmb, r = (int32_t)blockIdx.x - mb0;
    const int32_t c0 = nb0 + min(nbn, r * chunk), c1 = nb0 + min(nbn, (r + 1) * chunk);
    unsigned long long k0 = 0, k1 = 0;
    for (int32_t b = c0 + (int32_t)threadIdx.x; b < c1; b += kThreads) {
        k0 += ctr[2 * (int64_t)b];
        k1 += ctr[2 * (int64_t)b + 1];
    }
    double a[kMoments];
#pragma unroll
    for (int j = 0; j < kMoments; ++j) a[j] = 0.0;
    // every load of the lane's correspondences is issued before any is used;
    // lanes past the end read the pair's first point and add nothing
    int32_t jj[kMomItems];
    float dd[kMomItems];
    bool ok_[kMomItems];
    int64_t gp[kMomItems];
#pragma unroll
    for (int it = 0; it < kMomItems; ++it) {
        const int64_t i = (int64_t)job.start + threadIdx.x + it * kThreads;
        ok_[it] = i < P.m;
        gp[it] = P.p_base + (ok_[it] ? i : 0);
        jj[it] = nn_idx[gp[it]];
        dd[it] = nn_d2[gp[it]];
    }
#pragma unroll
    for (int it = 0; it < kMomItems; ++it) {
        if (ok_[it] && jj[it] < 0) {
            const unsigned long long key = fb_key[P.p_base + (-1 - jj[it])];
            jj[it] = (int32_t)(uint32_t)(key & 0xFFFFFFFFull);
            dd[it] = __uint_as_float((uint32_t)(key >> 32));
            nn_idx[gp[it]] = jj[it];
            nn_d2[gp[it]] = dd[it];
        }
        if ((uint32_t)jj[it] >= (uint64_t)P.n) {   // unresolved global search (never expected)
            if (ok_[it]) atomicOr(&flags[pair], 2);
            jj[it] = 0;
        }
    }
    float pv[kMomItems][3], qv[kMomItems][3];
#pragma unroll
    for (int it = 0; it < kMomItems; ++it) {
        const int64_t gq = P.q_base + jj[it];
        pv[it][0] = px[gp[it]];
        pv[it][1] = py[gp[it]];
        pv[it][2] = pz[gp[it]];
        qv[it][0] = qx[gq];
        qv[it][1] = qy[gq];
        qv[it][2] = qz[gq];
    }
#pragma unroll
    for (int it = 0; it < kMomItems; ++it) {
        // a select, not a product: a lane past the end adds exact zeros even
        // if what it read is not finite
        const bool o = ok_[it];
        const double c0 = P.cx, c1 = P.cy, c2 = P.cz;
        const double p[3] = {o ? (double)pv[it][0] - c0 : 0.0, o ? (double)pv[it][1] - c1 : 0.0,
                             o ? (double)pv[it][2] - c2 : 0.0};
        const double q[3] = {o ? (double)qv[it][0] - c0 : 0.0, o ? (double)qv[it][1] - c1 : 0.0,
                             o ? (double)qv[it][2] - c2 : 0.0};
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            a[r] += p[r];
            a[3 + r] += q[r];
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) a[6 + 3 * r + cc] += p[r] * q[cc];
        }
        a[15] += p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
        a[16] += q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
        a[17] += o ? (double)dd[it] : 0.0;
        a[18] += o ? 1.0 : 0.0;
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < kMoments; ++j) {
        const double sm = wave_sum(a[j]);
        if (lane == 0) red[j][w] = sm;
    }
    for (int d = kWave / 2; d > 0; d >>= 1) {
        k0 += __shfl_xor(k0, d, kWave);
        k1 += __shfl_xor(k1, d, kWave);
    }
    if (lane == 0) {
        cred[0][w] = k0;
        cred[1][w] = k1;
    }
    __syncthreads();
    if (threadIdx.x < kMoments) {
        double sm = red[threadIdx.x][0];
#pragma unroll
        for (int q = 1; q < kThreads / kWave; ++q) sm += red[threadIdx.x][q];
        part[(int64_t)blockIdx.x * kMoments + threadIdx.x] = sm;
    } else if (threadIdx.x < kMoments + 2) {
        const int c = threadIdx.x - kMoments;
        unsigned long long sm = cred[c][0];
#pragma unroll
        for (int q = 1; q < kThreads / kWave; ++q) sm += cred[c][q];
        ctr_part[2 * (int64_t)blockIdx.x + c] = sm;
    }
}

// One block per pair: the pair's moment and counter partials in block order
// (fixed, so the result does not depend on scheduling), then the solve of
// Eq. 1 and the iteration bookkeeping on one lane.  Everything the block
// reads is requested before the first use, so the loads overlap.
__global__ __launch_bounds__(kThreads) void k_solve(
    const PairDev* __restrict__ pd, const int32_t* __restrict__ job_begin, const double* __restrict__ part,
    const unsigned long long* __restrict__ ctr_part, PairState* __restrict__ st, int32_t* __restrict__ fb_count,
    double* __restrict__ rmse_hist, int32_t* __restrict__ fb_hist, int32_t* __restrict__ deg_hist,
    unsigned long long* __restrict__ ctr_hist, int k, int K, int early_stop, double eps)
{
    __shared__ double red[kMoments][kThreads / kWave];
    __shared__ double tot[kMoments];
    __shared__ unsigned long long cred[2][kThreads / kWave];
    const int pair = blockIdx.x;
    PairState& S = st[pair];
    const int done = S.done;
    const int32_t b0 = job_begin[pair], b1 = job_begin[pair + 1];
    double Rt[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) Rt[j] = S.Rt[j];
    const double cen[3] = {pd[pair].cx, pd[pair].cy, pd[pair].cz};
    const int32_t nfb = fb_count[pair];
    const double prev = S.prev_rmse;
    if (done) return;   // uniform over the block
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double acc[kMoments];
#pragma unroll
    for (int j = 0; j < kMoments; ++j) acc[j] = 0.0;
    unsigned long long c0 = 0, c1 = 0;
    for (int32_t b = b0 + threadIdx.x; b < b1; b += kThreads) {
#pragma unroll
        for (int j = 0; j < kMoments; ++j) acc[j] += part[(int64_t)b * kMoments + j];
        c0 += ctr_part[2 * (int64_t)b];
        c1 += ctr_part[2 * (int64_t)b + 1];
    }
#pragma unroll
    for (int j = 0; j < kMoments; ++j) {
        const double sm = wave_sum(acc[j]);
        if (lane == 0) red[j][w] = sm;
    }
    for (int d = kWave / 2; d > 0; d >>= 1) {
        c0 += __shfl_xor(c0, d, kWave);
        c1 += __shfl_xor(c1, d, kWave);
    }
    if (lane == 0) {
        cred[0][w] = c0;
        cred[1][w] = c1;
    }
    __syncthreads();
    if (threadIdx.x < kMoments) {
        double sm = red[threadIdx.x][0];
#pragma unroll
        for (int q = 1; q < kThreads / kWave; ++q) sm += red[threadIdx.x][q];
        tot[threadIdx.x] = sm;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int q = 1; q < kThreads / kWave; ++q) {
        cred[0][0] += cred[0][q];
        cred[1][0] += cred[1][q];
    }
    const double m = tot[18];
    const double rmse = m > 0.0 ? sqrt(tot[17] / m) : 0.0;
    const bool ok = kabsch(tot, cen, Rt);
    if (ok) {
        for (int j = 0; j < 12; ++j) {
            S.Rt[j] = Rt[j];
            S.Rtf[j] = (float)Rt[j];
        }
    } else {
        S.degenerate += 1;
    }
    const int64_t h = (int64_t)pair * K + k;
    rmse_hist[h] = rmse;
    fb_hist[h] = nfb;
    deg_hist[h] = ok ? 0 : 1;
    ctr_hist[2 * h] = cred[0][0];
    ctr_hist[2 * h + 1] = cred[1][0];
    fb_count[pair] = 0;
    S.iters = k + 1;
    if (early_stop && k >= 1 && fabs(rmse - prev) < eps) S.done = 1;
    S.prev_rmse = rmse;
}

// Initial state: pose rounded to float32 for the search; pairs with no
// source points are done from the start.
__global__ void k_set_state(const PairDev* __restrict__ pd, PairState* __restrict__ st, const double* __restrict__ rt64,
                            int npairs)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    PairState& S = st[p];
    S.done = pd[p].m > 0 ? 0 : 1;
    for (int j = 0; j < 12; ++j) {
        S.Rt[j] = rt64[12 * p + j];
        S.Rtf[j] = (float)rt64[12 * p + j];
    }
    S.prev_rmse = 0.0;
    S.iters = 0;
    S.degenerate = 0;
    S.status = 0;
}

}  // namespace

void launch_moments(const PairDev* pd, const BlockJob* jobs, int njobs, const float* px, const float* py,
                    const float* pz, const float* qx, const float* qy, const float* qz, const PairState* st,
                    const unsigned long long* fb_key, int32_t* nn_idx, float* nn_d2, double* part, int32_t* flags,
                    const int32_t* mom_begin, const int32_t* nns_begin, const unsigned long long* ctr,
                    unsigned long long* ctr_part, hipStream_t s)
{
    if (njobs <= 0) return;
    hipLaunchKernelGGL(k_moments, dim3(njobs), dim3(kThreads), 0, s, pd, jobs, px, py, pz, qx, qy, qz, st, fb_key,
                       nn_idx, nn_d2, part, flags, mom_begin, nns_begin, ctr, ctr_part);
}

void launch_solve(const PairDev* pd, int npairs, const int32_t* job_begin, const double* part,
                  const unsigned long long* ctr_part, PairState* st, int32_t* fb_count, double* rmse_hist,
                  int32_t* fb_hist, int32_t* deg_hist, unsigned long long* ctr_hist, int k, int K, int early_stop,
                  double eps, hipStream_t s)
{
    if (npairs <= 0) return;
    hipLaunchKernelGGL(k_solve, dim3(npairs), dim3(kThreads), 0, s, pd, job_begin, part, ctr_part, st, fb_count,
                       rmse_hist, fb_hist, deg_hist, ctr_hist, k, K, early_stop, eps);
}

int moments_items_per_block() { return kThreads * kMomItems; }

void launch_set_state(const PairDev* pd, PairState* st, const double* rt64, int npairs, hipStream_t s)
{
    if (npairs <= 0) return;
    hipLaunchKernelGGL(k_set_state, dim3((npairs + 63) / 64), dim3(64), 0, s, pd, st, rt64, npairs);
}

// Flags pairs whose source holds NaN or Inf (bit 0 of PairState::status).
__global__ void k_check_finite(const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                               const float* __restrict__ px, const float* __restrict__ py,
                               const float* __restrict__ pz, int32_t* __restrict__ flags)
{
    const BlockJob job = jobs[blockIdx.x];
    const PairDev& P = pd[job.pair];
    const int64_t i = (int64_t)job.start + threadIdx.x;
    if (i >= P.m) return;
    const int64_t g = P.p_base + i;
    if (!(isfinite(px[g]) && isfinite(py[g]) && isfinite(pz[g]))) atomicOr(&flags[job.pair], 1);
}

void launch_check_finite(const PairDev* pd, const BlockJob* jobs, int njobs, const float* px, const float* py,
                         const float* pz, int32_t* flags, hipStream_t s)
{
    if (njobs <= 0) return;
    hipLaunchKernelGGL(k_check_finite, dim3(njobs), dim3(256), 0, s, pd, jobs, px, py, pz, flags);
}

}  // namespace vicp
