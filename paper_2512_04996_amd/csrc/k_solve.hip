// k_solve.hip -- the closed-form rigid transform of Eq. 1 per pair, in
// float64, and the ICP iteration bookkeeping (Sec. II.A; stop rule of
// Sec. IV.A).  One block per pair reduces the moment partials that the
// search blocks wrote, adds the queries resolved by the global search in
// index order (both in a fixed order), then one lane forms the cross-covariance
// H = sum (p - pbar)(q - qbar)^T = sum p q^T - m pbar qbar^T, takes its SVD
// H = U S V^T by one-sided Jacobi, and sets R = V diag(1, 1, det(V U^T)) U^T,
// t = qbar - R pbar; when det H is clearly positive the same R is taken as
// the orthogonal polar factor of H^T by a few Newton steps instead.  When the second singular value is below 1e-12 times the
// first, the rotation is not determined and the previous pose is kept.
#include <math.h>

#include "vicp_internal.hpp"

namespace vicp {

namespace {

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
// far from convergence).  X starts as A / ||A||_F (the polar factor does not
// change), so every quantity is of order one and the scale g, which only
// speeds convergence, is computed in float32.  Returns false when X becomes
// singular or the iteration does not settle; the caller then uses the SVD.
__host__ __device__ bool polar3(const double A[3][3], double Q[3][3])
{
    // float64 only and compared within tolerance: fused multiply-adds allowed
    // (the float32 search keeps every rounding as written)
#pragma clang fp contract(fast)
    double X[3][3];
    double na = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) na += A[i][j] * A[i][j];
    if (!(na > 0.0)) return false;
    const double inv = 1.0 / sqrt(na);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) X[i][j] = A[i][j] * inv;
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
        const double g = scale ? (double)sqrtf(sqrtf((float)nc) / ((float)det * sqrtf((float)nx))) : 1.0;
        const double a = 0.5 * g, b = 0.5 / (g * det);
        double diff = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                const double v = a * X[i][j] + b * C[i][j];
                diff += (v - X[i][j]) * (v - X[i][j]);
                X[i][j] = v;
            }
        if (diff < 1e-4) scale = false;
        // quadratic convergence: after a step of size below 1e-8 the new
        // iterate is within rounding of the polar factor
        if (diff < 1e-16) {
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) Q[i][j] = X[i][j];
            return true;
        }
    }
    return false;
}

// 1/x in the float64 solve.  On the device: the hardware reciprocal refined
// by two Newton steps, a chain of five operations instead of the ten or so
// of a correctly rounded division (the result is within an ulp or two; the
// solve is compared within tolerance).  On the host: a division.
__host__ __device__ __forceinline__ double recip(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    return fma(fma(-x, r, 1.0), r, r);
#else
    return 1.0 / x;
#endif
}

// Roughly 1/sqrt(x), for a scale factor whose exact value does not matter.
__host__ __device__ __forceinline__ double rough_rsqrt(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsq(x);
#else
    return 1.0 / sqrt(x);
#endif
}

// True when the rotation part of Q (row-major 3x3) is orthogonal to 1e-12.
__host__ __device__ bool rot_orthogonal(const double* Q)
{
    double orth = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) {
            const double d = Q[i] * Q[j] + Q[3 + i] * Q[3 + j] + Q[6 + i] * Q[6 + j] - (i == j ? 1.0 : 0.0);
            orth = fmax(orth, fabs(d));
        }
    return orth < 1e-12;
}

// Orthogonal polar factor of A refined from a nearby rotation Q0 (the
// previous pose's rotation, orthogonal): with M = R^T A, the rotation
// increment exp([w]x) that makes M symmetric solves (tr(S) I - S) w =
// 2 axial(skew M) to first order, S = sym(M); it is applied as the Cayley
// rotation of w (exactly orthogonal), and the step repeats until |w| < 1e-8
// (the error then is at rounding: the convergence is cubic, two steps from
// the previous pose of an ICP iteration).  A is scaled by any positive
// factor (the polar factor does not change) to keep the products of order
// one.  Accepted only if the final S is positive definite (so R is the polar
// factor, not another stationary point); otherwise returns false.
__host__ __device__ bool polar_refine(const double A[3][3], double scale, const double Q0[3][3], double Q[3][3])
{
    // float64 only and compared within tolerance: fused multiply-adds allowed
    // (the float32 search keeps every rounding as written)
#pragma clang fp contract(fast)
    double R[3][3], An[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            R[i][j] = Q0[i][j];
            An[i][j] = A[i][j] * scale;
        }
#pragma unroll 1
    for (int it = 0; it < 8; ++it) {
        double M[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) M[i][j] = R[0][i] * An[0][j] + R[1][i] * An[1][j] + R[2][i] * An[2][j];
        const double s00 = M[0][0], s11 = M[1][1], s22 = M[2][2];
        const double s01 = 0.5 * (M[0][1] + M[1][0]), s02 = 0.5 * (M[0][2] + M[2][0]), s12 = 0.5 * (M[1][2] + M[2][1]);
        const double k[3] = {M[2][1] - M[1][2], M[0][2] - M[2][0], M[1][0] - M[0][1]};   // 2 axial(skew M)
        // T = tr(S) I - S is symmetric: w = adj(T) k / det T
        const double t00 = s11 + s22, t11 = s00 + s22, t22 = s00 + s11;
        const double a00 = t11 * t22 - s12 * s12, a01 = s02 * s12 + s01 * t22, a02 = s01 * s12 + s02 * t11;
        const double a11 = t00 * t22 - s02 * s02, a12 = s01 * s02 + t00 * s12, a22 = t00 * t11 - s01 * s01;
        const double dT = t00 * a00 - s01 * a01 - s02 * a02;
        if (!(dT > 0.0)) return false;
        const double idT = recip(dT);
        const double w0 = (a00 * k[0] + a01 * k[1] + a02 * k[2]) * idT;
        const double w1 = (a01 * k[0] + a11 * k[1] + a12 * k[2]) * idT;
        const double w2 = (a02 * k[0] + a12 * k[1] + a22 * k[2]) * idT;
        const double ww = w0 * w0 + w1 * w1 + w2 * w2;
        // Cayley rotation of w with h = w / 2: I + f ([h]x + h h^T - |h|^2 I),
        // f = 2 / (1 + |h|^2)
        const double h0 = 0.5 * w0, h1 = 0.5 * w1, h2 = 0.5 * w2;
        const double f = 2.0 * recip(1.0 + 0.25 * ww);
        const double h01 = h0 * h1, h02 = h0 * h2, h12 = h1 * h2;
        const double D[3][3] = {{1.0 - f * (h1 * h1 + h2 * h2), f * (h01 - h2), f * (h02 + h1)},
                                {f * (h01 + h2), 1.0 - f * (h0 * h0 + h2 * h2), f * (h12 - h0)},
                                {f * (h02 - h1), f * (h12 + h0), 1.0 - f * (h0 * h0 + h1 * h1)}};
        double Rn[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Rn[i][j] = R[i][0] * D[0][j] + R[i][1] * D[1][j] + R[i][2] * D[2][j];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) R[i][j] = Rn[i][j];
        if (ww < 1e-16) {
            // S positive definite: its leading minors are positive
            const bool pd = s00 > 0.0 && s00 * s11 - s01 * s01 > 0.0 &&
                            s00 * (s11 * s22 - s12 * s12) - s01 * (s01 * s22 - s12 * s02) +
                                    s02 * (s01 * s12 - s11 * s02) > 0.0;
            if (!pd) return false;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) Q[i][j] = R[i][j];
            return true;
        }
    }
    return false;
}

// Moments about the centre c (sum p, sum q, sum p q^T, sum |p|^2, sum |q|^2,
// sum d, count); returns false (pose untouched)
// when H has rank < 2: its second singular value is below 1e-12 of the first
// or below the rounding floor of the one-pass sums, 1e-13 sqrt(sum|p|^2 sum|q|^2)
// (taken about c), so that a cross-covariance made of rounding noise (e.g.
// every correspondence on one target point) never yields a rotation.
// Rprev (row-major, may be null): the previous rotation, from which the polar
// factor is refined; prev_orth says it is known to be orthogonal (a previous
// solve's result), otherwise it is checked here.
__host__ __device__ bool kabsch(const double* mom, const double c[3], double Rt[12], const double* Rprev,
                                bool prev_orth)
{
    // float64 only and compared within tolerance: fused multiply-adds allowed
    // (the float32 search keeps every rounding as written)
#pragma clang fp contract(fast)
    const double m = mom[18];
    if (!(m > 0.0)) return false;
    double pb[3], qb[3], H[3][3];
    const double im = recip(m);
    for (int a = 0; a < 3; ++a) {
        pb[a] = mom[a] * im;
        qb[a] = mom[3 + a] * im;
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) H[a][b] = mom[6 + 3 * a + b] - m * pb[a] * qb[b];
    const double pq = mom[15] * mom[16];
    double R[3][3];
    // R = V U^T is the orthogonal polar factor of H^T (H^T = V S U^T =
    // (V U^T)(U S U^T)); when H is far above the rounding floor and det H is
    // clearly positive, no reflection fix is needed: the polar factor is
    // refined from the previous rotation, or else taken by the Newton polar
    // iteration.  The tests ||H|| > 1e6 floor and det H > 1e-6 ||H||^3 are
    // taken on squares (no square root on the way to the refinement).
    double Ht[3][3], nh = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            Ht[i][j] = H[j][i];
            nh += H[i][j] * H[i][j];
        }
    const double dH = det3(Ht);
    const bool well = nh > 1e-14 * pq && dH > 0.0 && dH * dH > 1e-12 * nh * nh * nh;
    bool fast = false;
    if (well && Rprev && (prev_orth || rot_orthogonal(Rprev))) {
        const double Q0[3][3] = {{Rprev[0], Rprev[1], Rprev[2]}, {Rprev[3], Rprev[4], Rprev[5]},
                                 {Rprev[6], Rprev[7], Rprev[8]}};
        fast = polar_refine(Ht, rough_rsqrt(nh), Q0, R);
    }
    if (well && !fast) fast = polar3(Ht, R);
    if (!fast) {
        const double floor_ = 1e-13 * sqrt(pq);
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
constexpr int kSolveThreads = 256;
constexpr int kSolveWaves = kSolveThreads / kWave;
constexpr int kFbWindow = 32 * kSolveThreads;   // queries per pass over the global-search list
constexpr int kUnitSlices = 12;                 // threads per fold-unit sum: (19 + 2) * 12 <= 256
constexpr int kUnitBatch = 16;                  // fold-unit loads in flight per thread
static_assert((kMoments + 2) * kUnitSlices <= kSolveThreads, "unit slices");

// Adds the moments of one correspondence (p, q about the centre c, squared
// distance d) to a[].
__device__ __forceinline__ void add_moments(double* a, float px, float py, float pz, float qx, float qy, float qz,
                                            float d, double c0, double c1, double c2)
{
    const double p[3] = {(double)px - c0, (double)py - c1, (double)pz - c2};
    const double q[3] = {(double)qx - c0, (double)qy - c1, (double)qz - c2};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        a[r] += p[r];
        a[3 + r] += q[r];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) a[6 + 3 * r + cc] += p[r] * q[cc];
    }
    a[15] += p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
    a[16] += q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
    a[17] += (double)d;
    a[18] += 1.0;
}

// One block per pair.  (1) The pair's fold units (moment-major, stride
// nunits) are summed per moment and counter by kUnitSlices threads each, in
// a fixed order.  (2) Queries resolved by the
// global search, when there are any: their list is in arbitrary order, so it
// is replayed in windows of kFbWindow source indices through an LDS bitmap;
// each thread adds the correspondences of its own 32 indices per window in
// index order, and a fixed-order block reduction adds them to (1).  (3) The
// solve of Eq. 1 and the iteration bookkeeping on one lane.
__global__ __launch_bounds__(kSolveThreads) void k_solve(
    const PairDev* __restrict__ pd, const int32_t* __restrict__ fold_begin, int32_t nunits,
    const double* __restrict__ fpart, const unsigned long long* __restrict__ fctr, PairState* __restrict__ st,
    int32_t* __restrict__ fb_count, const uint32_t* __restrict__ fb_list, const unsigned long long* __restrict__ fb_key,
    const float* __restrict__ px, const float* __restrict__ py, const float* __restrict__ pz,
    const float* __restrict__ qx, const float* __restrict__ qy, const float* __restrict__ qz,
    int32_t* __restrict__ flags, double* __restrict__ rmse_hist, int32_t* __restrict__ fb_hist,
    int32_t* __restrict__ deg_hist, unsigned long long* __restrict__ ctr_hist, int k, int K, int early_stop,
    double eps, int32_t* __restrict__ nn_idx, float* __restrict__ nn_d2)
{
    __shared__ double tot[kMoments];
    __shared__ unsigned long long ctot[2];
    __shared__ double usl[kMoments][kUnitSlices + 1];
    __shared__ unsigned long long ucsl[2][kUnitSlices + 1];
    __shared__ double red[kMoments][kSolveWaves];
    __shared__ uint32_t wbits[kFbWindow / 32];
    __shared__ uint32_t wslot[kFbWindow];
    const int pair = blockIdx.x;
    PairState& S = st[pair];
    const PairDev& P = pd[pair];
    const int done = S.done;
    // a single pair owns every fold unit: its range needs no table load
    const bool one = gridDim.x == 1;
    const int32_t u0 = one ? 0 : fold_begin[pair], u1 = one ? nunits : fold_begin[pair + 1];
    const int32_t nfb = fb_count[pair];
    const int32_t nmiss = fb_count[gridDim.x + pair];   // every global search, shell-resolved or listed
    const double prev = S.prev_rmse;
    // the current rotation, the start of the polar refinement: read by every
    // thread (uniform loads, all in flight together; a per-thread condition
    // made the compiler wait for each in turn), used by thread 0
    double Rp[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) Rp[j] = S.Rt[j];
    // the pair's fold units: kUnitSlices threads per sum each add an
    // interleaved slice of the units in order (kUnitBatch loads in flight,
    // added as a fixed tree), then one thread adds the slices in order
    if (threadIdx.x < (kMoments + 2) * kUnitSlices) {
        const int j = threadIdx.x / kUnitSlices, sl = threadIdx.x % kUnitSlices;
        if (j < kMoments) {
            const double* row = fpart + (int64_t)j * nunits;
            double sm = 0.0;
            for (int32_t u = u0 + sl; u < u1; u += kUnitSlices * kUnitBatch) {
                double v[kUnitBatch];
#pragma unroll
                for (int i = 0; i < kUnitBatch; ++i) {
                    const int32_t ui = u + i * kUnitSlices;
                    v[i] = ui < u1 ? row[ui] : 0.0;
                }
#pragma unroll
                for (int w = kUnitBatch / 2; w >= 1; w >>= 1)
#pragma unroll
                    for (int i = 0; i < w; ++i) v[i] += v[i + w];
                sm += v[0];
            }
            usl[j][sl] = sm;
        } else {
            const unsigned long long* row = fctr + (int64_t)(j - kMoments) * nunits;
            unsigned long long sm = 0;
            for (int32_t u = u0 + sl; u < u1; u += kUnitSlices * kUnitBatch) {
                unsigned long long v[kUnitBatch];
#pragma unroll
                for (int i = 0; i < kUnitBatch; ++i) {
                    const int32_t ui = u + i * kUnitSlices;
                    v[i] = ui < u1 ? row[ui] : 0ull;
                }
#pragma unroll
                for (int i = 0; i < kUnitBatch; ++i) sm += v[i];
            }
            ucsl[j - kMoments][sl] = sm;
        }
    }
    __syncthreads();
    if (threadIdx.x < kMoments) {
        double sm = usl[threadIdx.x][0];
#pragma unroll
        for (int e = 1; e < kUnitSlices; ++e) sm += usl[threadIdx.x][e];
        tot[threadIdx.x] = sm;
    } else if (threadIdx.x < kMoments + 2) {
        unsigned long long sm = 0;
#pragma unroll
        for (int e = 0; e < kUnitSlices; ++e) sm += ucsl[threadIdx.x - kMoments][e];
        ctot[threadIdx.x - kMoments] = sm;
    }
    // tested after the fold, whose loads do not depend on it, so that the
    // flag's latency overlaps theirs (a finished pair's fold units hold
    // stale sums that are never used)
    if (done) return;   // uniform over the block
    const double cen[3] = {P.cx, P.cy, P.cz};
    if (nfb > 0) {   // uniform over the block
        const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
        double acc[kMoments];
#pragma unroll
        for (int j = 0; j < kMoments; ++j) acc[j] = 0.0;
        for (int64_t w0 = 0; w0 < P.m; w0 += kFbWindow) {
            wbits[threadIdx.x] = 0u;
            __syncthreads();
            for (int32_t e = threadIdx.x; e < nfb; e += kSolveThreads) {
                const int64_t r = (int64_t)fb_list[P.p_base + e] - w0;
                if (r >= 0 && r < kFbWindow) {
                    atomicOr(&wbits[r >> 5], 1u << (r & 31));
                    wslot[r] = (uint32_t)e;
                }
            }
            __syncthreads();
            uint32_t bits = wbits[threadIdx.x];
            while (bits) {
                const int u = __ffs(bits) - 1;
                bits &= bits - 1u;
                const int r = 32 * (int)threadIdx.x + u;
                const unsigned long long key = fb_key[P.p_base + wslot[r]];
                const uint32_t j = (uint32_t)(key & 0xFFFFFFFFull);
                if (j >= (uint64_t)P.n) {   // unresolved global search (never expected)
                    atomicOr(&flags[pair], 2);
                    continue;
                }
                const int64_t gp = P.p_base + w0 + r, gq = P.q_base + j;
                const float d = __uint_as_float((uint32_t)(key >> 32));
                add_moments(acc, px[gp], py[gp], pz[gp], qx[gq], qy[gq], qz[gq], d, cen[0], cen[1], cen[2]);
                if (nn_idx) {   // the correspondences, when asked for
                    nn_idx[gp] = (int32_t)j;
                    nn_d2[gp] = d;
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < kMoments; ++j) {
            const double sm = wave_sum_f64(acc[j]);
            if (lane == 0) red[j][w] = sm;
        }
        __syncthreads();
        if (threadIdx.x < kMoments) {
            double sm = tot[threadIdx.x];
#pragma unroll
            for (int q = 0; q < kSolveWaves; ++q) sm += red[threadIdx.x][q];
            tot[threadIdx.x] = sm;
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double Rt[12];   // written by kabsch only when it succeeds
    const double m = tot[18];
    const double rmse = m > 0.0 ? sqrt(tot[17] / m) : 0.0;
    const bool ok = kabsch(tot, cen, Rt, Rp, S.rot_ok != 0);
    if (ok) {
        for (int j = 0; j < 12; ++j) {
            S.Rt[j] = Rt[j];
            S.Rtf[j] = (float)Rt[j];
        }
        S.rot_ok = 1;
    } else {
        S.degenerate += 1;
    }
    const int64_t h = (int64_t)pair * K + k;
    rmse_hist[h] = rmse;
    fb_hist[h] = nmiss;
    deg_hist[h] = ok ? 0 : 1;
    ctr_hist[2 * h] = ctot[0];
    ctr_hist[2 * h + 1] = ctot[1];
    fb_count[pair] = 0;
    fb_count[gridDim.x + pair] = 0;
    S.iters = k + 1;
    if (early_stop && k >= 1 && fabs(rmse - prev) < eps) S.done = 1;
    S.prev_rmse = rmse;
}

// Initial state: pose rounded to float32 for the search; pairs with no
// source points are done from the start; the global-search counts and the
// fault flags start at zero.
struct PoseBlob {
    double rt[12 * kInlinePairs];
};

__device__ __forceinline__ void set_state_one(const PairDev* __restrict__ pd, PairState* __restrict__ st, int p,
                                              const double* rt, int npairs, int32_t* __restrict__ fb_count,
                                              int32_t* __restrict__ flags)
{
    init_pair_state(st, p, rt, pd[p].m, npairs, fb_count, flags);
}

// The poses travel in the launch's arguments (up to kInlinePairs pairs).
__global__ void k_set_state_inline(const PairDev* __restrict__ pd, PairState* __restrict__ st, PoseBlob b,
                                   int npairs, int32_t* __restrict__ fb_count, int32_t* __restrict__ flags)
{
    const int p = threadIdx.x;
    if (p < npairs) set_state_one(pd, st, p, b.rt + 12 * p, npairs, fb_count, flags);
}

__global__ void k_set_state(const PairDev* __restrict__ pd, PairState* __restrict__ st, const double* __restrict__ rt64,
                            int npairs, int32_t* __restrict__ fb_count, int32_t* __restrict__ flags)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    set_state_one(pd, st, p, rt64 + 12 * p, npairs, fb_count, flags);
}

}  // namespace

void launch_solve(const PairDev* pd, int npairs, const int32_t* fold_begin, int32_t nunits, const double* fpart,
                  const unsigned long long* fctr, PairState* st, int32_t* fb_count, const uint32_t* fb_list,
                  const unsigned long long* fb_key, const float* px, const float* py, const float* pz,
                  const float* qx, const float* qy, const float* qz, int32_t* flags, double* rmse_hist,
                  int32_t* fb_hist, int32_t* deg_hist, unsigned long long* ctr_hist, int k, int K, int early_stop,
                  double eps, int32_t* nn_idx, float* nn_d2, hipStream_t s)
{
    if (npairs <= 0) return;
    launch_timed(k_solve, dim3(npairs), dim3(kSolveThreads), s, pd, fold_begin, nunits, fpart, fctr, st, fb_count,
                 fb_list, fb_key, px, py, pz, qx, qy, qz, flags, rmse_hist, fb_hist, deg_hist, ctr_hist, k, K,
                 early_stop, eps, nn_idx, nn_d2);
}

void launch_set_state_inline(const PairDev* pd, PairState* st, const double* host_rt, int npairs,
                             int32_t* fb_count, int32_t* flags, hipStream_t s)
{
    if (npairs <= 0 || npairs > kInlinePairs) return;
    PoseBlob b{};
    for (int i = 0; i < 12 * npairs; ++i) b.rt[i] = host_rt[i];
    hipLaunchKernelGGL(k_set_state_inline, dim3(1), dim3(64), 0, s, pd, st, b, npairs, fb_count, flags);
}

void launch_set_state(const PairDev* pd, PairState* st, const double* rt64, int npairs, int32_t* fb_count,
                      int32_t* flags, hipStream_t s)
{
    if (npairs <= 0) return;
    hipLaunchKernelGGL(k_set_state, dim3((npairs + 63) / 64), dim3(64), 0, s, pd, st, rt64, npairs, fb_count, flags);
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
