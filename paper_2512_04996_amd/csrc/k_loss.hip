// k_loss.hip -- differentiable point-to-point loss on the dilation NNS.
//
// Pose xi = (rho, phi) in R^6 per pair; T(xi) = Exp(xi) in SE(3) with
// R = Exp(phi) (Rodrigues) and t = J(phi) rho, J the SO(3) left Jacobian.
// The correspondences c_i come from the local/global search at T rounded to
// float32 (the same kernels as registration) and are held fixed; the loss
// L_b = (1/m) sum_i |R p_i + t - q_c(i)|^2 and its gradients are evaluated in
// float64 (full-rate on this GPU):
//   dL/dp_i  = (2/m) R^T r_i
//   dL/dxi   = JJ(xi)^T [ (2/m) sum r_i ; (2/m) sum s_i x r_i ]
// where s_i = T p_i, r_i = s_i - q_c(i), and JJ is the 6x6 SE(3) left
// Jacobian [[J, Qm], [0, J]]: the two sums are the gradient for a left
// perturbation Exp(d) T(xi), and Exp(xi + e) = Exp(JJ e) Exp(xi) to first order.
#include <math.h>

#include "vicp_internal.hpp"

namespace vicp {

namespace {

constexpr int kWave = 64;

__device__ void skew(const double w[3], double W[3][3])
{
    W[0][0] = 0.0;
    W[0][1] = -w[2];
    W[0][2] = w[1];
    W[1][0] = w[2];
    W[1][1] = 0.0;
    W[1][2] = -w[0];
    W[2][0] = -w[1];
    W[2][1] = w[0];
    W[2][2] = 0.0;
}

__device__ void matmul3(const double A[3][3], const double B[3][3], double C[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[i][j] = A[i][0] * B[0][j] + A[i][1] * B[1][j] + A[i][2] * B[2][j];
}

// One lane per pair: the pose, its float32 rounding and the 6x6 Jacobian.
__global__ void k_se3(const double* __restrict__ xi, int npairs, PairState* __restrict__ st, double* __restrict__ jl6,
                      int32_t* __restrict__ fb_count, int32_t* __restrict__ flags)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    // the pass's global-search list length, global-search count and fault
    // flags start at zero
    fb_count[p] = 0;
    fb_count[npairs + p] = 0;
    flags[p] = 0;
    const double rho[3] = {xi[6 * p + 0], xi[6 * p + 1], xi[6 * p + 2]};
    const double phi[3] = {xi[6 * p + 3], xi[6 * p + 4], xi[6 * p + 5]};
    const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    const double th = sqrt(th2);
    // a = sin/th, b = (1-cos)/th^2, c = (th-sin)/th^3,
    // e = (th^2 + 2cos - 2)/(2 th^4), f = (2 th - 3 sin + th cos)/(2 th^5)
    double a, b, c, e, f;
    if (th < 0.05) {
        const double t4 = th2 * th2;
        a = 1.0 - th2 / 6.0 + t4 / 120.0;
        b = 0.5 - th2 / 24.0 + t4 / 720.0;
        c = 1.0 / 6.0 - th2 / 120.0 + t4 / 5040.0;
        e = 1.0 / 24.0 - th2 / 720.0 + t4 / 40320.0;
        f = 1.0 / 120.0 - th2 / 2520.0 + t4 / 120960.0;
    } else {
        double sn, cs;
        sincos(th, &sn, &cs);
        a = sn / th;
        b = (1.0 - cs) / th2;
        c = (th - sn) / (th2 * th);
        e = (th2 + 2.0 * cs - 2.0) / (2.0 * th2 * th2);
        f = (2.0 * th - 3.0 * sn + th * cs) / (2.0 * th2 * th2 * th);
    }
    double F[3][3], F2[3][3], J[3][3], R[3][3];
    skew(phi, F);
    matmul3(F, F, F2);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double id = (i == j) ? 1.0 : 0.0;
            R[i][j] = id + a * F[i][j] + b * F2[i][j];
            J[i][j] = id + b * F[i][j] + c * F2[i][j];
        }
    PairState& S = st[p];
    for (int i = 0; i < 3; ++i) {
        const double t = J[i][0] * rho[0] + J[i][1] * rho[1] + J[i][2] * rho[2];
        for (int j = 0; j < 3; ++j) {
            S.Rt[3 * i + j] = R[i][j];
            S.Rtf[3 * i + j] = (float)R[i][j];
        }
        S.Rt[9 + i] = t;
        S.Rtf[9 + i] = (float)t;
    }
    S.done = 0;
    S.rot_ok = 0;
    // Qm = 1/2 P + c (F P + P F + F P F) + e (F F P + P F F - 3 F P F) + f (F P F F + F F P F)
    double Pm[3][3], FP[3][3], PF[3][3], FPF[3][3], FFP[3][3], PFF[3][3], FPFF[3][3], FFPF[3][3];
    skew(rho, Pm);
    matmul3(F, Pm, FP);
    matmul3(Pm, F, PF);
    matmul3(FP, F, FPF);
    matmul3(F, FP, FFP);
    matmul3(PF, F, PFF);
    matmul3(FPF, F, FPFF);
    matmul3(F, FPF, FFPF);
    double* Jo = jl6 + 36 * p;
    for (int i = 0; i < 36; ++i) Jo[i] = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double Qm = 0.5 * Pm[i][j] + c * (FP[i][j] + PF[i][j] + FPF[i][j]) +
                              e * (FFP[i][j] + PFF[i][j] - 3.0 * FPF[i][j]) + f * (FPFF[i][j] + FFPF[i][j]);
            Jo[6 * i + j] = J[i][j];
            Jo[6 * i + 3 + j] = Qm;
            Jo[6 * (i + 3) + 3 + j] = J[i][j];
        }
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Per query: resolve the correspondence, residual in float64; forward keeps
// sum |r|^2 and the count, backward (gloss != null) also writes dL/dp and
// keeps sum r and sum s x r.  One partial of kGradTerms per block.
__global__ __launch_bounds__(256) void k_loss_terms(const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                                                    const float* __restrict__ px, const float* __restrict__ py,
                                                    const float* __restrict__ pz, const float* __restrict__ qx,
                                                    const float* __restrict__ qy, const float* __restrict__ qz,
                                                    const PairState* __restrict__ st,
                                                    const unsigned long long* __restrict__ fb_key,
                                                    int32_t* __restrict__ nn_idx, const double* __restrict__ gloss,
                                                    float* __restrict__ dpx, float* __restrict__ dpy,
                                                    float* __restrict__ dpz, double* __restrict__ part,
                                                    int32_t* __restrict__ flags)
{
    __shared__ double red[kGradTerms][256 / kWave];
    const BlockJob job = jobs[blockIdx.x];
    const PairDev& P = pd[job.pair];
    const PairState& S = st[job.pair];
    double a[kGradTerms];
#pragma unroll
    for (int k = 0; k < kGradTerms; ++k) a[k] = 0.0;
    const int64_t i = (int64_t)job.start + threadIdx.x;
    if (i < P.m) {
        const int64_t gp = P.p_base + i;
        int32_t j = nn_idx[gp];
        if (j < 0) {
            j = (int32_t)(uint32_t)(fb_key[P.p_base + (-1 - j)] & 0xFFFFFFFFull);
            nn_idx[gp] = j;
        }
        if ((uint32_t)j >= (uint64_t)P.n) {   // unresolved global search (never expected): flag, do not read
            atomicOr(&flags[job.pair], 2);
            j = 0;
        }
        const int64_t gq = P.q_base + j;
        const double x = px[gp], y = py[gp], z = pz[gp];
        const double* R = S.Rt;
        double s[3], r[3];
        s[0] = fma(R[0], x, fma(R[1], y, fma(R[2], z, R[9])));
        s[1] = fma(R[3], x, fma(R[4], y, fma(R[5], z, R[10])));
        s[2] = fma(R[6], x, fma(R[7], y, fma(R[8], z, R[11])));
        r[0] = s[0] - (double)qx[gq];
        r[1] = s[1] - (double)qy[gq];
        r[2] = s[2] - (double)qz[gq];
        a[6] = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        a[7] = 1.0;
        if (gloss) {
            const double sc = 2.0 * gloss[job.pair] / (double)P.m;
            dpx[gp] = (float)(sc * (R[0] * r[0] + R[3] * r[1] + R[6] * r[2]));
            dpy[gp] = (float)(sc * (R[1] * r[0] + R[4] * r[1] + R[7] * r[2]));
            dpz[gp] = (float)(sc * (R[2] * r[0] + R[5] * r[1] + R[8] * r[2]));
            a[0] = r[0];
            a[1] = r[1];
            a[2] = r[2];
            a[3] = s[1] * r[2] - s[2] * r[1];
            a[4] = s[2] * r[0] - s[0] * r[2];
            a[5] = s[0] * r[1] - s[1] * r[0];
        }
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < kGradTerms; ++k) {
        const double sm = wave_sum(a[k]);
        if (lane == 0) red[k][w] = sm;
    }
    __syncthreads();
    if (threadIdx.x < kGradTerms) {
        double sm = red[threadIdx.x][0];
#pragma unroll
        for (int k = 1; k < 256 / kWave; ++k) sm += red[threadIdx.x][k];
        part[(int64_t)blockIdx.x * kGradTerms + threadIdx.x] = sm;
    }
}

// One block per pair: fixed-order reduction of the pair's partials, then
// the loss (forward) or dL/dxi (backward).
__global__ __launch_bounds__(256) void k_loss_finish(const PairDev* __restrict__ pd, const int32_t* __restrict__ job_begin,
                                                     const double* __restrict__ part, const double* __restrict__ jl6,
                                                     const double* __restrict__ gloss, double* __restrict__ loss,
                                                     double* __restrict__ dxi)
{
    __shared__ double red[kGradTerms][256];
    const int pair = blockIdx.x;
    const int32_t b0 = job_begin[pair], b1 = job_begin[pair + 1];
    double acc[kGradTerms];
#pragma unroll
    for (int j = 0; j < kGradTerms; ++j) acc[j] = 0.0;
    for (int32_t b = b0 + threadIdx.x; b < b1; b += 256) {
#pragma unroll
        for (int j = 0; j < kGradTerms; ++j) acc[j] += part[(int64_t)b * kGradTerms + j];
    }
#pragma unroll
    for (int j = 0; j < kGradTerms; ++j) red[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
#pragma unroll
            for (int j = 0; j < kGradTerms; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double m = (double)pd[pair].m;
    if (!gloss) {
        if (loss) loss[pair] = m > 0.0 ? red[6][0] / m : 0.0;
        return;
    }
    const double sc = m > 0.0 ? 2.0 * gloss[pair] / m : 0.0;
    double g[6];
    for (int k = 0; k < 6; ++k) g[k] = sc * red[k][0];
    const double* Jo = jl6 + 36 * pair;
    for (int a = 0; a < 6; ++a) {
        double v = 0.0;
        for (int b = 0; b < 6; ++b) v += Jo[6 * b + a] * g[b];
        dxi[6 * pair + a] = v;
    }
}

}  // namespace

void launch_se3(const double* xi, int npairs, PairState* st, double* jl6, int32_t* fb_count, int32_t* flags,
                hipStream_t s)
{
    if (npairs <= 0) return;
    hipLaunchKernelGGL(k_se3, dim3((npairs + 63) / 64), dim3(64), 0, s, xi, npairs, st, jl6, fb_count, flags);
}

void launch_loss_terms(const PairDev* pd, const BlockJob* jobs, int njobs, const float* px, const float* py,
                       const float* pz, const float* qx, const float* qy, const float* qz, const PairState* st,
                       const unsigned long long* fb_key, int32_t* nn_idx, const double* gloss, float* dpx, float* dpy,
                       float* dpz, double* part, int32_t* flags, hipStream_t s)
{
    if (njobs <= 0) return;
    hipLaunchKernelGGL(k_loss_terms, dim3(njobs), dim3(256), 0, s, pd, jobs, px, py, pz, qx, qy, qz, st, fb_key, nn_idx,
                       gloss, dpx, dpy, dpz, part, flags);
}

void launch_loss_finish(const PairDev* pd, int npairs, const int32_t* job_begin, const double* part, const double* jl6,
                        const double* gloss, double* loss, double* dxi, hipStream_t s)
{
    if (npairs <= 0) return;
    hipLaunchKernelGGL(k_loss_finish, dim3(npairs), dim3(256), 0, s, pd, job_begin, part, jl6, gloss, loss, dxi);
}

}  // namespace vicp
