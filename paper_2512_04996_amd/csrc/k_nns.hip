// k_nns.hip -- correspondence search (Alg. 4) and the moments of Eq. 1.
//
// Local search: one lane per source point.  The transformed point's voxel is
// found by the same float32 quantisation as the targets; its count word is
// read through the offsets; a Mask(root) word redirects to the root voxel's
// segment (indirect addressing, no replicated points).  Candidates are read
// as float4 (x, y, z, index) from the segment-ordered copy of the target, one
// coalesced 16-byte load each; segments are in ascending index order, so a
// strict "<" keeps the lowest index among equal distances.
//
// Global search (empty undilated voxel or outside the grid): the query is
// appended to a per-pair list and an exact brute force over all targets
// resolves it; partial minima from target tiles merge through a 64-bit
// atomic minimum of (distance bits << 32 | index), which is order-free, so
// the result is deterministic.
#include <math.h>

#include "vicp_internal.hpp"

namespace vicp {

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ void transform(const float* __restrict__ R, float x, float y, float z, float& sx, float& sy,
                                          float& sz)
{
    sx = __builtin_fmaf(R[0], x, __builtin_fmaf(R[1], y, __builtin_fmaf(R[2], z, R[9])));
    sy = __builtin_fmaf(R[3], x, __builtin_fmaf(R[4], y, __builtin_fmaf(R[5], z, R[10])));
    sz = __builtin_fmaf(R[6], x, __builtin_fmaf(R[7], y, __builtin_fmaf(R[8], z, R[11])));
}

__device__ __forceinline__ float dist2(float sx, float sy, float sz, float qx, float qy, float qz)
{
    const float dx = sx - qx, dy = sy - qy, dz = sz - qz;
    return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

template <int BS>
__global__ __launch_bounds__(BS) void k_nns_local(const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                                                  const float* __restrict__ px, const float* __restrict__ py,
                                                  const float* __restrict__ pz, const PairState* __restrict__ st,
                                                  const uint32_t* __restrict__ off, const uint32_t* __restrict__ vm,
                                                  const float4* __restrict__ qs4, int32_t* __restrict__ nn_idx,
                                                  float* __restrict__ nn_d2, int32_t* __restrict__ fb_count,
                                                  uint32_t* __restrict__ fb_list, unsigned long long* __restrict__ fb_key,
                                                  unsigned long long* __restrict__ ctr)
{
    const BlockJob job = jobs[blockIdx.x];
    const PairDev& P = pd[job.pair];
    const PairState& S = st[job.pair];
    if (S.done) return;   // uniform over the block
    const int64_t i = (int64_t)job.start + threadIdx.x;
    const bool active = i < P.m;
    const int64_t gp = P.p_base + i;
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    uint32_t c = 0;
    int64_t cs = 0;
    bool dil = false;
    if (active) {
        transform(S.Rtf, px[gp], py[gp], pz[gp], sx, sy, sz);
        const float fx = (sx - P.ox) * P.inv;
        const float fy = (sy - P.oy) * P.inv;
        const float fz = (sz - P.oz) * P.inv;
        const bool in = (fx >= 0.0f) && (fx < P.fDx) && (fy >= 0.0f) && (fy < P.fDy) && (fz >= 0.0f) && (fz < P.fDz);
        if (in) {
            const uint32_t v =
                (uint32_t)floorf(fx) + (uint32_t)P.Dx * ((uint32_t)floorf(fy) + (uint32_t)P.Dy * (uint32_t)floorf(fz));
            const int64_t g = P.v_base + v;
            const uint32_t og = off[g];
            const uint32_t h = vm[(int64_t)og + 1];
            if (h & kMask) {
                // dilated: follow Mask(root) to the root voxel's segment
                const int64_t gr = P.v_base + (h & ~kMask);
                const uint32_t ogr = off[gr];
                c = vm[(int64_t)ogr + 1];
                cs = (int64_t)ogr - 2 * gr;
                dil = true;
            } else {
                c = h;
                cs = (int64_t)og - 2 * g;
            }
        }
        if (c == 0) {
            const int32_t pos = atomicAdd(&fb_count[job.pair], 1);
            fb_list[P.p_base + pos] = (uint32_t)i;
            fb_key[P.p_base + pos] = ~0ull;
            nn_idx[gp] = -1 - pos;
        } else {
            float bd = INFINITY;
            uint32_t bj = 0;
            const float4* seg = qs4 + cs;
            for (uint32_t t = 0; t < c; ++t) {
                const float4 q = seg[t];
                const float d = dist2(sx, sy, sz, q.x, q.y, q.z);
                if (d < bd) {
                    bd = d;
                    bj = __float_as_uint(q.w);
                }
            }
            nn_idx[gp] = (int32_t)bj;
            nn_d2[gp] = bd;
        }
    }
    // telemetry: candidates scanned and dilated lookups, one atomic per wave
    unsigned long long cw = c;
    for (int d = kWave / 2; d > 0; d >>= 1) cw += __shfl_xor(cw, d, kWave);
    const unsigned long long dw = (unsigned long long)__popcll(__ballot(dil));
    if ((threadIdx.x & (kWave - 1)) == 0 && (cw | dw)) {
        atomicAdd(&ctr[2 * job.pair], cw);
        atomicAdd(&ctr[2 * job.pair + 1], dw);
    }
}

// Global search.  Work item = (pair, chunk of kFbQ listed queries, tile of
// kFbT targets); items are enumerated from the device-side list lengths, so
// the launch shape is fixed (graph-capturable) whatever the number of misses.
constexpr int kFbThreads = 256;
constexpr int kFbQ = kFbThreads;
constexpr int kFbT = 1024;
constexpr int kMaxPairs = 4096;

__global__ __launch_bounds__(kFbThreads) void k_fallback(const PairDev* __restrict__ pd, int npairs,
                                                         const float* __restrict__ qx, const float* __restrict__ qy,
                                                         const float* __restrict__ qz, const float* __restrict__ px,
                                                         const float* __restrict__ py, const float* __restrict__ pz,
                                                         const PairState* __restrict__ st,
                                                         const int32_t* __restrict__ fb_count,
                                                         const uint32_t* __restrict__ fb_list,
                                                         unsigned long long* __restrict__ fb_key)
{
    __shared__ int32_t s_pref[kMaxPairs + 1];
    __shared__ float tx[kFbT], ty[kFbT], tz[kFbT];
    // items per pair, loaded in parallel, then an in-LDS running sum
    for (int p = threadIdx.x; p < npairs; p += kFbThreads) {
        const int64_t F = fb_count[p];
        s_pref[p + 1] = F > 0 ? (int32_t)(((F + kFbQ - 1) / kFbQ) * ((pd[p].n + kFbT - 1) / kFbT)) : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t acc = 0;
        s_pref[0] = 0;
        for (int p = 1; p <= npairs; ++p) {
            acc += s_pref[p];
            s_pref[p] = acc;
        }
    }
    __syncthreads();
    const int32_t total = s_pref[npairs];
    for (int32_t item = blockIdx.x; item < total; item += gridDim.x) {
        int lo = 0, hi = npairs;   // last p with s_pref[p] <= item
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_pref[mid] <= item) lo = mid;
            else hi = mid;
        }
        const int p = lo;
        const PairDev& P = pd[p];
        const int32_t local = item - s_pref[p];
        const int32_t ntile = (int32_t)((P.n + kFbT - 1) / kFbT);
        const int32_t qc = local / ntile, tile = local % ntile;
        const int64_t t0 = (int64_t)tile * kFbT;
        const int tn = (int)min((int64_t)kFbT, P.n - t0);
        __syncthreads();
        for (int j = threadIdx.x; j < tn; j += kFbThreads) {
            const int64_t g = P.q_base + t0 + j;
            tx[j] = qx[g];
            ty[j] = qy[g];
            tz[j] = qz[g];
        }
        __syncthreads();
        const int32_t slot = qc * kFbQ + threadIdx.x;
        if (slot < fb_count[p]) {
            const uint32_t i = fb_list[P.p_base + slot];
            const int64_t gp = P.p_base + i;
            float sx, sy, sz;
            transform(st[p].Rtf, px[gp], py[gp], pz[gp], sx, sy, sz);
            float bd = INFINITY;
            int bj = 0;
            for (int j = 0; j < tn; ++j) {
                const float d = dist2(sx, sy, sz, tx[j], ty[j], tz[j]);
                if (d < bd) {
                    bd = d;
                    bj = j;
                }
            }
            const unsigned long long key =
                ((unsigned long long)__float_as_uint(bd) << 32) | (unsigned long long)(uint32_t)(t0 + bj);
            atomicMin(&fb_key[P.p_base + slot], key);
        }
    }
}

// Writes the global-search results of the listed queries into nn_idx/nn_d2.
__global__ __launch_bounds__(256) void k_fb_finalize(const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                                                     const unsigned long long* __restrict__ fb_key,
                                                     int32_t* __restrict__ nn_idx, float* __restrict__ nn_d2,
                                                     int32_t* __restrict__ flags)
{
    const BlockJob job = jobs[blockIdx.x];
    const PairDev& P = pd[job.pair];
    const int64_t i = (int64_t)job.start + threadIdx.x;
    if (i >= P.m) return;
    const int64_t gp = P.p_base + i;
    const int32_t j = nn_idx[gp];
    if (j >= 0) return;
    const unsigned long long key = fb_key[P.p_base + (-1 - j)];
    const uint32_t jj = (uint32_t)(key & 0xFFFFFFFFull);
    if (jj >= (uint64_t)P.n) atomicOr(&flags[job.pair], 2);   // unresolved global search (never expected)
    nn_idx[gp] = (int32_t)jj;
    nn_d2[gp] = __uint_as_float((uint32_t)(key >> 32));
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Moments of the correspondences in float64 (sum p, sum q, sum p q^T,
// sum d, count), one partial per block, reduced in a fixed order.
__global__ __launch_bounds__(256) void k_moments(const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                                                 const float* __restrict__ px, const float* __restrict__ py,
                                                 const float* __restrict__ pz, const float* __restrict__ qx,
                                                 const float* __restrict__ qy, const float* __restrict__ qz,
                                                 const PairState* __restrict__ st,
                                                 const unsigned long long* __restrict__ fb_key,
                                                 int32_t* __restrict__ nn_idx, float* __restrict__ nn_d2,
                                                 double* __restrict__ part, int32_t* __restrict__ flags)
{
    __shared__ double red[kMoments][256 / kWave];
    const BlockJob job = jobs[blockIdx.x];
    const PairDev& P = pd[job.pair];
    double a[kMoments];
#pragma unroll
    for (int k = 0; k < kMoments; ++k) a[k] = 0.0;
    const int64_t i = (int64_t)job.start + threadIdx.x;
    if (!st[job.pair].done && i < P.m) {
        const int64_t gp = P.p_base + i;
        int32_t j = nn_idx[gp];
        float d;
        if (j < 0) {
            const unsigned long long key = fb_key[P.p_base + (-1 - j)];
            j = (int32_t)(uint32_t)(key & 0xFFFFFFFFull);
            d = __uint_as_float((uint32_t)(key >> 32));
            nn_idx[gp] = j;
            nn_d2[gp] = d;
        } else {
            d = nn_d2[gp];
        }
        if ((uint32_t)j >= (uint64_t)P.n) {   // unresolved global search (never expected): flag, do not read
            atomicOr(&flags[job.pair], 2);
            j = 0;
        }
        const int64_t gq = P.q_base + j;
        const double p[3] = {px[gp], py[gp], pz[gp]};
        const double q[3] = {qx[gq], qy[gq], qz[gq]};
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            a[r] = p[r];
            a[3 + r] = q[r];
#pragma unroll
            for (int c = 0; c < 3; ++c) a[6 + 3 * r + c] = p[r] * q[c];
        }
        a[15] = (double)d;
        a[16] = 1.0;
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < kMoments; ++k) {
        const double s = wave_sum(a[k]);
        if (lane == 0) red[k][w] = s;
    }
    __syncthreads();
    if (threadIdx.x < kMoments) {
        double s = red[threadIdx.x][0];
#pragma unroll
        for (int k = 1; k < 256 / kWave; ++k) s += red[threadIdx.x][k];
        part[(int64_t)blockIdx.x * kMoments + threadIdx.x] = s;
    }
}

__global__ void k_copy_fb(const int32_t* __restrict__ fb_count, int32_t* __restrict__ out, int npairs)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < npairs) out[p] = fb_count[p];
}

}  // namespace

void launch_nns_local(const PairDev* pd, const BlockJob* jobs, int njobs, int block, const float* px, const float* py,
                      const float* pz, const PairState* st, const uint32_t* off, const uint32_t* vm, const float4* qs4,
                      int32_t* nn_idx, float* nn_d2, int32_t* fb_count, uint32_t* fb_list,
                      unsigned long long* fb_key, unsigned long long* ctr, hipStream_t s)
{
    if (njobs <= 0) return;
#define VICP_NNS(BS)                                                                                                  \
    hipLaunchKernelGGL(k_nns_local<BS>, dim3(njobs), dim3(BS), 0, s, pd, jobs, px, py, pz, st, off, vm, qs4, nn_idx, \
                       nn_d2, fb_count, fb_list, fb_key, ctr)
    switch (block) {
    case 64: VICP_NNS(64); break;
    case 128: VICP_NNS(128); break;
    case 512: VICP_NNS(512); break;
    default: VICP_NNS(256); break;
    }
#undef VICP_NNS
}

void launch_fallback(const PairDev* pd, int npairs, int grid, const float* qx, const float* qy, const float* qz,
                     const float* px, const float* py, const float* pz, const PairState* st, const int32_t* fb_count,
                     const uint32_t* fb_list, unsigned long long* fb_key, hipStream_t s)
{
    if (npairs <= 0 || npairs > kMaxPairs) return;
    hipLaunchKernelGGL(k_fallback, dim3(grid), dim3(kFbThreads), 0, s, pd, npairs, qx, qy, qz, px, py, pz, st,
                       fb_count, fb_list, fb_key);
}

void launch_fb_finalize(const PairDev* pd, const BlockJob* jobs, int njobs, const unsigned long long* fb_key,
                        int32_t* nn_idx, float* nn_d2, int32_t* flags, hipStream_t s)
{
    if (njobs <= 0) return;
    hipLaunchKernelGGL(k_fb_finalize, dim3(njobs), dim3(256), 0, s, pd, jobs, fb_key, nn_idx, nn_d2, flags);
}

void launch_moments(const PairDev* pd, const BlockJob* jobs, int njobs, const float* px, const float* py,
                    const float* pz, const float* qx, const float* qy, const float* qz, const PairState* st,
                    const unsigned long long* fb_key, int32_t* nn_idx, float* nn_d2, double* part, int32_t* flags,
                    hipStream_t s)
{
    if (njobs <= 0) return;
    hipLaunchKernelGGL(k_moments, dim3(njobs), dim3(256), 0, s, pd, jobs, px, py, pz, qx, qy, qz, st, fb_key, nn_idx,
                       nn_d2, part, flags);
}

void launch_copy_fb(const int32_t* fb_count, int32_t* out, int npairs, hipStream_t s)
{
    if (npairs <= 0) return;
    hipLaunchKernelGGL(k_copy_fb, dim3((npairs + 255) / 256), dim3(256), 0, s, fb_count, out, npairs);
}

}  // namespace vicp
