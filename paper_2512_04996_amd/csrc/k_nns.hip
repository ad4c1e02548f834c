// k_nns.hip -- correspondence search (Alg. 4).
//
// Local search: one lane per source point.  The transformed point's voxel is
// found by the same float32 quantisation as the targets.  Its entry in the
// search directory (derived from the offsets and count words, and for a
// Mask(root) voxel from the root's, so still no replicated points) gives the
// start and count of its candidates in one 8-byte load, where reading
// offset -> count word -> root offset -> root count word would chain four
// dependent loads.  Candidates are read as float4 (x, y, z, index) from the
// segment-ordered copy of the target, a fixed number of 16-byte loads in
// flight per lane (indices past the end are clamped to the last candidate:
// a repeated candidate never changes a strict minimum); segments are in
// ascending index order, so a strict "<" keeps the lowest index among equal
// distances.
//
// Query order: lanes of a wave that look up different voxels diverge (the
// wave runs the longest segment) and gather from unrelated cache lines.  The
// search can therefore run over a copy of the source bucketed by target
// voxel at the current pose (a counting sort: LDS-hashed bucket counts, a
// plain scan, a placement pass), so neighbouring lanes share segments.
// Results are written back by original index, so the order never changes a
// result.
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

// Voxel of a transformed point, or false when it is outside the grid.
__device__ __forceinline__ bool voxel_of(const PairDev& P, float sx, float sy, float sz, uint32_t& v)
{
    const float fx = (sx - P.ox) * P.inv;
    const float fy = (sy - P.oy) * P.inv;
    const float fz = (sz - P.oz) * P.inv;
    const bool in = (fx >= 0.0f) && (fx < P.fDx) && (fy >= 0.0f) && (fy < P.fDy) && (fz >= 0.0f) && (fz < P.fDz);
    if (in) v = (uint32_t)floorf(fx) + (uint32_t)P.Dx * ((uint32_t)floorf(fy) + (uint32_t)P.Dy * (uint32_t)floorf(fz));
    return in;
}

__device__ __forceinline__ void consider(const float4& q, float sx, float sy, float sz, float& bd, uint32_t& bj)
{
    const float d = dist2(sx, sy, sz, q.x, q.y, q.z);
    if (d < bd) {
        bd = d;
        bj = __float_as_uint(q.w);
    }
}

// LPQ lanes cooperate on one query: each scans every LPQ-th candidate of the
// segment in ascending order (so it keeps the lowest index among its equal
// distances), then the lanes combine by the lexicographic minimum of
// (distance, index) -- the same result as one lane scanning everything, with
// LPQ times more waves in flight to hide the load latency.
template <int BS, int LPQ, bool kSorted>
__global__ __launch_bounds__(BS) void k_nns_local(const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                                                  const float* __restrict__ px, const float* __restrict__ py,
                                                  const float* __restrict__ pz, const float4* __restrict__ ps4,
                                                  const PairState* __restrict__ st, const uint2* __restrict__ dir,
                                                  const float4* __restrict__ qs4,
                                                  int32_t* __restrict__ nn_idx, float* __restrict__ nn_d2,
                                                  int32_t* __restrict__ fb_count, uint32_t* __restrict__ fb_list,
                                                  unsigned long long* __restrict__ fb_key,
                                                  unsigned long long* __restrict__ ctr)
{
    static_assert(LPQ == 1 || LPQ == 2 || LPQ == 4 || LPQ == 8, "lanes per query");
    constexpr int QPB = BS / LPQ;   // queries per block
    const BlockJob job = jobs[blockIdx.x];
    const PairDev& P = pd[job.pair];
    const PairState& S = st[job.pair];
    if (S.done) return;   // uniform over the block
    const int sub = threadIdx.x % LPQ;
    const int64_t t = (int64_t)job.start + threadIdx.x / LPQ;
    const bool active = t < P.m;
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t c = 0, i = 0;
    int64_t cs = 0;
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    bool dil = false;
    if (active) {
        float x, y, z;
        if (kSorted) {
            const float4 pp = ps4[P.p_base + t];
            x = pp.x;
            y = pp.y;
            z = pp.z;
            i = __float_as_uint(pp.w);
        } else {
            x = px[P.p_base + t];
            y = py[P.p_base + t];
            z = pz[P.p_base + t];
            i = (uint32_t)t;
        }
        transform(S.Rtf, x, y, z, sx, sy, sz);
        uint32_t v;
        if (voxel_of(P, sx, sy, sz, v)) {
            const uint2 e = dir[P.v_base + v];
            c = e.y & ~kMask;
            cs = e.x;
            dil = (e.y & kMask) != 0u;
        }
    }
    const int64_t gp = P.p_base + i;
    // queries for the global search: one list append per wave, each query at
    // its rank among the wave's misses (counted on its first lane)
    const bool miss = active && c == 0 && sub == 0;
    const unsigned long long mmask = __ballot(miss);
    if (mmask) {
        const int leader = __ffsll((long long)mmask) - 1;
        int32_t base = 0;
        if (lane == leader) base = atomicAdd(&fb_count[job.pair], (int32_t)__popcll(mmask));
        base = __shfl(base, leader, kWave);
        if (miss) {
            const int32_t pos = base + (int32_t)__popcll(mmask & ((1ull << lane) - 1ull));
            fb_list[P.p_base + pos] = i;
            fb_key[P.p_base + pos] = ~0ull;
            nn_idx[gp] = -1 - pos;
        }
    }
    float bd = INFINITY;
    uint32_t bj = 0xFFFFFFFFu;
    if (active && c > 0) {
        // U candidates per lane per round, all loads issued before the first
        // compare; no serial remainder
        constexpr int U = LPQ <= 2 ? 8 : 4;
        const float4* seg = qs4 + cs;
        const uint32_t last = c - 1u;
        for (uint32_t k = sub; k < c; k += U * LPQ) {
            float4 a[U];
#pragma unroll
            for (int u = 0; u < U; ++u) a[u] = seg[min(k + (uint32_t)(u * LPQ), last)];
#pragma unroll
            for (int u = 0; u < U; ++u) consider(a[u], sx, sy, sz, bd, bj);
        }
    }
    if (LPQ > 1) {
#pragma unroll
        for (int d = 1; d < LPQ; d <<= 1) {
            const float od = __shfl_xor(bd, d, kWave);
            const uint32_t oj = (uint32_t)__shfl_xor((int)bj, d, kWave);
            if (od < bd || (od == bd && oj < bj)) {
                bd = od;
                bj = oj;
            }
        }
    }
    if (active && c > 0 && sub == 0) {
        nn_idx[gp] = (int32_t)bj;
        nn_d2[gp] = bd;
    }
    // telemetry without atomics: one partial per block (candidates scanned,
    // dilated lookups), summed per pair by the solve
    __shared__ unsigned long long red[2][BS / kWave];
    unsigned long long cw = (sub == 0) ? c : 0u;
    for (int d = kWave / 2; d > 0; d >>= 1) cw += __shfl_xor(cw, d, kWave);
    const unsigned long long dw = (unsigned long long)__popcll(__ballot(dil && sub == 0));
    if (lane == 0) {
        red[0][threadIdx.x / kWave] = cw;
        red[1][threadIdx.x / kWave] = dw;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        unsigned long long sm = 0;
        for (int w = 0; w < BS / kWave; ++w) sm += red[threadIdx.x][w];
        ctr[2 * (int64_t)blockIdx.x + threadIdx.x] = sm;
    }
    (void)QPB;
}

// --------------------------------------------------------------------------
// source bucketing by target voxel at the current pose (outside -> bucket V)
// --------------------------------------------------------------------------
constexpr int kBThreads = 256;
constexpr int kBSlots = 2 * kBThreads;

__global__ __launch_bounds__(kBThreads) void k_src_bucket(const PairDev* __restrict__ pd,
                                                          const BlockJob* __restrict__ jobs,
                                                          const float* __restrict__ px, const float* __restrict__ py,
                                                          const float* __restrict__ pz,
                                                          const PairState* __restrict__ st, uint32_t* __restrict__ sh,
                                                          uint32_t* __restrict__ skey, uint32_t* __restrict__ srank)
{
    __shared__ uint32_t key_[kBSlots];
    __shared__ uint32_t cnt_[kBSlots];
    __shared__ uint32_t base_[kBSlots];
    for (int s = threadIdx.x; s < kBSlots; s += kBThreads) {
        key_[s] = kNone;
        cnt_[s] = 0;
    }
    __syncthreads();
    const BlockJob job = jobs[blockIdx.x];
    const PairDev& P = pd[job.pair];
    const int64_t i = (int64_t)job.start + threadIdx.x;
    const bool valid = i < P.m;
    uint32_t key = 0, slot = 0, lr = 0;
    if (valid) {
        const int64_t gp = P.p_base + i;
        float sx, sy, sz;
        transform(st[job.pair].Rtf, px[gp], py[gp], pz[gp], sx, sy, sz);
        uint32_t v;
        if (!voxel_of(P, sx, sy, sz, v)) v = (uint32_t)P.V;
        key = (uint32_t)(P.v_base + job.pair) + v;   // pair p owns buckets [v_base + p, v_base + p + V]
        slot = (key * 2654435761u) >> 23;
        while (true) {
            const uint32_t prev = atomicCAS(&key_[slot], kNone, key);
            if (prev == kNone || prev == key) break;
            slot = (slot + 1) & (kBSlots - 1);
        }
        lr = atomicAdd(&cnt_[slot], 1u);
    }
    __syncthreads();
    for (int s = threadIdx.x; s < kBSlots; s += kBThreads) {
        const uint32_t k = key_[s];
        if (k != kNone) base_[s] = atomicAdd(&sh[k], cnt_[s]);
    }
    __syncthreads();
    if (valid) {
        skey[P.p_base + i] = key;
        srank[P.p_base + i] = base_[slot] + lr;
    }
}

// Places each source point at its bucket position (a global position inside
// the pair's range, because buckets are concatenated in pair order).
__global__ __launch_bounds__(256) void k_src_place(const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                                                   const float* __restrict__ px, const float* __restrict__ py,
                                                   const float* __restrict__ pz, const uint32_t* __restrict__ skey,
                                                   const uint32_t* __restrict__ srank,
                                                   const uint32_t* __restrict__ soff, float4* __restrict__ ps4)
{
    const BlockJob job = jobs[blockIdx.x];
    const PairDev& P = pd[job.pair];
    const int64_t i = (int64_t)job.start + threadIdx.x;
    if (i >= P.m) return;
    const int64_t gp = P.p_base + i;
    const int64_t pos = (int64_t)soff[skey[gp]] + srank[gp];
    ps4[pos] = make_float4(px[gp], py[gp], pz[gp], __uint_as_float((uint32_t)i));
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

__global__ void k_copy_fb(const int32_t* __restrict__ fb_count, int32_t* __restrict__ out, int npairs)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < npairs) out[p] = fb_count[p];
}

}  // namespace

void launch_nns_local(const PairDev* pd, const BlockJob* jobs, int njobs, int block, int lpq, bool sorted,
                      const float* px, const float* py, const float* pz, const float4* ps4, const PairState* st,
                      const uint2* dir, const float4* qs4, int32_t* nn_idx, float* nn_d2,
                      int32_t* fb_count, uint32_t* fb_list, unsigned long long* fb_key, unsigned long long* ctr,
                      hipStream_t s)
{
    if (njobs <= 0) return;
#define VICP_NNS(BS, L, SORTED)                                                                                      \
    hipLaunchKernelGGL((k_nns_local<BS, L, SORTED>), dim3(njobs), dim3(BS), 0, s, pd, jobs, px, py, pz, ps4, st,    \
                       dir, qs4, nn_idx, nn_d2, fb_count, fb_list, fb_key, ctr)
#define VICP_NNS_L(BS, SORTED)                       \
    switch (lpq) {                                   \
    case 2: VICP_NNS(BS, 2, SORTED); break;          \
    case 4: VICP_NNS(BS, 4, SORTED); break;          \
    case 8: VICP_NNS(BS, 8, SORTED); break;          \
    default: VICP_NNS(BS, 1, SORTED); break;         \
    }
#define VICP_NNS_BS(SORTED)                          \
    switch (block) {                                 \
    case 128: VICP_NNS_L(128, SORTED); break;        \
    case 512: VICP_NNS_L(512, SORTED); break;        \
    default: VICP_NNS_L(256, SORTED); break;         \
    }
    if (sorted) {
        VICP_NNS_BS(true)
    } else {
        VICP_NNS_BS(false)
    }
#undef VICP_NNS_BS
#undef VICP_NNS_L
#undef VICP_NNS
}

void launch_src_bucket(const PairDev* pd, const BlockJob* jobs, int njobs, const float* px, const float* py,
                       const float* pz, const PairState* st, uint32_t* sh, uint32_t* skey, uint32_t* srank,
                       hipStream_t s)
{
    if (njobs <= 0) return;
    hipLaunchKernelGGL(k_src_bucket, dim3(njobs), dim3(kBThreads), 0, s, pd, jobs, px, py, pz, st, sh, skey, srank);
}

void launch_src_place(const PairDev* pd, const BlockJob* jobs, int njobs, const float* px, const float* py,
                      const float* pz, const uint32_t* skey, const uint32_t* srank, const uint32_t* soff,
                      float4* ps4, hipStream_t s)
{
    if (njobs <= 0) return;
    hipLaunchKernelGGL(k_src_place, dim3(njobs), dim3(256), 0, s, pd, jobs, px, py, pz, skey, srank, soff, ps4);
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

void launch_copy_fb(const int32_t* fb_count, int32_t* out, int npairs, hipStream_t s)
{
    if (npairs <= 0) return;
    hipLaunchKernelGGL(k_copy_fb, dim3((npairs + 255) / 256), dim3(256), 0, s, fb_count, out, npairs);
}

}  // namespace vicp
