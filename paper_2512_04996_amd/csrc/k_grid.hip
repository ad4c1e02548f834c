// k_grid.hip -- target grid build: bounding box, voxelise + count (Alg. 1,
// GPU part), offsets by a single-pass scan (Alg. 1, CPU part, moved to the
// GPU), scatter into segments and canonical in-segment order (Alg. 2); the
// source's bucketing by target voxel (the search's query order), the same
// count / scan / place / rank shape over the source; and each of those four
// passes paired with the target's in one launch.  Kernel bodies are device
// functions of a block index, so a paired launch runs either body.
#include <algorithm>

#include "vicp_internal.hpp"

namespace vicp {

namespace {

constexpr int kThreads = 256;
constexpr int kWave = 64;

// Order-preserving map float -> uint32 (for atomic min/max of floats).
__device__ __forceinline__ uint32_t ordered(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ uint32_t wave_min(uint32_t v)
{
    for (int d = kWave / 2; d > 0; d >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, d, kWave));
    return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v)
{
    for (int d = kWave / 2; d > 0; d >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, d, kWave));
    return v;
}

// Voxel of a target point (float32: subtract, multiply, floor; x fastest).
// Returns false when the point is outside the grid.
__device__ __forceinline__ bool voxel_id(const PairDev& P, float x, float y, float z, uint32_t& v)
{
    float fx = (x - P.ox) * P.inv;
    float fy = (y - P.oy) * P.inv;
    float fz = (z - P.oz) * P.inv;
    bool in = (fx >= 0.0f) && (fx < P.fDx) && (fy >= 0.0f) && (fy < P.fDy) && (fz >= 0.0f) && (fz < P.fDz);
    if (!in) return false;
    uint32_t ix = (uint32_t)floorf(fx), iy = (uint32_t)floorf(fy), iz = (uint32_t)floorf(fz);
    v = ix + (uint32_t)P.Dx * (iy + (uint32_t)P.Dy * iz);
    return true;
}

// --------------------------------------------------------------------------
// bounding box partial per block: box[8 b + 0..2] = ordered min, [3..5] =
// ordered max, [6] = non-finite flag, [7] = the build's tag.  box is host
// memory mapped for the device: the host waits for the tags instead of a
// copy and a stream synchronisation.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_aabb(const float* __restrict__ qx, const float* __restrict__ qy,
                                                   const float* __restrict__ qz, const PairDev* __restrict__ pd,
                                                   const BlockJob* __restrict__ jobs, int items, uint32_t* box,
                                                   uint32_t tag)
{
    __shared__ uint32_t red[7][kThreads / kWave];
    const BlockJob job = jobs[blockIdx.x];
    const PairDev& P = pd[job.pair];
    uint32_t mn[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, mx[3] = {0u, 0u, 0u}, bad = 0;
    const int64_t end = min((int64_t)job.start + items, P.n);
    // kAabbUnroll points per thread per round, every load issued before the
    // first compare (a load-compare loop waits for each point in turn)
    constexpr int kAabbUnroll = 8;
    for (int64_t i0 = job.start + threadIdx.x; i0 < end; i0 += (int64_t)kAabbUnroll * kThreads) {
        float c[kAabbUnroll][3];
#pragma unroll
        for (int u = 0; u < kAabbUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * kThreads;
            const int64_t g = P.q_base + (i < end ? i : job.start);
            c[u][0] = qx[g];
            c[u][1] = qy[g];
            c[u][2] = qz[g];
        }
#pragma unroll
        for (int u = 0; u < kAabbUnroll; ++u) {
            if (i0 + (int64_t)u * kThreads >= end) continue;
            for (int a = 0; a < 3; ++a) {
                if (!isfinite(c[u][a])) {
                    bad = 1;
                    continue;
                }
                uint32_t o = ordered(c[u][a]);
                mn[a] = min(mn[a], o);
                mx[a] = max(mx[a], o);
            }
        }
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int a = 0; a < 3; ++a) {
        mn[a] = wave_min(mn[a]);
        mx[a] = wave_max(mx[a]);
    }
    bad = wave_max(bad);
    if (lane == 0) {
        for (int a = 0; a < 3; ++a) {
            red[a][w] = mn[a];
            red[3 + a][w] = mx[a];
        }
        red[6][w] = bad;
    }
    __syncthreads();
    // one partial per block (no atomics: same-address atomics from many
    // blocks serialise across the XCDs); the host, which needs the box
    // anyway, combines the partials per pair.  One thread writes the seven
    // values, then, after a system-scope fence (the host must never see the
    // tag before the values), the tag.
    if (threadIdx.x == 0) {
        uint32_t* out = box + 8 * (int64_t)blockIdx.x;
        for (int f = 0; f < 7; ++f) {
            uint32_t r = red[f][0];
            for (int k = 1; k < kThreads / kWave; ++k) r = (f < 3) ? min(r, red[f][k]) : max(r, red[f][k]);
            out[f] = r;
        }
        __threadfence_system();
        __hip_atomic_store(out + 7, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// --------------------------------------------------------------------------
// voxelise + count with a per-block LDS hash (32-bit key, 32-bit count):
// one global atomic per distinct (block, voxel), which also hands each point
// its slot inside the voxel's segment.  BS points per block share one hash
// of 2 BS slots.
// --------------------------------------------------------------------------
constexpr int kSlots = 2 * kThreads;

constexpr int log2i(int x) { return x <= 1 ? 0 : 1 + log2i(x / 2); }

//
// kDirect: VANICP's monolithic layout instead.  The point's slot is its
// position in the voxel's fixed block of `cap` records, and the point is
// copied there as (x, y, z, index) when the block has room; `hist` then
// counts every point of the voxel, so a count above `cap` marks a block that
// overflowed.
template <bool kDirect, int BS>
__device__ __forceinline__ void count_block(int bid, const float* __restrict__ qx, const float* __restrict__ qy,
                                              const float* __restrict__ qz, const PairDev* __restrict__ pd,
                                              const BlockJob* __restrict__ jobs, uint32_t* __restrict__ hist,
                                              uint32_t* __restrict__ vox, uint32_t* __restrict__ rank,
                                              uint32_t* err, float4* __restrict__ blk, uint32_t cap,
                                              uint32_t* __restrict__ big_list, uint32_t* __restrict__ big_count)
{
    constexpr int kS = 2 * BS;
    constexpr int kShift = 32 - log2i(kS);
    __shared__ uint32_t skey[kS];
    __shared__ uint32_t scnt[kS];
    __shared__ uint32_t sbase[kS];
    for (int s = threadIdx.x; s < kS; s += BS) {
        skey[s] = kNone;
        scnt[s] = 0;
    }
    __syncthreads();
    const BlockJob job = jobs[bid];
    const PairDev& P = pd[job.pair];
    const int64_t i = (int64_t)job.start + threadIdx.x;
    bool valid = i < P.n;
    uint32_t v = 0, slot = 0, lr = 0;
    int64_t g = 0;
    float x = 0.0f, y = 0.0f, z = 0.0f;
    if (valid) {
        g = P.q_base + i;
        x = qx[g];
        y = qy[g];
        z = qz[g];
        if (!voxel_id(P, x, y, z, v)) {
            atomicOr(err, 1u);   // cannot happen for a target inside its own box
            valid = false;
        }
    }
    if (valid) {
        slot = (v * 2654435761u) >> kShift;
        while (true) {
            uint32_t prev = atomicCAS(&skey[slot], kNone, v);
            if (prev == kNone || prev == v) break;
            slot = (slot + 1) & (kS - 1);
        }
        lr = atomicAdd(&scnt[slot], 1u);
    }
    __syncthreads();
    // one global atomic per occupied slot, this thread's kS / BS slots all in
    // flight together (a loop of atomics waits for each return in turn)
    {
        constexpr int kPer = kS / BS;
        uint32_t kk[kPer], cc[kPer], bb[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            kk[j] = skey[threadIdx.x + j * BS];
            cc[j] = scnt[threadIdx.x + j * BS];
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) bb[j] = kk[j] != kNone ? atomicAdd(&hist[P.v_base + kk[j]], cc[j]) : 0u;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            sbase[threadIdx.x + j * BS] = bb[j];
            // the one addition that takes a count across kSegSortMin lists
            // the voxel (counts only grow, so that happens once per voxel)
            if (big_list && kk[j] != kNone && bb[j] < kSegSortMin && bb[j] + cc[j] >= kSegSortMin)
                big_list[atomicAdd(big_count, 1u)] = (uint32_t)(P.v_base + kk[j]);
        }
    }
    __syncthreads();
    if (valid) {
        const uint32_t r = sbase[slot] + lr;
        if (kDirect) {
            if (r < cap) blk[(P.v_base + v) * (int64_t)cap + r] = make_float4(x, y, z, __uint_as_float((uint32_t)i));
        } else {
            vox[g] = v;
            rank[g] = r;
        }
    }
}

template <bool kDirect, int BS>
__global__ __launch_bounds__(BS) void k_count(const float* __restrict__ qx, const float* __restrict__ qy,
                                              const float* __restrict__ qz, const PairDev* __restrict__ pd,
                                              const BlockJob* __restrict__ jobs, uint32_t* __restrict__ hist,
                                              uint32_t* __restrict__ vox, uint32_t* __restrict__ rank,
                                              uint32_t* err, float4* __restrict__ blk, uint32_t cap,
                                              uint32_t* __restrict__ big_list, uint32_t* __restrict__ big_count)
{
    count_block<kDirect, BS>((int)blockIdx.x, qx, qy, qz, pd, jobs, hist, vox, rank, err, blk, cap, big_list, big_count);
}

// --------------------------------------------------------------------------
// The same count with Alg. 1's fused hash entry: one 32-bit LDS word holds
// the voxel key (high kPackKeyBits bits) and its count in the block (low
// bits), updated by compare-and-swap; the previous count is the point's
// rank in the block.  Two changes keep it correct: the empty slot is
// 0xFFFFFFFF (the paper's 0 aliases voxel 0 with count 0), and the key is 23
// bits wide (the paper's 16 bits hold at most 65,536 voxels); a block's 256
// points need 9 count bits.  Grids of 2^23 voxels or more use k_count.
// --------------------------------------------------------------------------
constexpr int kPackCountBits = 9;
constexpr int kPackKeyBits = 32 - kPackCountBits;
constexpr uint32_t kPackCountMask = (1u << kPackCountBits) - 1u;

__global__ __launch_bounds__(kThreads) void k_count_packed(const float* __restrict__ qx, const float* __restrict__ qy,
                                                           const float* __restrict__ qz,
                                                           const PairDev* __restrict__ pd,
                                                           const BlockJob* __restrict__ jobs,
                                                           uint32_t* __restrict__ hist, uint32_t* __restrict__ vox,
                                                           uint32_t* __restrict__ rank, uint32_t* err)
{
    __shared__ uint32_t sent[kSlots];   // (key << kPackCountBits) | count, or empty
    __shared__ uint32_t sbase[kSlots];
    for (int s = threadIdx.x; s < kSlots; s += kThreads) sent[s] = kNone;
    __syncthreads();
    const BlockJob job = jobs[blockIdx.x];
    const PairDev& P = pd[job.pair];
    const int64_t i = (int64_t)job.start + threadIdx.x;
    bool valid = i < P.n;
    uint32_t v = 0, slot = 0, lr = 0;
    int64_t g = 0;
    if (valid) {
        g = P.q_base + i;
        if (!voxel_id(P, qx[g], qy[g], qz[g], v)) {
            atomicOr(err, 1u);
            valid = false;
        }
    }
    if (valid) {
        slot = (v * 2654435761u) >> 23;
        while (true) {
            const uint32_t cur = sent[slot];
            if (cur == kNone) {   // claim the slot with count 1
                if (atomicCAS(&sent[slot], kNone, (v << kPackCountBits) | 1u) == kNone) {
                    lr = 0;
                    break;
                }
                continue;   // someone else claimed it: read again
            }
            if ((cur >> kPackCountBits) == v) {   // this voxel's entry: count + 1
                if (atomicCAS(&sent[slot], cur, cur + 1u) == cur) {
                    lr = cur & kPackCountMask;
                    break;
                }
                continue;
            }
            slot = (slot + 1) & (kSlots - 1);
        }
    }
    __syncthreads();
    for (int s = threadIdx.x; s < kSlots; s += kThreads) {
        const uint32_t e = sent[s];
        if (e != kNone) sbase[s] = atomicAdd(&hist[P.v_base + (e >> kPackCountBits)], e & kPackCountMask);
    }
    __syncthreads();
    if (valid) {
        vox[g] = v;
        rank[g] = sbase[slot] + lr;
    }
}

// Segment headers and search directory from offsets computed elsewhere (the
// host-side offset scan of the Alg. 1 ablation): vm[off[g]] = 0,
// vm[off[g] + 1] = hist[g], dir[g] = (off[g] - 2g, hist[g]).
__global__ void k_seg_headers(const uint32_t* __restrict__ hist, const uint32_t* __restrict__ off, int64_t total,
                              uint32_t* __restrict__ vm, uint2* __restrict__ dir)
{
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t o = off[g], h = hist[g];
        vm[o] = 0u;
        vm[o + 1] = h;
        dir[g] = make_uint2(o - 2u * (uint32_t)g, h);
    }
}

// --------------------------------------------------------------------------
// offsets: off[g] = sum_{u<g} (hist[u] + 2), off[total] = n + 2V, and the
// segment headers vm[off[g]] = 0, vm[off[g] + 1] = hist[g] (kSeg), or a
// plain exclusive scan of hist (!kSeg, for bucketing source points).  Single
// pass, decoupled look-back (tile ids from a ticket so predecessors are
// resident when a tile waits on them).
//
// kSeg also writes the search directory dir[g] = (off[g] - 2g, hist[g]): the
// start of voxel g's points in the segment-ordered float4 copy of the target
// and its count, so that a search reaches its candidates with one load (the
// last dilation ring points empty voxels at their root's entry).
// --------------------------------------------------------------------------
#ifndef VICP_SCAN_ITEMS
#define VICP_SCAN_ITEMS 8
#endif
constexpr int kScanItems = VICP_SCAN_ITEMS;
constexpr int kScanTile = kThreads * kScanItems;
constexpr unsigned long long kFlagAgg = 1ull << 32;
constexpr unsigned long long kFlagIncl = 2ull << 32;

__device__ __forceinline__ unsigned long long ld_status(const unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_status(unsigned long long* p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool kSeg>
__device__ __forceinline__ void scan_block(int bid, const uint32_t* __restrict__ hist, int64_t total,
                                                   uint32_t* __restrict__ off, uint32_t* __restrict__ vm,
                                                   uint2* __restrict__ dir, unsigned long long* status,
                                                   uint32_t* ticket)
{
    // Each thread scans kScanItems consecutive entries; the tile moves between
    // global memory and that blocked layout through LDS (padded rows), so that
    // every global load and store of hist, off and dir is contiguous across
    // the lanes of a wave.
    constexpr int kPad = kScanItems + 1;
    __shared__ uint32_t s_h[kThreads * kPad];
    __shared__ uint32_t s_o[kThreads * kPad];
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wave[kThreads / kWave];
    __shared__ uint32_t s_prefix;
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t tbase = tile * kScanTile;
    auto lds = [](int idx) { return (idx / kScanItems) * kPad + idx % kScanItems; };
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int idx = j * kThreads + (int)threadIdx.x;
        const int64_t g = tbase + idx;
        s_h[lds(idx)] = (g < total) ? hist[g] : 0u;
    }
    __syncthreads();
    const int64_t base = tbase + (int64_t)threadIdx.x * kScanItems;
    uint32_t h[kScanItems];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t g = base + k;
        h[k] = s_h[threadIdx.x * kPad + k];
        sum += (g < total) ? h[k] + (kSeg ? 2u : 0u) : 0u;
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t incl = sum;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t y = (uint32_t)__shfl_up((int)incl, d, kWave);
        if (lane >= d) incl += y;
    }
    if (lane == kWave - 1) s_wave[w] = incl;
    __syncthreads();
    uint32_t wave_off = 0, agg = 0;
#pragma unroll
    for (int k = 0; k < kThreads / kWave; ++k) {
        const uint32_t t = s_wave[k];
        if (k < w) wave_off += t;
        agg += t;
    }
    const uint32_t thread_excl = wave_off + incl - sum;
    if (w == 0) {
        if (tile == 0) {
            if (lane == 0) {
                st_status(&status[0], kFlagIncl | agg);
                s_prefix = 0;
            }
        } else {
            if (lane == 0) st_status(&status[tile], kFlagAgg | agg);
            uint32_t excl = 0;
            int64_t k = tile - 1;
            while (true) {
                const int64_t t = k - lane;
                unsigned long long sv;
                while (true) {
                    sv = (t >= 0) ? ld_status(&status[t]) : kFlagIncl;
                    if (!__any((sv >> 32) == 0)) break;
                    __builtin_amdgcn_s_sleep(1);
                }
                const unsigned long long incl_mask = __ballot((sv >> 32) == 2);
                const int first = incl_mask ? __ffsll((long long)incl_mask) - 1 : kWave;
                uint32_t c = (lane <= first) ? (uint32_t)(sv & 0xFFFFFFFFull) : 0u;
                for (int d = kWave / 2; d > 0; d >>= 1) c += (uint32_t)__shfl_xor((int)c, d, kWave);
                excl += c;
                if (incl_mask) break;
                k -= kWave;
            }
            if (lane == 0) {
                st_status(&status[tile], kFlagIncl | (unsigned long long)(excl + agg));
                s_prefix = excl;
            }
        }
    }
    __syncthreads();
    uint32_t run = s_prefix + thread_excl;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t g = base + k;
        s_o[threadIdx.x * kPad + k] = run;
        if (g < total) {
            run += h[k] + (kSeg ? 2u : 0u);
            if (g == total - 1) off[total] = run;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int idx = j * kThreads + (int)threadIdx.x;
        const int64_t g = tbase + idx;
        if (g < total) {
            const uint32_t o = s_o[lds(idx)];
            off[g] = o;
            if (kSeg) {
                // segment headers from the striped layout too: neighbouring
                // lanes write neighbouring segments
                const uint32_t c = s_h[lds(idx)];
                vm[o] = 0u;
                vm[o + 1] = c;
                dir[g] = make_uint2(o - 2u * (uint32_t)g, c);
            }
        }
    }
}

template <bool kSeg>
__global__ __launch_bounds__(kThreads) void k_scan(const uint32_t* __restrict__ hist, int64_t total,
                                                   uint32_t* __restrict__ off, uint32_t* __restrict__ vm,
                                                   uint2* __restrict__ dir, unsigned long long* status,
                                                   uint32_t* ticket)
{
    scan_block<kSeg>((int)blockIdx.x, hist, total, off, vm, dir, status, ticket);
}

// --------------------------------------------------------------------------
// scatter: point i of pair p goes to its voxel's compact slot (any order)
// --------------------------------------------------------------------------
__device__ __forceinline__ void place_block(int bid, const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                                                    const uint32_t* __restrict__ vox, const uint32_t* __restrict__ rank,
                                                    const uint32_t* __restrict__ off, uint32_t* __restrict__ tmp)
{
    const BlockJob job = jobs[bid];
    const PairDev& P = pd[job.pair];
    const int64_t i = (int64_t)job.start + threadIdx.x;
    if (i >= P.n) return;
    const int64_t gi = P.q_base + i;
    const int64_t g = P.v_base + vox[gi];
    const int64_t pos = (int64_t)off[g] - 2 * g + rank[gi];
    tmp[pos] = (uint32_t)i;
}

__global__ __launch_bounds__(kThreads) void k_place(const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                                                    const uint32_t* __restrict__ vox, const uint32_t* __restrict__ rank,
                                                    const uint32_t* __restrict__ off, uint32_t* __restrict__ tmp)
{
    place_block((int)blockIdx.x, pd, jobs, vox, rank, off, tmp);
}

// --------------------------------------------------------------------------
// canonical order: each compact slot k holds point e of voxel g; its final
// position is the number of points of g with a smaller index (ascending
// order, the reading of Alg. 2 that removes the lock-order dependence).
// Also writes the segment-ordered float4 copy of the target.
// --------------------------------------------------------------------------
__device__ __forceinline__ void rank_sort_block(int bid, const float* __restrict__ qx, const float* __restrict__ qy,
                                                        const float* __restrict__ qz, const PairDev* __restrict__ pd,
                                                        const BlockJob* __restrict__ jobs, const uint32_t* __restrict__ vox,
                                                        const uint32_t* __restrict__ hist, const uint32_t* __restrict__ off,
                                                        const uint32_t* __restrict__ tmp, uint32_t* __restrict__ vm,
                                                        float4* __restrict__ qs4, uint32_t sort_min)
{
    __shared__ uint32_t chunk[kThreads / 64][kCoopChunk];
    const BlockJob job = jobs[bid];
    const PairDev& P = pd[job.pair];
    const int64_t k = (int64_t)job.start + threadIdx.x;
    if (k >= P.n) return;
    const uint32_t e = tmp[P.q_base + k];
    const int64_t ge = P.q_base + e;
    const int64_t g = P.v_base + vox[ge];
    const uint32_t og = off[g];
    const int64_t cs = (int64_t)og - 2 * g;
    const uint32_t c = hist[g];
    if (c >= sort_min && c <= kSegSortMax) return;   // sorted whole by k_sort_segments
    // a wave inside one long segment ranks it together (no early return
    // follows, so every lane reaches both branches' barriers alike)
    const bool coop = wave_full_and_uniform(g) && c >= kCoopMin;
    const uint32_t r = coop ? rank_in_wave(tmp, cs, c, e, chunk[threadIdx.x / 64]) : rank_in(tmp, cs, c, e);
    vm[(int64_t)og + 2 + r] = e;
    qs4[cs + r] = make_float4(qx[ge], qy[ge], qz[ge], __uint_as_float(e));
}

__global__ __launch_bounds__(kThreads) void k_rank_sort(const float* __restrict__ qx, const float* __restrict__ qy,
                                                        const float* __restrict__ qz, const PairDev* __restrict__ pd,
                                                        const BlockJob* __restrict__ jobs, const uint32_t* __restrict__ vox,
                                                        const uint32_t* __restrict__ hist, const uint32_t* __restrict__ off,
                                                        const uint32_t* __restrict__ tmp, uint32_t* __restrict__ vm,
                                                        float4* __restrict__ qs4, uint32_t sort_min)
{
    rank_sort_block((int)blockIdx.x, qx, qy, qz, pd, jobs, vox, hist, off, tmp, vm, qs4, sort_min);
}

// Long segments (kSegSortMin to kSegSortMax points) of a single-pair grid,
// listed by the count: one block per segment writes the segment in
// ascending index order to vm and its float4 copy to qs4, the same words the
// per-point rank writes.  The indices of a segment are distinct, so when
// their range [lo, hi] spans at most kBitmapBits values, an LDS bitmap of
// the range and the running popcount of its words give every index its rank
// directly (O(c + range / 32)); otherwise the block sorts them in LDS with a
// bitonic network (O(c log^2 c)).  Blocks take listed segments in turn.
constexpr int kSortThreads = 1024;
constexpr int kSortBlocks = 256;   // one per long segment on the paper's 16^3 grids (two fit a CU)
constexpr uint32_t kBitmapWords = kSegSortMax / 2;   // bitmap and prefix share the sort buffer
constexpr uint32_t kBitmapBits = 32 * kBitmapWords;

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x)
{
    for (int d = 32; d >= 1; d >>= 1) x = min(x, (uint32_t)__shfl_xor((int)x, d, 64));
    return x;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x)
{
    for (int d = 32; d >= 1; d >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, d, 64));
    return x;
}

__global__ __launch_bounds__(kSortThreads) void k_sort_segments(
    const float* __restrict__ qx, const float* __restrict__ qy, const float* __restrict__ qz,
    const PairDev* __restrict__ pd, const uint32_t* __restrict__ big_list, const uint32_t* __restrict__ big_count,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ off, const uint32_t* __restrict__ tmp,
    uint32_t* __restrict__ vm, float4* __restrict__ qs4)
{
    constexpr int kW = kSortThreads / 64;
    constexpr uint32_t kPer = kBitmapWords / kSortThreads;   // bitmap words per thread
    __shared__ uint32_t sk[kSegSortMax];
    __shared__ uint32_t sred[2][kW];
    __shared__ uint32_t spart[kW];
    const PairDev& P = pd[0];
    const int lane = threadIdx.x & 63, w = threadIdx.x / 64;
    const uint32_t nbig = *big_count;
    for (uint32_t b = blockIdx.x; b < nbig; b += gridDim.x) {
        const uint32_t g = big_list[b];
        const uint32_t c = hist[g];
        if (c > kSegSortMax) continue;   // uniform over the block: ranked point by point
        const uint32_t og = off[g];
        const int64_t cs = (int64_t)og - 2 * (int64_t)g;
        // the range of the segment's indices
        uint32_t lo = 0xFFFFFFFFu, hi = 0;
        for (uint32_t i = threadIdx.x; i < c; i += kSortThreads) {
            const uint32_t e = tmp[cs + i];
            lo = min(lo, e);
            hi = max(hi, e);
        }
        lo = wave_min_u32(lo);
        hi = wave_max_u32(hi);
        __syncthreads();   // the previous segment is done with sk and sred
        if (lane == 0) {
            sred[0][w] = lo;
            sred[1][w] = hi;
        }
        __syncthreads();
        lo = sred[0][0];
        hi = sred[1][0];
#pragma unroll
        for (int e = 1; e < kW; ++e) {
            lo = min(lo, sred[0][e]);
            hi = max(hi, sred[1][e]);
        }
        if (hi - lo < kBitmapBits) {   // uniform over the block
            uint32_t* bits = sk;
            uint32_t* pre = sk + kBitmapWords;
            const uint32_t nw = ((hi - lo) >> 5) + 1;
            for (uint32_t i = threadIdx.x; i < nw; i += kSortThreads) bits[i] = 0u;
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < c; i += kSortThreads) {
                const uint32_t d = tmp[cs + i] - lo;
                atomicOr(&bits[d >> 5], 1u << (d & 31));
            }
            __syncthreads();
            // exclusive running popcount: kPer consecutive words per thread,
            // then a scan of the threads' sums
            const uint32_t w0 = threadIdx.x * kPer;
            uint32_t cnt[kPer];
            uint32_t sum = 0;
#pragma unroll
            for (uint32_t q = 0; q < kPer; ++q) {
                cnt[q] = w0 + q < nw ? (uint32_t)__popc(bits[w0 + q]) : 0u;
                sum += cnt[q];
            }
            uint32_t incl = sum;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t y = (uint32_t)__shfl_up((int)incl, d, 64);
                if (lane >= d) incl += y;
            }
            if (lane == 63) spart[w] = incl;
            __syncthreads();
            uint32_t run = incl - sum;
            for (int e = 0; e < w; ++e) run += spart[e];
#pragma unroll
            for (uint32_t q = 0; q < kPer; ++q) {
                if (w0 + q < nw) pre[w0 + q] = run;
                run += cnt[q];
            }
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < c; i += kSortThreads) {
                const uint32_t e = tmp[cs + i];
                const uint32_t d = e - lo;
                const uint32_t r = pre[d >> 5] + (uint32_t)__popc(bits[d >> 5] & ((1u << (d & 31)) - 1u));
                const int64_t ge = P.q_base + e;
                vm[(int64_t)og + 2 + r] = e;
                qs4[cs + r] = make_float4(qx[ge], qy[ge], qz[ge], __uint_as_float(e));
            }
            continue;
        }
        uint32_t np = 1;
        while (np < c) np <<= 1;
        for (uint32_t i = threadIdx.x; i < np; i += kSortThreads) sk[i] = i < c ? tmp[cs + i] : 0xFFFFFFFFu;
        __syncthreads();
        // one thread per compare-exchange pair (p -> elements i, i + j).  At
        // distance j <= 32 the 64 pairs of a wave lie in 128 elements of its
        // own, so a wave barrier orders the stage; the block synchronises
        // around stages of larger distance only.
        for (uint32_t k = 2; k <= np; k <<= 1)
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                for (uint32_t p = threadIdx.x; p < np / 2; p += kSortThreads) {
                    const uint32_t i = ((p & ~(j - 1u)) << 1) | (p & (j - 1u));
                    const uint32_t a = sk[i], bb = sk[i + j];
                    const bool up = (i & k) == 0;
                    if ((a > bb) == up) {
                        sk[i] = bb;
                        sk[i + j] = a;
                    }
                }
                const uint32_t jn = j > 1 ? j >> 1 : k;   // the next stage's distance
                if (j >= 64 || jn >= 64) {
                    __syncthreads();
                } else {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
            }
        for (uint32_t r = threadIdx.x; r < c; r += kSortThreads) {
            const uint32_t e = sk[r];
            const int64_t ge = P.q_base + e;
            vm[(int64_t)og + 2 + r] = e;
            qs4[cs + r] = make_float4(qx[ge], qy[ge], qz[ge], __uint_as_float(e));
        }
    }
}

// Zeroes up to four arrays (u32, u64, u32, u32) in one launch.
__global__ void k_clear4(uint32_t* __restrict__ a, int64_t na, unsigned long long* __restrict__ b, int64_t nb,
                         uint32_t* __restrict__ c, int64_t nc, uint32_t* __restrict__ d, int64_t nd, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < na) a[i] = 0u;
        if (i < nb) b[i] = 0ull;
        if (i < nc) c[i] = 0u;
        if (i < nd) d[i] = 0u;
    }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// --------------------------------------------------------------------------
// source bucketing by target voxel at the current pose (outside -> bucket V)
// --------------------------------------------------------------------------
constexpr int kBThreads = 256;
constexpr int kBSlots = 2 * kBThreads;

__device__ __forceinline__ void src_bucket_block(int bid, const PairDev* __restrict__ pd,
                                                          const BlockJob* __restrict__ jobs,
                                                          const float* __restrict__ px, const float* __restrict__ py,
                                                          const float* __restrict__ pz,
                                                          const PairState* __restrict__ st, uint32_t* __restrict__ sh,
                                                          uint32_t* __restrict__ skey, uint32_t* __restrict__ srank,
                                                          int32_t* __restrict__ sbig, int32_t* __restrict__ flags)
{
    __shared__ uint32_t key_[kBSlots];
    __shared__ uint32_t cnt_[kBSlots];
    __shared__ uint32_t base_[kBSlots];
    for (int s = threadIdx.x; s < kBSlots; s += kBThreads) {
        key_[s] = kNone;
        cnt_[s] = 0;
    }
    __syncthreads();
    const BlockJob job = jobs[bid];
    const PairDev& P = pd[job.pair];
    const int64_t i = (int64_t)job.start + threadIdx.x;
    const bool valid = i < P.m;
    uint32_t key = 0, slot = 0, lr = 0;
    if (valid) {
        const int64_t gp = P.p_base + i;
        const float x = px[gp], y = py[gp], z = pz[gp];
        // this pass reads every source point, so it also flags non-finite
        // coordinates (bit 0 of the pair's fault flags)
        if (!(isfinite(x) && isfinite(y) && isfinite(z))) atomicOr(&flags[job.pair], 1);
        float sx, sy, sz;
        transform(st[job.pair].Rtf, x, y, z, sx, sy, sz);
        uint32_t v;
        int64_t b;
        if (voxel_of(P, sx, sy, sz, v))
            b = (int64_t)v * P.s_chunks + (P.s_shift < 62 ? (i >> P.s_shift) : 0);
        else
            b = P.V * P.s_chunks + (i >> kOutShift);
        key = (uint32_t)(P.s_base + b);
        slot = (key * 2654435761u) >> 23;
        while (true) {
            const uint32_t prev = atomicCAS(&key_[slot], kNone, key);
            if (prev == kNone || prev == key) break;
            slot = (slot + 1) & (kBSlots - 1);
        }
        lr = atomicAdd(&cnt_[slot], 1u);
    }
    __syncthreads();
    // one global atomic per occupied slot, this thread's slots all in flight
    // together (a loop of atomics waits for each return in turn)
    {
        constexpr int kPer = kBSlots / kBThreads;
        uint32_t kk[kPer], cc[kPer], bb[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            kk[j] = key_[threadIdx.x + j * kBThreads];
            cc[j] = cnt_[threadIdx.x + j * kBThreads];
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) bb[j] = kk[j] != kNone ? atomicAdd(&sh[kk[j]], cc[j]) : 0u;
        bool big = false;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            base_[threadIdx.x + j * kBThreads] = bb[j];
            big |= kk[j] != kNone && bb[j] + cc[j] > kRankCap;
        }
        if (big) atomicOr(&sbig[job.pair], 1);
    }
    __syncthreads();
    if (valid) {
        skey[P.p_base + i] = key;
        srank[P.p_base + i] = base_[slot] + lr;
    }
}

__global__ __launch_bounds__(kBThreads) void k_src_bucket(const PairDev* __restrict__ pd,
                                                          const BlockJob* __restrict__ jobs,
                                                          const float* __restrict__ px, const float* __restrict__ py,
                                                          const float* __restrict__ pz,
                                                          const PairState* __restrict__ st, uint32_t* __restrict__ sh,
                                                          uint32_t* __restrict__ skey, uint32_t* __restrict__ srank,
                                                          int32_t* __restrict__ sbig, int32_t* __restrict__ flags)
{
    src_bucket_block((int)blockIdx.x, pd, jobs, px, py, pz, st, sh, skey, srank, sbig, flags);
}

// Puts each source point's index at its bucket position (a global position
// inside the pair's range, because buckets are concatenated in pair order);
// the order inside a bucket is whatever the counting atomics gave.
__device__ __forceinline__ void src_place_block(int bid, const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                                                   const uint32_t* __restrict__ skey,
                                                   const uint32_t* __restrict__ srank,
                                                   const uint32_t* __restrict__ soff, uint32_t* __restrict__ sidx)
{
    const BlockJob job = jobs[bid];
    const PairDev& P = pd[job.pair];
    const int64_t i = (int64_t)job.start + threadIdx.x;
    if (i >= P.m) return;
    const int64_t gp = P.p_base + i;
    sidx[(int64_t)soff[skey[gp]] + srank[gp]] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void k_src_place(const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                                                   const uint32_t* __restrict__ skey,
                                                   const uint32_t* __restrict__ srank,
                                                   const uint32_t* __restrict__ soff, uint32_t* __restrict__ sidx)
{
    src_place_block((int)blockIdx.x, pd, jobs, skey, srank, soff, sidx);
}

// Final position = bucket start + the number of smaller indices in the
// bucket (ascending order within a bucket); a pair with a bucket above
// kRankCap keeps its points in index order instead.
__device__ __forceinline__ void src_rank_block(int bid, const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                                                  const float* __restrict__ px, const float* __restrict__ py,
                                                  const float* __restrict__ pz, const uint32_t* __restrict__ skey,
                                                  const uint32_t* __restrict__ soff, const uint32_t* __restrict__ sidx,
                                                  const int32_t* __restrict__ sbig, float4* __restrict__ ps4)
{
    const BlockJob job = jobs[bid];
    const PairDev& P = pd[job.pair];
    const int64_t i = (int64_t)job.start + threadIdx.x;
    if (i >= P.m) return;
    const int64_t gp = P.p_base + i;
    int64_t pos = gp;
    if (sbig[job.pair] == 0) {
        const uint32_t key = skey[gp];
        const uint32_t lo = soff[key], hi = soff[key + 1];
        pos = (int64_t)lo + rank_in(sidx, lo, hi - lo, (uint32_t)i);
    }
    ps4[pos] = make_float4(px[gp], py[gp], pz[gp], __uint_as_float((uint32_t)i));
}

__global__ __launch_bounds__(256) void k_src_rank(const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                                                  const float* __restrict__ px, const float* __restrict__ py,
                                                  const float* __restrict__ pz, const uint32_t* __restrict__ skey,
                                                  const uint32_t* __restrict__ soff, const uint32_t* __restrict__ sidx,
                                                  const int32_t* __restrict__ sbig, float4* __restrict__ ps4)
{
    src_rank_block((int)blockIdx.x, pd, jobs, px, py, pz, skey, soff, sidx, sbig, ps4);
}


// --------------------------------------------------------------------------
// The refill and the source plan side by side (vicp_rebuild_register): the
// two are independent, so each of their passes shares one launch with the
// other's matching pass, the refill's blocks first, then the plan's.  A
// block runs one of the two bodies, so each keeps its own barriers, LDS and
// scan tickets (a scan's tiles wait only on earlier tiles of the same scan,
// which took their tickets first and so are already running).
// --------------------------------------------------------------------------
static_assert(kBThreads == kThreads, "the paired passes share one block size");

__global__ __launch_bounds__(kThreads) void k_count_bucket(
    const float* __restrict__ qx, const float* __restrict__ qy, const float* __restrict__ qz,
    const PairDev* __restrict__ pd, const BlockJob* __restrict__ qjobs, int nq, uint32_t* __restrict__ hist,
    uint32_t* __restrict__ vox, uint32_t* __restrict__ rank, uint32_t* err, const BlockJob* __restrict__ pjobs,
    const float* __restrict__ px, const float* __restrict__ py, const float* __restrict__ pz,
    const PairState* __restrict__ st, uint32_t* __restrict__ sh, uint32_t* __restrict__ skey,
    uint32_t* __restrict__ srank, int32_t* __restrict__ sbig, int32_t* __restrict__ flags)
{
    const int b = (int)blockIdx.x;
    if (b < nq)
        count_block<false, kThreads>(b, qx, qy, qz, pd, qjobs, hist, vox, rank, err, nullptr, 0u, nullptr, nullptr);
    else
        src_bucket_block(b - nq, pd, pjobs, px, py, pz, st, sh, skey, srank, sbig, flags);
}

__global__ __launch_bounds__(kThreads) void k_scan_pair(const uint32_t* __restrict__ hist, int64_t total,
                                                        uint32_t* __restrict__ off, uint32_t* __restrict__ vm,
                                                        uint2* __restrict__ dir, unsigned long long* status,
                                                        uint32_t* ticket, int na, const uint32_t* __restrict__ sh,
                                                        int64_t nb, uint32_t* __restrict__ soff,
                                                        unsigned long long* s_status, uint32_t* s_ticket)
{
    if ((int)blockIdx.x < na)
        scan_block<true>(0, hist, total, off, vm, dir, status, ticket);
    else
        scan_block<false>(0, sh, nb, soff, nullptr, nullptr, s_status, s_ticket);
}

__global__ __launch_bounds__(kThreads) void k_place_pair(const PairDev* __restrict__ pd,
                                                         const BlockJob* __restrict__ qjobs, int nq,
                                                         const uint32_t* __restrict__ vox,
                                                         const uint32_t* __restrict__ rank,
                                                         const uint32_t* __restrict__ off, uint32_t* __restrict__ tmp,
                                                         const BlockJob* __restrict__ pjobs,
                                                         const uint32_t* __restrict__ skey,
                                                         const uint32_t* __restrict__ srank,
                                                         const uint32_t* __restrict__ soff, uint32_t* __restrict__ sidx)
{
    const int b = (int)blockIdx.x;
    if (b < nq)
        place_block(b, pd, qjobs, vox, rank, off, tmp);
    else
        src_place_block(b - nq, pd, pjobs, skey, srank, soff, sidx);
}

__global__ __launch_bounds__(kThreads) void k_rank_pair(
    const float* __restrict__ qx, const float* __restrict__ qy, const float* __restrict__ qz,
    const PairDev* __restrict__ pd, const BlockJob* __restrict__ qjobs, int nq, const uint32_t* __restrict__ vox,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ off, const uint32_t* __restrict__ tmp,
    uint32_t* __restrict__ vm, float4* __restrict__ qs4, const BlockJob* __restrict__ pjobs,
    const float* __restrict__ px, const float* __restrict__ py, const float* __restrict__ pz,
    const uint32_t* __restrict__ skey, const uint32_t* __restrict__ soff, const uint32_t* __restrict__ sidx,
    const int32_t* __restrict__ sbig, float4* __restrict__ ps4)
{
    const int b = (int)blockIdx.x;
    if (b < nq)
        rank_sort_block(b, qx, qy, qz, pd, qjobs, vox, hist, off, tmp, vm, qs4, 0xFFFFFFFFu);
    else
        src_rank_block(b - nq, pd, pjobs, px, py, pz, skey, soff, sidx, sbig, ps4);
}

}  // namespace

void launch_aabb(const float* qx, const float* qy, const float* qz, const PairDev* pd, const BlockJob* jobs,
                 int njobs, int items_per_block, uint32_t* box, uint32_t tag, hipStream_t s)
{
    if (njobs <= 0) return;
    launch_timed(k_aabb, dim3(njobs), dim3(kThreads), s, qx, qy, qz, pd, jobs, items_per_block, box, tag);
}

void launch_count(const float* qx, const float* qy, const float* qz, const PairDev* pd, const BlockJob* jobs,
                  int njobs, int block, uint32_t* hist, uint32_t* vox, uint32_t* rank, uint32_t* err, bool packed,
                  hipStream_t s, uint32_t* big_list, uint32_t* big_count)
{
    if (njobs <= 0) return;
    if (packed)
        launch_timed(k_count_packed, dim3(njobs), dim3(kThreads), s, qx, qy, qz, pd, jobs, hist, vox, rank, err);
    else if (block == 1024)
        launch_timed(k_count<false, 1024>, dim3(njobs), dim3(1024), s, qx, qy, qz, pd, jobs, hist, vox, rank, err,
                     (float4*)nullptr, 0u, big_list, big_count);
    else if (block == 512)
        launch_timed(k_count<false, 512>, dim3(njobs), dim3(512), s, qx, qy, qz, pd, jobs, hist, vox, rank, err,
                     (float4*)nullptr, 0u, big_list, big_count);
    else
        launch_timed(k_count<false, kThreads>, dim3(njobs), dim3(kThreads), s, qx, qy, qz, pd, jobs, hist, vox, rank,
                     err, (float4*)nullptr, 0u, big_list, big_count);
}

void launch_count_direct(const float* qx, const float* qy, const float* qz, const PairDev* pd, const BlockJob* jobs,
                         int njobs, uint32_t* cnt, uint32_t* err, float4* blk, uint32_t cap, hipStream_t s)
{
    if (njobs <= 0) return;
    hipLaunchKernelGGL((k_count<true, kThreads>), dim3(njobs), dim3(kThreads), 0, s, qx, qy, qz, pd, jobs, cnt,
                       (uint32_t*)nullptr, (uint32_t*)nullptr, err, blk, cap, (uint32_t*)nullptr,
                       (uint32_t*)nullptr);
}

bool count_packed_fits(int64_t voxels) { return voxels < ((int64_t)1 << kPackKeyBits); }

void launch_seg_headers(const uint32_t* hist, const uint32_t* off, int64_t total, uint32_t* vm, uint2* dir,
                        hipStream_t s)
{
    if (total <= 0) return;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_seg_headers, dim3(blocks), dim3(256), 0, s, hist, off, total, vm, dir);
}

int scan_tiles(int64_t total) { return (int)((total + kScanTile - 1) / kScanTile); }

void launch_scan(const uint32_t* hist, int64_t total, uint32_t* off, uint32_t* vm, uint2* dir,
                 unsigned long long* status, uint32_t* ticket, hipStream_t s)
{
    const int tiles = scan_tiles(total);
    if (tiles <= 0) return;
    if (vm)
        launch_timed(k_scan<true>, dim3(tiles), dim3(kThreads), s, hist, total, off, vm, dir, status, ticket);
    else
        launch_timed(k_scan<false>, dim3(tiles), dim3(kThreads), s, hist, total, off, vm, dir, status, ticket);
}

void launch_place(const PairDev* pd, const BlockJob* jobs, int njobs, const uint32_t* vox, const uint32_t* rank,
                  const uint32_t* off, uint32_t* tmp, hipStream_t s)
{
    if (njobs <= 0) return;
    launch_timed(k_place, dim3(njobs), dim3(kThreads), s, pd, jobs, vox, rank, off, tmp);
}

void launch_rank_sort(const float* qx, const float* qy, const float* qz, const PairDev* pd, const BlockJob* jobs,
                      int njobs, const uint32_t* vox, const uint32_t* hist, const uint32_t* off, const uint32_t* tmp,
                      uint32_t* vm, float4* qs4, hipStream_t s, uint32_t sort_min)
{
    if (njobs <= 0) return;
    launch_timed(k_rank_sort, dim3(njobs), dim3(kThreads), s, qx, qy, qz, pd, jobs, vox, hist, off, tmp, vm, qs4,
                 sort_min);
}

void launch_sort_segments(const float* qx, const float* qy, const float* qz, const PairDev* pd,
                          const uint32_t* big_list, const uint32_t* big_count, const uint32_t* hist,
                          const uint32_t* off, const uint32_t* tmp, uint32_t* vm, float4* qs4, hipStream_t s)
{
    launch_timed(k_sort_segments, dim3(kSortBlocks), dim3(kSortThreads), s, qx, qy, qz, pd, big_list, big_count, hist, off,
                 tmp, vm, qs4);
}

void launch_clear4(uint32_t* a, int64_t na, unsigned long long* b, int64_t nb, uint32_t* c, int64_t nc, uint32_t* d,
                   int64_t nd, hipStream_t s)
{
    const int64_t n = std::max(std::max(na, nb), std::max(nc, nd));
    if (n <= 0) return;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_clear4, dim3(blocks), dim3(256), 0, s, a, na, b, nb, c, nc, d, nd, n);
}

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s)
{
    if (count <= 0) return;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, count);
}

void launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t count, hipStream_t s)
{
    if (count <= 0) return;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, s, p, v, count);
}

void launch_src_bucket(const PairDev* pd, const BlockJob* jobs, int njobs, const float* px, const float* py,
                       const float* pz, const PairState* st, uint32_t* sh, uint32_t* skey, uint32_t* srank,
                       int32_t* sbig, int32_t* flags, hipStream_t s)
{
    if (njobs <= 0) return;
    hipLaunchKernelGGL(k_src_bucket, dim3(njobs), dim3(kBThreads), 0, s, pd, jobs, px, py, pz, st, sh, skey, srank,
                       sbig, flags);
}

void launch_src_place(const PairDev* pd, const BlockJob* jobs, int njobs, const uint32_t* skey,
                      const uint32_t* srank, const uint32_t* soff, uint32_t* sidx, hipStream_t s)
{
    if (njobs <= 0) return;
    hipLaunchKernelGGL(k_src_place, dim3(njobs), dim3(256), 0, s, pd, jobs, skey, srank, soff, sidx);
}

void launch_src_rank(const PairDev* pd, const BlockJob* jobs, int njobs, const float* px, const float* py,
                     const float* pz, const uint32_t* skey, const uint32_t* soff, const uint32_t* sidx,
                     const int32_t* sbig, float4* ps4, hipStream_t s)
{
    if (njobs <= 0) return;
    hipLaunchKernelGGL(k_src_rank, dim3(njobs), dim3(256), 0, s, pd, jobs, px, py, pz, skey, soff, sidx, sbig, ps4);
}


void launch_count_bucket(const float* qx, const float* qy, const float* qz, const PairDev* pd,
                         const BlockJob* qjobs, int nq, uint32_t* hist, uint32_t* vox, uint32_t* rank, uint32_t* err,
                         const BlockJob* pjobs, int np, const float* px, const float* py, const float* pz,
                         const PairState* st, uint32_t* sh, uint32_t* skey, uint32_t* srank, int32_t* sbig,
                         int32_t* flags, hipStream_t s)
{
    if (nq + np <= 0) return;
    launch_timed(k_count_bucket, dim3(nq + np), dim3(kThreads), s, qx, qy, qz, pd, qjobs, nq, hist, vox, rank, err,
                 pjobs, px, py, pz, st, sh, skey, srank, sbig, flags);
}

void launch_scan_pair(const uint32_t* hist, int64_t total, uint32_t* off, uint32_t* vm, uint2* dir,
                      unsigned long long* status, uint32_t* ticket, const uint32_t* sh, int64_t nb, uint32_t* soff,
                      unsigned long long* s_status, uint32_t* s_ticket, hipStream_t s)
{
    const int na = scan_tiles(total), nbt = scan_tiles(nb);
    if (na + nbt <= 0) return;
    launch_timed(k_scan_pair, dim3(na + nbt), dim3(kThreads), s, hist, total, off, vm, dir, status, ticket, na, sh, nb,
                 soff, s_status, s_ticket);
}

void launch_place_pair(const PairDev* pd, const BlockJob* qjobs, int nq, const uint32_t* vox, const uint32_t* rank,
                       const uint32_t* off, uint32_t* tmp, const BlockJob* pjobs, int np, const uint32_t* skey,
                       const uint32_t* srank, const uint32_t* soff, uint32_t* sidx, hipStream_t s)
{
    if (nq + np <= 0) return;
    launch_timed(k_place_pair, dim3(nq + np), dim3(kThreads), s, pd, qjobs, nq, vox, rank, off, tmp, pjobs, skey,
                 srank, soff, sidx);
}

void launch_rank_pair(const float* qx, const float* qy, const float* qz, const PairDev* pd, const BlockJob* qjobs,
                      int nq, const uint32_t* vox, const uint32_t* hist, const uint32_t* off, const uint32_t* tmp,
                      uint32_t* vm, float4* qs4, const BlockJob* pjobs, int np, const float* px, const float* py,
                      const float* pz, const uint32_t* skey, const uint32_t* soff, const uint32_t* sidx,
                      const int32_t* sbig, float4* ps4, hipStream_t s)
{
    if (nq + np <= 0) return;
    launch_timed(k_rank_pair, dim3(nq + np), dim3(kThreads), s, qx, qy, qz, pd, qjobs, nq, vox, hist, off, tmp, vm,
                 qs4, pjobs, px, py, pz, skey, soff, sidx, sbig, ps4);
}

}  // namespace vicp
