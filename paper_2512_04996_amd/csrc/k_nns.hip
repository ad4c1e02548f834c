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
// Within a bucket the points are then put in ascending index order (each
// counts the smaller indices of its bucket), so the bucketed copy, and every
// per-block sum taken over it, is the same from run to run.
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

__device__ __forceinline__ float dist2(float sx, float sy, float sz, float qx, float qy, float qz)
{
    const float dx = sx - qx, dy = sy - qy, dz = sz - qz;
    return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

// The value of lane (this lane xor d): a DPP quad permutation for d = 1, 2
// (a VALU move), an LDS permute otherwise.
__device__ __forceinline__ uint32_t xor_lanes(uint32_t x, int d)
{
    if (d == 1) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, true);   // quad_perm 1,0,3,2
    if (d == 2) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, true);   // quad_perm 2,3,0,1
    return (uint32_t)__shfl_xor((int)x, d, kWave);
}

__device__ __forceinline__ float xor_lanes(float x, int d) { return __uint_as_float(xor_lanes(__float_as_uint(x), d)); }

// Selects, not branches: a branch lets the compiler sink the index load into
// the taken path and then wait for every load in flight.  kTies: candidates
// come in no particular order, so equal distances compare indices.
template <bool kTies>
__device__ __forceinline__ void consider(const float4& q, float sx, float sy, float sz, float& bd, uint32_t& bj)
{
    const float d = dist2(sx, sy, sz, q.x, q.y, q.z);
    const bool better = d < bd || (kTies && d == bd && __float_as_uint(q.w) < bj);
    bd = better ? d : bd;
    bj = better ? __float_as_uint(q.w) : bj;
}

// The same, keeping the candidate's position in the segment instead of its
// index (positions ascend with indices in a segment), so that a lane carries
// two values per candidate instead of five; the winner's coordinates are
// read once at the end.
__device__ __forceinline__ void consider_pos(const float4& q, uint32_t pos, float sx, float sy, float sz, float& bd,
                                             uint32_t& bk)
{
    const float d = dist2(sx, sy, sz, q.x, q.y, q.z);
    const bool better = d < bd;
    bd = better ? d : bd;
    bk = better ? pos : bk;
}

// The same, also keeping the best candidate's coordinates.
template <bool kTies>
__device__ __forceinline__ void consider(const float4& q, float sx, float sy, float sz, float& bd, uint32_t& bj,
                                         float& bx, float& by, float& bz)
{
    const float d = dist2(sx, sy, sz, q.x, q.y, q.z);
    const bool better = d < bd || (kTies && d == bd && __float_as_uint(q.w) < bj);
    bd = better ? d : bd;
    bj = better ? __float_as_uint(q.w) : bj;
    bx = better ? q.x : bx;
    by = better ? q.y : by;
    bz = better ? q.z : bz;
}

// Exact global search by voxel shells.  A query whose voxel is empty and
// undilated, or outside the grid, takes the exact minimum of (d, j) over all
// n targets (Alg. 4's global search).  Rather than scanning all n, the wave
// visits the occupied voxels of a growing cube of voxels around the query's
// voxel (clamped into the grid) and stops once every target outside the
// visited cube is provably farther than the best found: its squared
// distance is then above the best one even after the float32 rounding of
// the distance, so it can neither win nor tie.  The bound takes each face of
// the cube that is not on the grid's boundary: a target beyond it lies
// beyond that face on its axis and inside the grid box on the other two.
// Faces and the grid box are widened by a margin for the float32 rounding
// of the voxel assignment (floor((q - o) * inv)), so a target assigned to a
// voxel may lie slightly outside it.  All 64 lanes call it with the same
// point; every lane gets the result.  False (nothing found) when a cube of
// kShellMax voxels around does not settle it: the query then goes to the
// exhaustive search, and so does a query whose cube holds so many points
// that a lane would scan more than kShellPoints of them (coarse grids with
// thousands of points in a voxel: the tiled exhaustive search is the faster
// there).  Each batch of a lane's voxels loads its directory entries
// together, then the points of its occupied voxels as one flat run (so a
// lane waits for two rounds of loads per batch, not one per voxel).
constexpr int kShellFirst = 2;   // the smallest first cube: 5^3 voxels
constexpr int kShellMax = 8;     // the largest: 17^3 voxels
constexpr int kShellBatch = 6;     // directory loads in flight per lane (registration)
constexpr int kShellLoads = 4;     // point loads in flight per lane (registration)
constexpr int kShellBatchNN = 12;  // the same in the correspondence search
constexpr int kShellLoadsNN = 8;
constexpr int kShellFirstNN = 4;   // its smallest first cube, 9^3 voxels: one round of 12 x 64 entries
constexpr uint32_t kShellPoints = 384;   // points a lane may scan before the wave gives up

// The point and every quantity derived from it are the same in all lanes
// (scalar registers); a lane keeps only its best candidate's (d, j) and
// segment slot, and the winner's coordinates are read once at the end.
template <int kBatch, int kLoads, int kFirst>
__device__ __forceinline__ bool shell_nearest(const PairDev& P, const uint2* __restrict__ dir,
                                              const float4* __restrict__ qs4, float sx, float sy, float sz,
                                              float& rd, uint32_t& rj, float& rx, float& ry, float& rz)
{
    if (!(isfinite(sx) && isfinite(sy) && isfinite(sz))) return false;   // left to the exhaustive search
    const int lane = threadIdx.x & (kWave - 1);
    const float inv = P.inv, vox = 1.0f / P.inv;
    const float s[3] = {sx, sy, sz};
    const float o[3] = {P.ox, P.oy, P.oz};
    const int D[3] = {P.Dx, P.Dy, P.Dz};
    int c[3];
    float mg[3], d2box[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float f = (s[a] - o[a]) * inv;
        c[a] = f < 0.0f ? 0 : (f >= (float)(D[a] - 1) ? D[a] - 1 : (int)floorf(f));
        c[a] = __builtin_amdgcn_readfirstlane(c[a]);
        // 1e-5 of the coordinates' magnitude and 1e-3 of a voxel: far above
        // the float32 rounding of the assignment and of this arithmetic
        mg[a] = 1e-5f * (fabsf(o[a]) + ((float)D[a] + 1.0f) * vox) + 1e-3f * vox;
        const float lo = o[a] - mg[a], hi = o[a] + (float)D[a] * vox + mg[a];
        const float g = s[a] < lo ? lo - s[a] : (s[a] > hi ? s[a] - hi : 0.0f);
        d2box[a] = g * g;
    }
    float bd = INFINITY;
    uint32_t bj = 0xFFFFFFFFu, bslot = 0u;
    uint32_t scanned = 0u;
    int done_r = -1;   // the cube of this radius has been visited
    // the first cube reaches one voxel past the dilation: a global search's
    // voxel has no occupied voxel within L1 distance L
    int R = min(max(P.pad + 1, kFirst), kShellMax);
    while (true) {
        const int w = 2 * R + 1;
        const int items = w * w * w;
        for (int i0 = lane; i0 < items; i0 += kWave * kBatch) {
            // the batch's directory entries, all in flight together
            uint2 e[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                e[u] = make_uint2(0u, 0u);
                const int it = i0 + u * kWave;
                if (it >= items) continue;
                const int dz = it / (w * w) - R, rem = it % (w * w);
                const int dy = rem / w - R, dx = rem % w - R;
                if (max(abs(dx), max(abs(dy), abs(dz))) <= done_r) continue;   // visited before
                const int vx = c[0] + dx, vy = c[1] + dy, vz = c[2] + dz;
                if (vx < 0 || vy < 0 || vz < 0 || vx >= D[0] || vy >= D[1] || vz >= D[2]) continue;
                e[u] = dir[P.v_base + vx + (int64_t)D[0] * (vy + (int64_t)D[1] * vz)];
            }
            // the points of the batch's occupied voxels (own count, no mask:
            // a dilated voxel's entry points at its root, visited as itself)
            // as one flat run, kLoads loads in flight; a lane past its last
            // point repeats it (a repeat never wins)
            uint32_t end[kBatch];
            uint32_t total = 0u;
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                total += (e[u].y & kMask) ? 0u : e[u].y;
                end[u] = total;
            }
            scanned += total;
            if (__ballot(scanned > kShellPoints)) return false;   // uniform: too many points
            for (uint32_t t0 = 0; t0 < total; t0 += kLoads) {
                float4 q[kLoads];
                uint32_t sl[kLoads];
#pragma unroll
                for (int t = 0; t < kLoads; ++t) {
                    const uint32_t f = min(t0 + (uint32_t)t, total - 1u);
                    uint32_t slot = 0u, start = 0u;
#pragma unroll
                    for (int u = 0; u < kBatch; ++u) {
                        const bool here = f >= start && f < end[u];
                        slot = here ? e[u].x + (f - start) : slot;
                        start = end[u];
                    }
                    sl[t] = slot;
                    q[t] = qs4[slot];
                }
#pragma unroll
                for (int t = 0; t < kLoads; ++t) {
                    const float d = dist2(sx, sy, sz, q[t].x, q[t].y, q[t].z);
                    const uint32_t j = __float_as_uint(q[t].w);
                    const bool better = d < bd || (d == bd && j < bj);
                    bd = better ? d : bd;
                    bj = better ? j : bj;
                    bslot = better ? sl[t] : bslot;
                }
            }
        }
        // the wave's minimum of (d, j): distances are >= 0, so their bits
        // order as the values do
        unsigned long long key = ((unsigned long long)__float_as_uint(bd) << 32) | bj;
#pragma unroll
        for (int m = 1; m < kWave; m <<= 1) {
            const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(key >> 32), m, kWave);
            const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)key, m, kWave);
            const unsigned long long other = ((unsigned long long)hi << 32) | lo;
            key = other < key ? other : key;
        }
        const float best = __uint_as_float((uint32_t)(key >> 32));
        // lower bound on the squared distance of any target outside the
        // visited cube
        float lb2 = INFINITY;
        bool all = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float rest = d2box[(a + 1) % 3] + d2box[(a + 2) % 3];
            if (c[a] - R > 0) {   // targets below the cube's low face on axis a
                all = false;
                const float g = s[a] - (o[a] + (float)(c[a] - R) * vox + mg[a]);
                lb2 = fminf(lb2, (g > 0.0f ? g * g : 0.0f) + rest);
            }
            if (c[a] + R < D[a] - 1) {   // above its high face
                all = false;
                const float g = (o[a] + (float)(c[a] + R + 1) * vox - mg[a]) - s[a];
                lb2 = fminf(lb2, (g > 0.0f ? g * g : 0.0f) + rest);
            }
        }
        const bool found = (uint32_t)(key >> 32) != 0x7F800000u;   // a finite best
        if (found && (all || lb2 * (1.0f - 1e-4f) > best)) {
            const unsigned long long mine = ((unsigned long long)__float_as_uint(bd) << 32) | bj;
            const int owner = __ffsll((long long)__ballot(mine == key)) - 1;
            const float4 wq = qs4[__builtin_amdgcn_readlane((int)bslot, owner)];
            rd = best;
            rj = (uint32_t)key;
            rx = wq.x;
            ry = wq.y;
            rz = wq.z;
            return true;
        }
        if (all || R >= kShellMax) return false;
        // the next cube: large enough for the bound to pass the best found
        // (its radius in voxels, plus one), or twice as large
        done_r = R;
        int next = 2 * R + 1;
        if (found) next = (int)fminf((float)kShellMax, ceilf(sqrtf(best) * inv) + 1.0f);
        R = max(R + 1, min(next, kShellMax));
    }
}

// LPQ lanes cooperate on one query: each scans every LPQ-th candidate of the
// segment in ascending order (so it keeps the lowest index among its equal
// distances), then the lanes combine by the lexicographic minimum of
// (distance, index) -- the same result as one lane scanning everything, with
// LPQ times more waves in flight to hide the load latency.
//
// kMom (registration): instead of writing each correspondence, each wave
// adds the float64 moments of Eq. 1 over its locally resolved queries (sum p,
// sum q, sum p q^T, sum |p|^2, sum |q|^2 about the grid centre, sum d, count)
// in a fixed lane order and writes one record, with its counters
// (candidates scanned, dilated lookups, queries sent to the global search).
// Records are wave-major: wave w of job b is record r = b * (BS / 64) + w,
// entry j at [r * kMoments + j], counter k at [r * 3 + k].  Queries sent to
// the global search add their moments later, once resolved.  Launch blocks
// are mapped to jobs XCD by XCD (xcd_job).
//
// kDirect: VANICP's monolithic layout (the comparator).  Voxel g's
// candidates are the records of its own fixed block, at g * cap, and its
// count word dcnt[g] (the root's count with the mask bit for a dilated
// voxel); a count above cap means an overflowed block and sends the query to
// the global search.  Records are in the order the voxelisation's atomics
// gave them, so ties compare indices.
//
// kMode 1 (registration over segments, for many candidates per query): each
// lane keeps the best distance and segment position only, and the winner's
// record is read once after the lanes combine (one more dependent load per
// query, three fewer selects per candidate).
//
// kOne (a single pair of one_m source points): a block's first query is its
// job index times the queries per block, so the query's load waits on no
// table, and the pair record, the pose and the query load go out together
// (with a table the chain is table -> pair record -> query).
//
// In registration nn_idx / nn_d2 are optional (null when not asked for): the
// correspondence and squared distance of each query resolved here (locally,
// or by the voxel shells of its global search) are written there too; the
// solve writes those of the exhaustively searched ones.
template <int BS, int LPQ, bool kSorted, bool kMom, bool kDirect, int kMode, bool kOne>
__global__ __launch_bounds__(BS) void k_nns_local(const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                                                  const float* __restrict__ px, const float* __restrict__ py,
                                                  const float* __restrict__ pz, const float4* __restrict__ ps4,
                                                  const PairState* __restrict__ st, const uint2* __restrict__ dir,
                                                  const float4* __restrict__ qs4, const float4* __restrict__ qsg,
                                                  int32_t* __restrict__ nn_idx, float* __restrict__ nn_d2,
                                                  int32_t* __restrict__ fb_count, int32_t* __restrict__ fb_miss,
                                                  uint32_t* __restrict__ fb_list,
                                                  unsigned long long* __restrict__ fb_key,
                                                  unsigned long long* __restrict__ ctr, double* __restrict__ part,
                                                  int all_global, const uint32_t* __restrict__ dcnt, uint32_t cap,
                                                  int64_t one_m)
{
    static_assert(LPQ == 1 || LPQ == 2 || LPQ == 4 || LPQ == 8, "lanes per query");
    constexpr bool kReload = kMode == 1;
    static_assert(kMode == 0 || kMode == 1, "search mode");
    static_assert(!kReload || (kMom && !kDirect), "position tracking needs index-ordered segments");
    constexpr int kWaves = BS / kWave;
    // A batched registration gives each XCD one contiguous eighth of the
    // jobs, whole pairs, so that an L2 holds its pairs' directories and
    // segments (the 64-pair batch: 3.66 against 4.2 ms).  A single pair, and
    // the correspondence form, whose pairs' global searches can crowd into
    // one eighth, keep the rotating chunks.
    const int jb = (kMom && !kOne) ? xcd_slab((int)blockIdx.x, (int)gridDim.x)
                                   : xcd_job((int)blockIdx.x, (int)gridDim.x);
    const BlockJob job = kOne ? BlockJob{0, jb * (BS / LPQ)} : jobs[jb];
    const PairDev& P = pd[job.pair];
    const PairState& S = st[job.pair];
    const int sub = threadIdx.x % LPQ;
    const int64_t t = (int64_t)job.start + threadIdx.x / LPQ;
    const bool inrange = t < (kOne ? one_m : P.m);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t c = 0, i = 0;
    int64_t cs = 0;
    float x = 0.0f, y = 0.0f, z = 0.0f;
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    bool dil = false;
    // The query's load goes out unconditionally (a lane past the end reads
    // the block's first query, which exists) and does not wait for the
    // pair's done flag, so the two latencies overlap.  A finished pair's
    // block runs with no active lane: it searches nothing and appends
    // nothing, and its partials are never read (the fold and the solve skip
    // finished pairs).  An early return would let the compiler sink the load
    // below the flag's test.
    {
        const int64_t tl = (kOne ? (int64_t)0 : P.p_base) + (inrange ? t : (int64_t)job.start);
        if (kSorted) {
            const float4 pp = ps4[tl];
            x = pp.x;
            y = pp.y;
            z = pp.z;
            i = __float_as_uint(pp.w);
        } else {
            x = px[tl];
            y = py[tl];
            z = pz[tl];
            i = (uint32_t)(tl - (kOne ? (int64_t)0 : P.p_base));
        }
    }
    const bool active = inrange && S.done == 0;
    if (active) {
        transform(S.Rtf, x, y, z, sx, sy, sz);
        uint32_t v;
        // all_global: every query takes the exact global search (the
        // exhaustive-NNS comparator)
        if (!all_global && voxel_of(P, sx, sy, sz, v)) {
            if (kDirect) {
                const uint32_t e = dcnt[P.v_base + v];
                const uint32_t cn = e & ~kMask;
                c = cn <= cap ? cn : 0u;
                cs = (P.v_base + (int64_t)v) * (int64_t)cap;
                dil = (e & kMask) != 0u && c != 0u;
            } else {
                const uint2 e = dir[P.v_base + v];
                c = e.y & ~kMask;
                cs = e.x;
                dil = (e.y & kMask) != 0u;
            }
        }
    }
    const int64_t gp = (kOne ? (int64_t)0 : P.p_base) + i;
    // queries for the global search (counted on their first lane)
    const bool miss = active && c == 0 && sub == 0;
    const unsigned long long mmask = __ballot(miss);
    float bd = INFINITY;
    uint32_t bj = 0xFFFFFFFFu;
    float bx = 0.0f, by = 0.0f, bz = 0.0f;
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
            for (int u = 0; u < U; ++u) {
                if (kReload) consider_pos(a[u], min(k + (uint32_t)(u * LPQ), last), sx, sy, sz, bd, bj);
                else if (kMom) consider<kDirect>(a[u], sx, sy, sz, bd, bj, bx, by, bz);
                else consider<kDirect>(a[u], sx, sy, sz, bd, bj);
            }
        }
    }
    if (LPQ > 1) {
#pragma unroll
        for (int d = 1; d < LPQ; d <<= 1) {
            const float od = xor_lanes(bd, d);
            const uint32_t oj = xor_lanes(bj, d);
            float ox = 0.0f, oy = 0.0f, oz = 0.0f;
            if (kMom && !kReload) {
                ox = xor_lanes(bx, d);
                oy = xor_lanes(by, d);
                oz = xor_lanes(bz, d);
            }
            const bool take = od < bd || (od == bd && oj < bj);
            bd = take ? od : bd;
            bj = take ? oj : bj;
            if (kMom && !kReload) {
                bx = take ? ox : bx;
                by = take ? oy : by;
                bz = take ? oz : bz;
            }
        }
    }
    uint32_t bidx = bj;   // the winner's target index
    if (kReload && active && c > 0 && sub == 0) {
        const float4 wv = qs4[cs + min(bj, c - 1u)];   // bj < c: every distance is finite inside a grid
        bx = wv.x;
        by = wv.y;
        bz = wv.z;
        bidx = __float_as_uint(wv.w);
    }
    // The wave resolves its global searches itself, one query at a time, by
    // the exact shell search over the segments (qsg, whichever layout the
    // local search reads; not for the exhaustive comparator); those the
    // shells do not settle are appended to the pair's list for the
    // exhaustive search, one append per wave, each query at its rank among
    // the wave's unresolved ones.  Every global search is counted in
    // fb_miss.
    bool shelled = false;
    unsigned long long left = mmask;
    if (mmask && !all_global) {
        unsigned long long pend = mmask;
        left = 0ull;
        while (pend) {   // uniform over the wave
            const int L = __ffsll((long long)pend) - 1;
            pend &= pend - 1ull;
            float rd, rx, ry, rz;
            uint32_t rj;
            const float lx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sx), L));
            const float ly = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sy), L));
            const float lz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sz), L));
            if (shell_nearest<kMom ? kShellBatch : kShellBatchNN, kMom ? kShellLoads : kShellLoadsNN,
                              kMom ? kShellFirst : kShellFirstNN>(P, dir, qsg, lx, ly, lz, rd, rj, rx, ry, rz)) {
                if (lane == L) {
                    shelled = true;
                    bd = rd;
                    bidx = rj;
                    bx = rx;
                    by = ry;
                    bz = rz;
                }
            } else {
                left |= 1ull << L;
            }
        }
    }
    if (mmask) {
        const int leader = __ffsll((long long)mmask) - 1;
        int32_t base = 0;
        if (lane == leader) {
            if (fb_miss) atomicAdd(&fb_miss[job.pair], (int32_t)__popcll(mmask));
            if (left) base = atomicAdd(&fb_count[job.pair], (int32_t)__popcll(left));
        }
        base = __shfl(base, leader, kWave);
        if ((left >> lane) & 1ull) {
            const int32_t pos = base + (int32_t)__popcll(left & ((1ull << lane) - 1ull));
            fb_list[P.p_base + pos] = i;
            fb_key[P.p_base + pos] = ~0ull;
            if (!kMom) nn_idx[gp] = -1 - pos;
        }
    }
    const bool found = (active && c > 0 && sub == 0) || shelled;
    if (found && (!kMom || nn_idx)) {
        nn_idx[gp] = (int32_t)bidx;
        nn_d2[gp] = bd;
    }
    if (!kMom) return;
    // Registration: one record per wave, the float64 moments of Eq. 1 over
    // the wave's locally resolved queries about the grid centre (sum p,
    // sum q, sum p q^T, sum |p|^2, sum |q|^2, sum d, count) and three exact
    // counters (candidates scanned, dilated lookups, queries sent to the
    // global search), reduced inside the wave in a fixed order.  No block
    // barrier: the waves of a block finish independently.  Each query's
    // first lane stores its 18 values as one row of the wave's LDS rows
    // (kStride odd words, so neither the row stores nor the column reads
    // fall on one bank); then three lanes per entry each add an interleaved
    // slice of the rows in order, and one lane per entry adds the three
    // slices in order.  A wave's LDS accesses execute in order, so a wave
    // barrier (no instruction, it only keeps the compiler from moving LDS
    // accesses across it) is all the rows need between store and read.
    constexpr int kQw = kWave / LPQ;   // queries per wave
    constexpr int kSums = kMoments - 1;
    constexpr int kStride = kSums | 1;
    constexpr int kSl = 3;             // slices per entry
    static_assert(kSums * kSl <= kWave, "slice layout");
    __shared__ double mq[kWaves][kQw * kStride];
    __shared__ double ms[kWaves][kSums * kSl];
    const int64_t rec = (int64_t)jb * kWaves + w;
    const uint32_t ndil = (uint32_t)__popcll(__ballot(dil && sub == 0));
    const uint32_t nfound = (uint32_t)__popcll(__ballot(found));
    const uint32_t cw = row_sum_u32<LPQ>((sub == 0) ? c : 0u);   // each 16-lane row's total in its lane 16 - LPQ
    const uint32_t ncand = (uint32_t)__builtin_amdgcn_readlane((int)cw, 16 - LPQ) +
                           (uint32_t)__builtin_amdgcn_readlane((int)cw, 32 - LPQ) +
                           (uint32_t)__builtin_amdgcn_readlane((int)cw, 48 - LPQ) +
                           (uint32_t)__builtin_amdgcn_readlane((int)cw, 64 - LPQ);
    {
        const double c0 = P.cx, c1 = P.cy, c2 = P.cz;
        const double p[3] = {found ? (double)x - c0 : 0.0, found ? (double)y - c1 : 0.0,
                             found ? (double)z - c2 : 0.0};
        const double q[3] = {found ? (double)bx - c0 : 0.0, found ? (double)by - c1 : 0.0,
                             found ? (double)bz - c2 : 0.0};
        if (sub == 0) {
            double* rowp = mq[w] + (lane / LPQ) * kStride;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                rowp[r] = p[r];
                rowp[3 + r] = q[r];
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) rowp[6 + 3 * r + cc] = p[r] * q[cc];
            }
            rowp[15] = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
            rowp[16] = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
            rowp[17] = found ? (double)bd : 0.0;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < kSums * kSl) {
        const int j = lane / kSl, sl = lane % kSl;
        double sm = 0.0;
#pragma unroll
        for (int e = 0; e < (kQw + kSl - 1) / kSl; ++e) {
            const int r = sl + kSl * e;
            if (r < kQw) sm += mq[w][r * kStride + j];
        }
        ms[w][j * kSl + sl] = sm;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < kSums) {
        double sm = ms[w][lane * kSl];
#pragma unroll
        for (int e = 1; e < kSl; ++e) sm += ms[w][lane * kSl + e];
        part[rec * kMoments + lane] = sm;
    } else if (lane == kSums) {
        part[rec * kMoments + kMoments - 1] = (double)nfound;
    } else if (lane >= 32 && lane < 35) {
        const int k = lane - 32;
        ctr[rec * 3 + k] = k == 0 ? (unsigned long long)ncand
                                  : (unsigned long long)(k == 1 ? ndil : (uint32_t)__popcll(mmask));
    }
}

// Global search.  Work item = (pair, chunk of kFbQ listed queries, tile of
// kFbT targets); items are enumerated from the device-side list lengths, so
// the launch shape is fixed (graph-capturable) whatever the number of misses.
constexpr int kFbThreads = kFbQueries;
constexpr int kFbQ = kFbQueries;
constexpr int kFbT = kFbTargets;
constexpr int kMaxPairs = kFbMaxPairs;

__global__ __launch_bounds__(kFbThreads) void k_fallback(const PairDev* __restrict__ pd, int npairs,
                                                         const float* __restrict__ qx, const float* __restrict__ qy,
                                                         const float* __restrict__ qz, const float* __restrict__ px,
                                                         const float* __restrict__ py, const float* __restrict__ pz,
                                                         const PairState* __restrict__ st,
                                                         const int32_t* __restrict__ fb_count,
                                                         const uint32_t* __restrict__ fb_list,
                                                         unsigned long long* __restrict__ fb_key,
                                                         const FoldJob* __restrict__ fjobs, int nunits,
                                                         const double* __restrict__ part,
                                                         const unsigned long long* __restrict__ ctr,
                                                         double* __restrict__ fpart,
                                                         unsigned long long* __restrict__ fctr)
{
    // the per-pair running sum of work items: npairs + 1 entries of dynamic
    // LDS (a single pair needs 16 bytes, not a table for the largest batch)
    extern __shared__ int64_t s_pref[];
    __shared__ float tx[kFbT], ty[kFbT], tz[kFbT];
    // the first kFbThreads pairs' list lengths and target counts do not
    // depend on the fold: loaded before it, used after it
    const bool own0 = (int)threadIdx.x < npairs;
    const int64_t F0 = own0 ? fb_count[threadIdx.x] : 0;
    const int64_t n0 = own0 ? pd[threadIdx.x].n : 0;
    // registration: first fold the search waves' moment records, kFoldChunk
    // records per unit, each summed in record order (the launch runs anyway,
    // and the fold does not depend on the global search)
    if (fjobs) {
        // rows padded by one element: the moment rows then start in different
        // banks, so neither the transposing stores nor the row sums conflict
        __shared__ double fv[kMoments][kFoldChunk + 1];
        __shared__ unsigned long long fc[2][kFoldChunk + 1];
        __shared__ double fsl[kMoments][8 + 1];
        for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
            // a finished pair's units are folded too (their sums go unused):
            // testing its flag first would delay every load behind it
            const FoldJob fj = fjobs[u];
            const int cnt = fj.b1 - fj.b0;
            // every load in flight before the first LDS store (a load-store
            // loop waits for each load in turn)
            constexpr int kLoads = (kMoments * kFoldChunk + kFbThreads - 1) / kFbThreads;
            static_assert(3 * kFoldChunk <= kFbThreads, "one counter load per thread");
            const double* src = part + (int64_t)fj.b0 * kMoments;
            double v[kLoads];
#pragma unroll
            for (int r = 0; r < kLoads; ++r) {
                const int e = threadIdx.x + r * kFbThreads;
                v[r] = e < kMoments * cnt ? src[e] : 0.0;
            }
            const int ec = threadIdx.x;
            const unsigned long long cv = ec < 3 * cnt ? ctr[(int64_t)fj.b0 * 3 + ec] : 0ull;
#pragma unroll
            for (int r = 0; r < kLoads; ++r) {
                const int e = threadIdx.x + r * kFbThreads;
                if (e < kMoments * cnt) {
                    const int bb = e / kMoments, j = e - bb * kMoments;
                    fv[j][bb] = v[r];
                }
            }
            if (ec < 3 * cnt) {
                const int bb = ec / 3, j = ec - bb * 3;
                if (j < 2) fc[j][bb] = cv;
            }
            __syncthreads();
            // kFoldSlices threads per moment each add an interleaved slice of
            // the blocks in order, then one adds the slices in order (a fixed
            // order, eight dependent adds each instead of 64)
            constexpr int kFoldSlices = 8;
            static_assert(kMoments * kFoldSlices <= kFbThreads - 2 && kFoldChunk % kFoldSlices == 0, "fold slices");
            if (threadIdx.x < kMoments * kFoldSlices) {
                const int j = threadIdx.x / kFoldSlices, sl = threadIdx.x % kFoldSlices;
                double sm = 0.0;
#pragma unroll
                for (int e = 0; e < kFoldChunk / kFoldSlices; ++e) {
                    const int bb = sl + e * kFoldSlices;
                    sm += bb < cnt ? fv[j][bb] : 0.0;
                }
                fsl[j][sl] = sm;
            } else if (threadIdx.x >= kFbThreads - 2) {
                const int j = threadIdx.x - (kFbThreads - 2);
                unsigned long long sm = 0;
                for (int bb = 0; bb < cnt; ++bb) sm += fc[j][bb];
                fctr[(int64_t)j * nunits + u] = sm;
            }
            __syncthreads();
            if (threadIdx.x < kMoments) {
                double sm = fsl[threadIdx.x][0];
#pragma unroll
                for (int e = 1; e < kFoldSlices; ++e) sm += fsl[threadIdx.x][e];
                fpart[(int64_t)threadIdx.x * nunits + u] = sm;
            }
        }
    }
    // items per pair (64-bit), loaded in parallel, then an in-LDS running sum
    for (int p = threadIdx.x; p < npairs; p += kFbThreads) {
        const bool first = p == (int)threadIdx.x;
        const int64_t F = first ? F0 : fb_count[p];
        const int64_t n = first ? n0 : pd[p].n;
        s_pref[p + 1] = fallback_items(F, n);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        s_pref[0] = 0;
        for (int p = 1; p <= npairs; ++p) {
            acc += s_pref[p];
            s_pref[p] = acc;
        }
    }
    __syncthreads();
    const int64_t total = s_pref[npairs];
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        int lo = 0, hi = npairs;   // last p with s_pref[p] <= item
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_pref[mid] <= item) lo = mid;
            else hi = mid;
        }
        const int p = lo;
        const PairDev& P = pd[p];
        const int64_t local = item - s_pref[p];
        const int64_t ntile = (P.n + kFbT - 1) / kFbT;
        const int64_t qc = local / ntile, tile = local % ntile;
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
        const int64_t slot = qc * kFbQ + threadIdx.x;
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

void launch_nns_local(const PairDev* pd, const BlockJob* jobs, int njobs, int block, int lpq, bool sorted, bool mom,
                      const float* px, const float* py, const float* pz, const float4* ps4, const PairState* st,
                      const uint2* dir, const float4* qs4, const float4* qsg, int32_t* nn_idx, float* nn_d2,
                      int32_t* fb_count, int32_t* fb_miss, uint32_t* fb_list, unsigned long long* fb_key, unsigned long long* ctr,
                      double* part, int all_global, const uint32_t* dcnt, uint32_t cap, int mode, int64_t one_m,
                      hipStream_t s)
{
    if (njobs <= 0) return;
    const bool one = one_m >= 0;
    // the position-tracking form, for many candidates per query: 4 or 8
    // lanes per query, registration over segments
    if (mode == 1 && mom && !dcnt) {
#define VICP_NNS_R(BS, L, SORTED)                                                                                  \
    if (one)                                                                                                       \
        launch_timed(k_nns_local<BS, L, SORTED, true, false, 1, true>, dim3(njobs), dim3(BS), s, pd, jobs, px, py,  \
                     pz, ps4, st, dir, qs4, qsg, nn_idx, nn_d2, fb_count, fb_miss, fb_list, fb_key, ctr, part, all_global, dcnt,    \
                     cap, one_m);                                                                                  \
    else                                                                                                           \
        launch_timed(k_nns_local<BS, L, SORTED, true, false, 1, false>, dim3(njobs), dim3(BS), s, pd, jobs, px, py, \
                     pz, ps4, st, dir, qs4, qsg, nn_idx, nn_d2, fb_count, fb_miss, fb_list, fb_key, ctr, part, all_global, dcnt,    \
                     cap, one_m)
#define VICP_NNS_RL(BS, SORTED)                                     \
    switch (lpq) {                                                  \
    case 1: VICP_NNS_R(BS, 1, SORTED); break;                       \
    case 2: VICP_NNS_R(BS, 2, SORTED); break;                       \
    case 4: VICP_NNS_R(BS, 4, SORTED); break;                       \
    default: VICP_NNS_R(BS, 8, SORTED); break;                      \
    }
#define VICP_NNS_RB(SORTED)                                         \
    switch (block) {                                                \
    case 128: { VICP_NNS_RL(128, SORTED) } break;                   \
    case 512: { VICP_NNS_RL(512, SORTED) } break;                   \
    default: { VICP_NNS_RL(256, SORTED) } break;                    \
    }
        if (sorted) {
            VICP_NNS_RB(true)
        } else {
            VICP_NNS_RB(false)
        }
#undef VICP_NNS_RB
#undef VICP_NNS_RL
#undef VICP_NNS_R
        return;
    }
#define VICP_NNS(BS, L, SORTED, MOM, DIRECT)                                                                       \
    if (one && !DIRECT)                                                                                            \
        launch_timed(k_nns_local<BS, L, SORTED, MOM, DIRECT, 0, true>, dim3(njobs), dim3(BS), s, pd, jobs, px, py,  \
                     pz, ps4, st, dir, qs4, qsg, nn_idx, nn_d2, fb_count, fb_miss, fb_list, fb_key, ctr, part, all_global, dcnt,    \
                     cap, one_m);                                                                                  \
    else                                                                                                           \
        launch_timed(k_nns_local<BS, L, SORTED, MOM, DIRECT, 0, false>, dim3(njobs), dim3(BS), s, pd, jobs, px, py, \
                     pz, ps4, st, dir, qs4, qsg, nn_idx, nn_d2, fb_count, fb_miss, fb_list, fb_key, ctr, part, all_global, dcnt,    \
                     cap, one_m)
#define VICP_NNS_L(BS, SORTED, MOM, DIRECT)                  \
    switch (lpq) {                                           \
    case 2: VICP_NNS(BS, 2, SORTED, MOM, DIRECT); break;     \
    case 4: VICP_NNS(BS, 4, SORTED, MOM, DIRECT); break;     \
    case 8: VICP_NNS(BS, 8, SORTED, MOM, DIRECT); break;     \
    default: VICP_NNS(BS, 1, SORTED, MOM, DIRECT); break;    \
    }
#define VICP_NNS_BS(SORTED, MOM, DIRECT)                     \
    switch (block) {                                         \
    case 128: VICP_NNS_L(128, SORTED, MOM, DIRECT); break;   \
    case 512: VICP_NNS_L(512, SORTED, MOM, DIRECT); break;   \
    default: VICP_NNS_L(256, SORTED, MOM, DIRECT); break;    \
    }
    // the direct layout serves registrations only
    if (dcnt && mom) {
        if (sorted) {
            VICP_NNS_BS(true, true, true)
        } else {
            VICP_NNS_BS(false, true, true)
        }
    } else if (mom) {
        if (sorted) {
            VICP_NNS_BS(true, true, false)
        } else {
            VICP_NNS_BS(false, true, false)
        }
    } else {
        if (sorted) {
            VICP_NNS_BS(true, false, false)
        } else {
            VICP_NNS_BS(false, false, false)
        }
    }
#undef VICP_NNS_BS
#undef VICP_NNS_L
#undef VICP_NNS
}

bool launch_fallback(const PairDev* pd, int npairs, int grid, const float* qx, const float* qy, const float* qz,
                     const float* px, const float* py, const float* pz, const PairState* st, const int32_t* fb_count,
                     const uint32_t* fb_list, unsigned long long* fb_key, const FoldJob* fjobs, int nunits,
                     const double* part, const unsigned long long* ctr, double* fpart,
                     unsigned long long* fctr, hipStream_t s)
{
    if (npairs <= 0 || npairs > kMaxPairs || grid <= 0) return false;
    launch_timed_lds(k_fallback, dim3(grid), dim3(kFbThreads), sizeof(int64_t) * (npairs + 1), s, pd, npairs, qx, qy,
                     qz, px, py, pz, st, fb_count, fb_list, fb_key, fjobs, nunits, part, ctr, fpart, fctr);
    return true;
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
