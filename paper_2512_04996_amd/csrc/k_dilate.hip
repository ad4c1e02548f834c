// k_dilate.hip -- voxel dilation (Alg. 3) under offset addressing.
//
// Ring r of a synchronous schedule: an empty voxel takes the lowest root id
// among its six in-bounds face neighbours' roots after ring r-1 (pull form,
// no atomics, no locks).  After the last ring every empty voxel that has a
// root gets Mask(root) in the count word of its segment, found through the
// offsets.  The ring state lives in a compact V-word array (root or none).
// The same pass points the voxel's search-directory entry at its root's
// points (start and count, with the mask bit set in the count).  Up to
// kFusedRings rings run in one launch on LDS tiles (k_dilate_fused), more
// ring by ring (k_dilate_ring); both give the same result.
#include "vicp_internal.hpp"

namespace vicp {

namespace {

// A job is kRingItems consecutive voxels of one pair; BS threads cover it.
constexpr int kRingItems = 256;

template <int BS>
__global__ __launch_bounds__(BS) void k_dilate_ring(const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                                                    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ off,
                                                    uint32_t* __restrict__ vm, uint2* __restrict__ dir,
                                                    const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                                    int first, int last)
{
    static_assert(kRingItems % BS == 0, "whole rounds");
    const BlockJob job = jobs[blockIdx.x];
    const PairDev& P = pd[job.pair];
    const int64_t vb = P.v_base;
    auto state = [&](uint32_t u) -> uint32_t {
        const int64_t gu = vb + u;
        return first ? (hist[gu] ? u : kNone) : src[gu];
    };
    for (int k = threadIdx.x; k < kRingItems; k += BS) {
        const int64_t vi = (int64_t)job.start + k;
        if (vi >= P.V) return;
        const uint32_t v = (uint32_t)vi;
        const int64_t g = vb + v;
        uint32_t cur = state(v);
        if (cur == kNone) {
            const uint32_t Dx = (uint32_t)P.Dx, Dy = (uint32_t)P.Dy, Dz = (uint32_t)P.Dz;
            const uint32_t x = v % Dx, yz = v / Dx;
            const uint32_t y = yz % Dy, z = yz / Dy;
            const uint32_t sxy = Dx * Dy;
            if (x > 0) cur = min(cur, state(v - 1));
            if (x + 1 < Dx) cur = min(cur, state(v + 1));
            if (y > 0) cur = min(cur, state(v - Dx));
            if (y + 1 < Dy) cur = min(cur, state(v + Dx));
            if (z > 0) cur = min(cur, state(v - sxy));
            if (z + 1 < Dz) cur = min(cur, state(v + sxy));
        }
        if (!last) {
            dst[g] = cur;
        } else if (cur != kNone && hist[g] == 0) {
            vm[(int64_t)off[g] + 1] = cur | kMask;
            const int64_t gr = vb + cur;
            dir[g] = make_uint2(off[gr] - 2u * (uint32_t)gr, hist[gr] | kMask);
        }
    }
}

// All L rings in one launch (L <= kFusedRings): each block takes a tile of
// TX x TY x TZ voxels plus an L-voxel halo into LDS, runs the L synchronous
// rings there (ring r is exact on the region shrunk by r, which contains every
// voxel it needs from ring r - 1), and writes the last ring's result for its
// tile.  Voxels outside the grid stay "none" and are never dilated, as in the
// per-ring form (only in-bounds neighbours count).
//
// The halo is loaded as search-directory entries (start of the voxel's points,
// count), which the offset scan wrote for every voxel: the count tells an
// occupied voxel, the start gives a voxel's segment offset back
// (off[g] = start + 2g), and a root, which always lies inside the loaded
// region, has its entry in LDS already, so no load waits on the rings.  The
// ring state is the root's position in the loaded region (LDS element
// index), whose order is the order of the voxel ids inside the grid (both
// are z-major, then y, then x), so the lowest-id rule is unchanged.  Entries
// of voxels that another block dilates while this one loads them carry the
// mask bit and read as empty, as the count word 0 they replace does.
template <int R, int TX, int TY, int TZ>
__global__ __launch_bounds__(256) void k_dilate_fused(const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                                                      uint32_t* __restrict__ vm, uint2* __restrict__ dir)
{
    constexpr int BS = 256;
    constexpr int EX = TX + 2 * R, EY = TY + 2 * R, EZ = TZ + 2 * R, NE = EX * EY * EZ;
    static_assert(NE < 0xFFFF, "element indices fit 16 bits");
    constexpr uint16_t kNone16 = 0xFFFF;
    __shared__ uint2 dl[NE];
    __shared__ uint16_t s0[NE], s1[NE];
    const BlockJob job = jobs[blockIdx.x];
    const PairDev& P = pd[job.pair];
    const int Dx = P.Dx, Dy = P.Dy, Dz = P.Dz;
    const int ntx = (Dx + TX - 1) / TX, nty = (Dy + TY - 1) / TY;
    const int tile = job.start;
    const int bx = (tile % ntx) * TX, by = ((tile / ntx) % nty) * TY, bz = (tile / (ntx * nty)) * TZ;
    const int64_t vb = P.v_base;
    auto inside = [&](int x, int y, int z) { return x >= 0 && x < Dx && y >= 0 && y < Dy && z >= 0 && z < Dz; };
    // every entry load in flight before the first LDS store (a load-store
    // loop waits for each load in turn); each element also keeps its depth
    // inside the loaded region (-1 outside the grid), so that a ring's test
    // is one compare: ring r updates the elements of depth >= r
    constexpr int kLoads = (NE + BS - 1) / BS;
    uint2 ev[kLoads];
    int lv[kLoads];
#pragma unroll
    for (int l = 0; l < kLoads; ++l) {
        const int e = threadIdx.x + BS * l;
        const int ex = e % EX, ey = (e / EX) % EY, ez = e / (EX * EY);
        const int x = bx - R + ex, y = by - R + ey, z = bz - R + ez;
        const bool ok = e < NE && inside(x, y, z);
        const uint32_t u = ok ? (uint32_t)x + (uint32_t)Dx * ((uint32_t)y + (uint32_t)Dy * (uint32_t)z) : 0u;
        ev[l] = dir[vb + u];   // unconditional (voxel 0 exists): no branch to wait at
        lv[l] = ok ? min(min(min(ex, EX - 1 - ex), min(ey, EY - 1 - ey)), min(ez, EZ - 1 - ez)) : -1;
    }
#pragma unroll
    for (int l = 0; l < kLoads; ++l) {
        const int e = threadIdx.x + BS * l;
        if (e < NE) {
            const bool occ = lv[l] >= 0 && ev[l].y != 0u && (ev[l].y & kMask) == 0u;
            dl[e] = ev[l];
            s0[e] = occ ? (uint16_t)e : kNone16;
        }
    }
    __syncthreads();
    uint16_t* cur = s0;
    uint16_t* nxt = s1;
#pragma unroll
    for (int r = 1; r <= R; ++r) {
#pragma unroll
        for (int l = 0; l < kLoads; ++l) {
            const int e = threadIdx.x + BS * l;
            if (e >= NE) continue;
            uint16_t v = cur[e];
            if (v == kNone16 && lv[l] >= r) {
                v = min(v, min(cur[e - 1], cur[e + 1]));
                v = min(v, min(cur[e - EX], cur[e + EX]));
                v = min(v, min(cur[e - EX * EY], cur[e + EX * EY]));
            }
            nxt[e] = v;
        }
        __syncthreads();
        uint16_t* t = cur;
        cur = nxt;
        nxt = t;
    }
    for (int e = threadIdx.x; e < TX * TY * TZ; e += BS) {
        const int ix = e % TX, iy = (e / TX) % TY, iz = e / (TX * TY);
        const int x = bx + ix, y = by + iy, z = bz + iz;
        if (!inside(x, y, z)) continue;
        const int self = (iz + R) * EX * EY + (iy + R) * EX + (ix + R);
        const uint16_t root = cur[self];
        // an occupied voxel keeps its own element as its state: any other
        // root marks an empty voxel that the rings reached
        if (root == kNone16 || root == (uint16_t)self) continue;
        const int rx = bx - R + root % EX, ry = by - R + (root / EX) % EY, rz = bz - R + root / (EX * EY);
        const uint32_t ru = (uint32_t)rx + (uint32_t)Dx * ((uint32_t)ry + (uint32_t)Dy * (uint32_t)rz);
        const uint32_t u = (uint32_t)x + (uint32_t)Dx * ((uint32_t)y + (uint32_t)Dy * (uint32_t)z);
        const int64_t g = vb + u;
        const uint2 own = dl[self], re = dl[root];
        // an entry with the mask bit was dilated by an earlier run of the same
        // rings (the autotuner re-runs the dilation): its words are final, and
        // its start is the root's, not the voxel's own
        if (own.y & kMask) continue;
        vm[(int64_t)(uint32_t)(own.x + 2u * (uint32_t)g) + 1] = ru | kMask;
        dir[g] = make_uint2(re.x, re.y | kMask);
    }
}

// VANICP's dilation writes points, not a reference: once the rings have
// run (state = own id for an occupied voxel, root id for a dilated one), the
// fixed block of every dilated voxel receives a copy of its root's records,
// and its count word the root's count with the mask bit.  A root whose block
// overflowed (count above cap) has no complete copy to give: nothing is
// copied and the count word alone tells the search to go global.  Four lanes
// per voxel, four 16-byte records each in flight.  Roots are occupied voxels
// and only empty voxels are written, so no count word is read and written by
// different lanes.
constexpr int kRepLanes = 4;
constexpr int kRepUnroll = 4;

__global__ __launch_bounds__(256) void k_replicate(const PairDev* __restrict__ pd, const uint32_t* __restrict__ state,
                                                   uint32_t* __restrict__ cnt, float4* __restrict__ blk, uint32_t cap)
{
    const PairDev& P = pd[0];
    const int64_t v = (int64_t)blockIdx.x * (256 / kRepLanes) + threadIdx.x / kRepLanes;
    if (v >= P.V) return;
    const uint32_t sub = threadIdx.x % kRepLanes;
    const uint32_t r = state[P.v_base + v];
    if (r == kNone || (int64_t)r == v) return;
    const uint32_t c = cnt[P.v_base + r];
    if (sub == 0) cnt[P.v_base + v] = c | kMask;
    if (c > cap) return;
    const float4* src = blk + (P.v_base + (int64_t)r) * cap;
    float4* dst = blk + (P.v_base + v) * cap;
    for (uint32_t k = sub; k < c; k += kRepLanes * kRepUnroll) {
        float4 a[kRepUnroll];
#pragma unroll
        for (int u = 0; u < kRepUnroll; ++u) {
            const uint32_t j = k + (uint32_t)(u * kRepLanes);
            if (j < c) a[u] = src[j];
        }
#pragma unroll
        for (int u = 0; u < kRepUnroll; ++u) {
            const uint32_t j = k + (uint32_t)(u * kRepLanes);
            if (j < c) dst[j] = a[u];
        }
    }
}

}  // namespace

// Tile shapes of the one-launch form (a schedule choice; every shape gives
// the same result).
struct TileShape {
    int x, y, z;
};
constexpr TileShape kTileShapes[kDilateShapes] = {{8, 8, 4}, {16, 8, 4}, {8, 8, 8}, {32, 8, 4}, {16, 16, 4}};

int64_t dilate_tiles(int shape, int Dx, int Dy, int Dz)
{
    const TileShape t = kTileShapes[(shape >= 0 && shape < kDilateShapes) ? shape : 0];
    return (int64_t)((Dx + t.x - 1) / t.x) * ((Dy + t.y - 1) / t.y) * ((Dz + t.z - 1) / t.z);
}

template <int R>
static bool launch_fused_r(int shape, const PairDev* pd, const BlockJob* jobs, int njobs, uint32_t* vm, uint2* dir,
                           hipStream_t s)
{
    switch (shape) {
    case 0: hipLaunchKernelGGL((k_dilate_fused<R, 8, 8, 4>), dim3(njobs), dim3(256), 0, s, pd, jobs, vm, dir); return true;
    case 1: hipLaunchKernelGGL((k_dilate_fused<R, 16, 8, 4>), dim3(njobs), dim3(256), 0, s, pd, jobs, vm, dir); return true;
    case 2: hipLaunchKernelGGL((k_dilate_fused<R, 8, 8, 8>), dim3(njobs), dim3(256), 0, s, pd, jobs, vm, dir); return true;
    case 3: hipLaunchKernelGGL((k_dilate_fused<R, 32, 8, 4>), dim3(njobs), dim3(256), 0, s, pd, jobs, vm, dir); return true;
    case 4: hipLaunchKernelGGL((k_dilate_fused<R, 16, 16, 4>), dim3(njobs), dim3(256), 0, s, pd, jobs, vm, dir); return true;
    default: return false;
    }
}

bool launch_dilate_fused(const PairDev* pd, const BlockJob* jobs, int njobs, int rings, int shape, uint32_t* vm,
                         uint2* dir, hipStream_t s)
{
    if (njobs <= 0) return true;
    switch (rings) {
    case 1: return launch_fused_r<1>(shape, pd, jobs, njobs, vm, dir, s);
    case 2: return launch_fused_r<2>(shape, pd, jobs, njobs, vm, dir, s);
    case 3: return launch_fused_r<3>(shape, pd, jobs, njobs, vm, dir, s);
    case 4: return launch_fused_r<4>(shape, pd, jobs, njobs, vm, dir, s);
    default: return false;
    }
}

void launch_replicate(const PairDev* pd, int64_t V, const uint32_t* state, uint32_t* cnt, float4* blk, uint32_t cap,
                      hipStream_t s)
{
    if (V <= 0 || !state) return;
    const int64_t blocks = (V + 256 / kRepLanes - 1) / (256 / kRepLanes);
    hipLaunchKernelGGL(k_replicate, dim3((unsigned)blocks), dim3(256), 0, s, pd, state, cnt, blk, cap);
}

void launch_dilate_ring(const PairDev* pd, const BlockJob* jobs, int njobs, int block, const uint32_t* hist,
                        const uint32_t* off, uint32_t* vm, uint2* dir, const uint32_t* src, uint32_t* dst, int first,
                        int last, hipStream_t s)
{
    if (njobs <= 0) return;
    switch (block) {
    case 64:
        hipLaunchKernelGGL(k_dilate_ring<64>, dim3(njobs), dim3(64), 0, s, pd, jobs, hist, off, vm, dir, src, dst, first, last);
        break;
    case 128:
        hipLaunchKernelGGL(k_dilate_ring<128>, dim3(njobs), dim3(128), 0, s, pd, jobs, hist, off, vm, dir, src, dst, first, last);
        break;
    default:
        hipLaunchKernelGGL(k_dilate_ring<256>, dim3(njobs), dim3(256), 0, s, pd, jobs, hist, off, vm, dir, src, dst, first, last);
        break;
    }
}

}  // namespace vicp
