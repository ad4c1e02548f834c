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

template <int BS>
__global__ __launch_bounds__(BS) void k_dilate_ring(const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                                                    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ off,
                                                    uint32_t* __restrict__ vm, uint2* __restrict__ dir,
                                                    const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                                    int first, int last)
{
    const BlockJob job = jobs[blockIdx.x];
    const PairDev& P = pd[job.pair];
    const int64_t vi = (int64_t)job.start + threadIdx.x;
    if (vi >= P.V) return;
    const uint32_t v = (uint32_t)vi;
    const int64_t vb = P.v_base;
    const int64_t g = vb + v;
    auto state = [&](uint32_t u) -> uint32_t {
        const int64_t gu = vb + u;
        return first ? (hist[gu] ? u : kNone) : src[gu];
    };
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

// All L rings in one launch (L <= kFusedRings): each block takes a tile of
// kTX x kTY x kTZ voxels plus an L-voxel halo into LDS, runs the L
// synchronous rings there (ring r is exact on the region shrunk by r, which
// contains every voxel it needs from ring r - 1), and writes the last ring's
// result for its tile.  Voxels outside the grid stay "none" and are never
// dilated, as in the per-ring form (only in-bounds neighbours count).
constexpr int kTX = 8, kTY = 8, kTZ = 4;

template <int R>
__global__ __launch_bounds__(256) void k_dilate_fused(const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                                                      const uint32_t* __restrict__ hist,
                                                      const uint32_t* __restrict__ off, uint32_t* __restrict__ vm,
                                                      uint2* __restrict__ dir)
{
    constexpr int EX = kTX + 2 * R, EY = kTY + 2 * R, EZ = kTZ + 2 * R, NE = EX * EY * EZ;
    __shared__ uint32_t s0[NE], s1[NE];
    const BlockJob job = jobs[blockIdx.x];
    const PairDev& P = pd[job.pair];
    const int Dx = P.Dx, Dy = P.Dy, Dz = P.Dz;
    const int ntx = (Dx + kTX - 1) / kTX, nty = (Dy + kTY - 1) / kTY;
    const int tile = job.start;
    const int bx = (tile % ntx) * kTX, by = ((tile / ntx) % nty) * kTY, bz = (tile / (ntx * nty)) * kTZ;
    const int64_t vb = P.v_base;
    auto inside = [&](int x, int y, int z) { return x >= 0 && x < Dx && y >= 0 && y < Dy && z >= 0 && z < Dz; };
    // every count load in flight before the first LDS store (a load-store
    // loop waits for each load in turn); each element also keeps its depth
    // inside the loaded region (-1 outside the grid), so that a ring's test
    // is one compare: ring r updates the elements of depth >= r
    constexpr int kLoads = (NE + 255) / 256;
    uint32_t hv[kLoads], uv[kLoads];
    int lv[kLoads];
#pragma unroll
    for (int l = 0; l < kLoads; ++l) {
        const int e = threadIdx.x + 256 * l;
        const int ex = e % EX, ey = (e / EX) % EY, ez = e / (EX * EY);
        const int x = bx - R + ex, y = by - R + ey, z = bz - R + ez;
        const bool ok = e < NE && inside(x, y, z);
        uv[l] = ok ? (uint32_t)x + (uint32_t)Dx * ((uint32_t)y + (uint32_t)Dy * (uint32_t)z) : kNone;
        hv[l] = hist[vb + (ok ? uv[l] : 0u)];   // unconditional (voxel 0 exists): no branch to wait at
        lv[l] = ok ? min(min(min(ex, EX - 1 - ex), min(ey, EY - 1 - ey)), min(ez, EZ - 1 - ez)) : -1;
    }
#pragma unroll
    for (int l = 0; l < kLoads; ++l) {
        const int e = threadIdx.x + 256 * l;
        if (e < NE) s0[e] = (uv[l] != kNone && hv[l] != 0u) ? uv[l] : kNone;
    }
    __syncthreads();
    uint32_t* cur = s0;
    uint32_t* nxt = s1;
#pragma unroll
    for (int r = 1; r <= R; ++r) {
#pragma unroll
        for (int l = 0; l < kLoads; ++l) {
            const int e = threadIdx.x + 256 * l;
            if (e >= NE) continue;
            uint32_t v = cur[e];
            if (v == kNone && lv[l] >= r) {
                v = min(v, min(cur[e - 1], cur[e + 1]));
                v = min(v, min(cur[e - EX], cur[e + EX]));
                v = min(v, min(cur[e - EX * EY], cur[e + EX * EY]));
            }
            nxt[e] = v;
        }
        __syncthreads();
        uint32_t* t = cur;
        cur = nxt;
        nxt = t;
    }
    for (int e = threadIdx.x; e < kTX * kTY * kTZ; e += 256) {
        const int ix = e % kTX, iy = (e / kTX) % kTY, iz = e / (kTX * kTY);
        const int x = bx + ix, y = by + iy, z = bz + iz;
        if (!inside(x, y, z)) continue;
        const uint32_t root = cur[(iz + R) * EX * EY + (iy + R) * EX + (ix + R)];
        const uint32_t u = (uint32_t)x + (uint32_t)Dx * ((uint32_t)y + (uint32_t)Dy * (uint32_t)z);
        const int64_t g = vb + u;
        // an occupied voxel keeps its own id as its state: any other root
        // marks an empty voxel that the rings reached
        if (root != kNone && root != u) {
            vm[(int64_t)off[g] + 1] = root | kMask;
            const int64_t gr = vb + root;
            dir[g] = make_uint2(off[gr] - 2u * (uint32_t)gr, hist[gr] | kMask);
        }
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

int64_t dilate_tiles(int Dx, int Dy, int Dz)
{
    return (int64_t)((Dx + kTX - 1) / kTX) * ((Dy + kTY - 1) / kTY) * ((Dz + kTZ - 1) / kTZ);
}

bool launch_dilate_fused(const PairDev* pd, const BlockJob* jobs, int njobs, int rings, const uint32_t* hist,
                         const uint32_t* off, uint32_t* vm, uint2* dir, hipStream_t s)
{
    if (njobs <= 0) return true;
    switch (rings) {
    case 1: hipLaunchKernelGGL(k_dilate_fused<1>, dim3(njobs), dim3(256), 0, s, pd, jobs, hist, off, vm, dir); return true;
    case 2: hipLaunchKernelGGL(k_dilate_fused<2>, dim3(njobs), dim3(256), 0, s, pd, jobs, hist, off, vm, dir); return true;
    case 3: hipLaunchKernelGGL(k_dilate_fused<3>, dim3(njobs), dim3(256), 0, s, pd, jobs, hist, off, vm, dir); return true;
    case 4: hipLaunchKernelGGL(k_dilate_fused<4>, dim3(njobs), dim3(256), 0, s, pd, jobs, hist, off, vm, dir); return true;
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
    case 512:
        hipLaunchKernelGGL(k_dilate_ring<512>, dim3(njobs), dim3(512), 0, s, pd, jobs, hist, off, vm, dir, src, dst, first, last);
        break;
    default:
        hipLaunchKernelGGL(k_dilate_ring<256>, dim3(njobs), dim3(256), 0, s, pd, jobs, hist, off, vm, dir, src, dst, first, last);
        break;
    }
}

}  // namespace vicp
