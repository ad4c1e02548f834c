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
// TX x TY x TZ voxels plus an L-voxel halo (the loaded region, EX x EY x EZ),
// runs the L synchronous rings there (ring r is exact on the region shrunk by
// r, which contains every voxel it needs from ring r - 1), and writes the
// last ring's result for its tile.  Voxels outside the grid stay "none" and
// are never dilated, as in the per-ring form (only in-bounds neighbours
// count).
//
// The halo is loaded as search-directory entries (start of the voxel's points,
// count), which the offset scan wrote for every voxel: the count tells an
// occupied voxel, the start gives a voxel's segment offset back
// (off[g] = start + 2g), and a root, which always lies inside the loaded
// region, has its entry in LDS already, so no load waits on the rings.  The
// ring state is the root's position in the loaded region (element index
// e = (ez EY + ey) EX + ex), whose order is the order of the voxel ids inside
// the grid (both are z-major, then y, then x), so the lowest-id rule is
// unchanged.  Entries of voxels that another block dilates while this one
// loads them carry the mask bit and read as empty, as the count word 0 they
// replace does.
//
// Each thread owns whole columns (all EZ elements of one (ex, ey)): the
// column's coordinates and bounds are worked out once, its states live in
// registers (its z neighbours are its own previous values), and only the
// four x / y neighbours of each element come from LDS.
template <int R, int TX, int TY, int TZ>
__global__ __launch_bounds__(256) void k_dilate_fused(const PairDev* __restrict__ pd, const BlockJob* __restrict__ jobs,
                                                      uint32_t* __restrict__ vm, uint2* __restrict__ dir)
{
    constexpr int BS = 256;
    constexpr int EX = TX + 2 * R, EY = TY + 2 * R, EZ = TZ + 2 * R;
    constexpr int NC = EX * EY, NE = NC * EZ;
    constexpr int CPT = (NC + BS - 1) / BS;   // columns per thread
    static_assert(NE < 0xFFFF, "element indices fit 16 bits");
    constexpr uint32_t kNone32 = 0xFFFFu;
    __shared__ uint2 dl[NE];
    __shared__ uint16_t sb[2][NE];
    // tiles of one slab of the grid per XCD: the halos neighbouring tiles
    // share then sit in the same L2
    const BlockJob job = jobs[xcd_slab((int)blockIdx.x, (int)gridDim.x)];
    const PairDev& P = pd[job.pair];
    const int Dx = P.Dx, Dy = P.Dy, Dz = P.Dz;
    const int ntx = (Dx + TX - 1) / TX, nty = (Dy + TY - 1) / TY;
    const int tile = job.start;
    const int bx = (tile % ntx) * TX, by = ((tile / ntx) % nty) * TY, bz = (tile / (ntx * nty)) * TZ;
    const int64_t vb = P.v_base;
    const uint32_t plane = (uint32_t)Dx * (uint32_t)Dy;
    int col[CPT], dxy[CPT];
    uint32_t st[CPT][EZ];
    // every entry load of the thread's columns in flight before the first
    // LDS store (a load-store loop waits for each load in turn)
    {
        uint2 ev[CPT][EZ];
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = threadIdx.x + BS * k;
            col[k] = c;
            const int ex = c % EX, ey = c / EX;
            const int x = bx - R + ex, y = by - R + ey;
            const bool inxy = c < NC && x >= 0 && x < Dx && y >= 0 && y < Dy;
            // depth of the column inside the loaded region (-1: no column)
            dxy[k] = inxy ? min(min(ex, EX - 1 - ex), min(ey, EY - 1 - ey)) : -1;
            const uint32_t uxy = inxy ? (uint32_t)x + (uint32_t)Dx * (uint32_t)y : 0u;
#pragma unroll
            for (int ez = 0; ez < EZ; ++ez) {
                const int z = bz - R + ez;
                const bool ok = inxy && z >= 0 && z < Dz;
                // unconditional (voxel 0 exists): no branch to wait at
                ev[k][ez] = dir[vb + (ok ? uxy + plane * (uint32_t)z : 0u)];
                const bool occ = ok && ev[k][ez].y != 0u && (ev[k][ez].y & kMask) == 0u;
                st[k][ez] = occ ? (uint32_t)(ez * NC + c) : kNone32;
            }
        }
#pragma unroll
        for (int k = 0; k < CPT; ++k)
            if (col[k] < NC) {
#pragma unroll
                for (int ez = 0; ez < EZ; ++ez) {
                    dl[ez * NC + col[k]] = ev[k][ez];
                    sb[0][ez * NC + col[k]] = (uint16_t)st[k][ez];
                }
            }
    }
    __syncthreads();
#pragma unroll
    for (int r = 1; r <= R; ++r) {
        const uint16_t* cur = sb[(r - 1) & 1];
        uint16_t* nxt = sb[r & 1];
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = col[k];
            const int ca = c < NC ? c : NC - 1;   // a thread without this column reads a real one, unused
            const bool live = dxy[k] >= r;        // the column lies r deep in the region
            uint32_t old[EZ];
#pragma unroll
            for (int ez = 0; ez < EZ; ++ez) old[ez] = st[k][ez];
            // selects, not branches: every element of the ring reads its four
            // x / y neighbours, which keeps the waves free of divergent paths
#pragma unroll
            for (int ez = r; ez < EZ - r; ++ez) {
                const int e = ez * NC + ca;
                uint32_t v = min(old[ez - 1], old[ez + 1]);
                v = min(v, (uint32_t)min(cur[e - 1], cur[e + 1]));
                v = min(v, (uint32_t)min(cur[e - EX], cur[e + EX]));
                st[k][ez] = (live && old[ez] == kNone32) ? v : old[ez];
            }
            if (r < R && c < NC) {
#pragma unroll
                for (int ez = 0; ez < EZ; ++ez) nxt[ez * NC + c] = (uint16_t)st[k][ez];
            }
        }
        if (r < R) __syncthreads();
    }
    // the tile's columns write their voxels' results
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int c = col[k];
        const int ex = c % EX, ey = c / EX;
        if (c >= NC || ex < R || ex >= R + TX || ey < R || ey >= R + TY) continue;
        const int x = bx - R + ex, y = by - R + ey;
        if (x >= Dx || y >= Dy) continue;
#pragma unroll
        for (int ez = R; ez < R + TZ; ++ez) {
            const int z = bz - R + ez;
            if (z >= Dz) continue;
            const uint32_t self = (uint32_t)(ez * NC + c);
            const uint32_t root = st[k][ez];
            // an occupied voxel keeps its own element as its state: any other
            // root marks an empty voxel that the rings reached
            if (root == kNone32 || root == self) continue;
            const uint2 own = dl[self], re = dl[root];
            // an entry with the mask bit was dilated by an earlier run of the
            // same rings (the autotuner re-runs the dilation): its words are
            // final, and its start is the root's, not the voxel's own
            if (own.y & kMask) continue;
            const int rc = (int)(root % NC), rz = (int)(root / NC);
            const uint32_t ru = (uint32_t)(bx - R + rc % EX) + (uint32_t)Dx * (uint32_t)(by - R + rc / EX) +
                                plane * (uint32_t)(bz - R + rz);
            const int64_t g = vb + (int64_t)((uint32_t)x + (uint32_t)Dx * (uint32_t)y + plane * (uint32_t)z);
            vm[(int64_t)(uint32_t)(own.x + 2u * (uint32_t)g) + 1] = ru | kMask;
            dir[g] = make_uint2(re.x, re.y | kMask);
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
    case 0: launch_timed(k_dilate_fused<R, 8, 8, 4>, dim3(njobs), dim3(256), s, pd, jobs, vm, dir); return true;
    case 1: launch_timed(k_dilate_fused<R, 16, 8, 4>, dim3(njobs), dim3(256), s, pd, jobs, vm, dir); return true;
    case 2: launch_timed(k_dilate_fused<R, 8, 8, 8>, dim3(njobs), dim3(256), s, pd, jobs, vm, dir); return true;
    case 3: launch_timed(k_dilate_fused<R, 32, 8, 4>, dim3(njobs), dim3(256), s, pd, jobs, vm, dir); return true;
    case 4: launch_timed(k_dilate_fused<R, 16, 16, 4>, dim3(njobs), dim3(256), s, pd, jobs, vm, dir); return true;
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
