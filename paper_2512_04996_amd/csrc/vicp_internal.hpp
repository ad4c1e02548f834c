// vicp_internal.hpp -- device-side data layout and kernel launchers of libvicp.
//
// Layout in HBM (all pairs of a batch share each array, concatenated in pair
// order; a single-pair grid is a batch of one):
//   qx, qy, qz   caller's target points (float32 SoA)            n_total
//   hist         per-voxel count (Alg. 1 VoxelHist)               V_total
//   off          per-voxel segment offset, exclusive scan of
//                count + 2 (Alg. 1 AddrOffset), one extra entry   V_total + 1
//   vm           dilated voxel index (Alg. 2/3 VoxelMem):
//                segment [0, count | Mask(root), indices...]      n_total + 2 V_total
//   qs4          the target points in segment order as float4
//                (x, y, z, index bits): one coalesced 16-byte
//                load per candidate in the local search          n_total
// Segment v of pair p starts at off[v_base + v] (a global word offset);
// its points sit in qs4 from off[g] - 2 g (g = v_base + v), because every
// voxel before g contributes exactly two header words to off[g].
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

namespace vicp {

constexpr uint32_t kMask = 0x80000000u;   // Mask(root) of Alg. 3
constexpr uint32_t kNone = 0xFFFFFFFFu;   // no root (dilation state)
constexpr int kMoments = 19;              // about the pair's centre c: sum p (3), sum q (3), sum p q^T (9),
                                          // sum |p|^2, sum |q|^2, sum d, count
constexpr int kGradTerms = 8;                  // sum r (3), sum s x r (3), sum |r|^2 (1), count (1)
// Source bucketing: points outside the grid go to buckets of kOutChunk
// consecutive indices, and a bucket larger than kRankCap turns the pair's
// bucketing off (identity order), so that ranking a point within its bucket
// costs at most kRankCap reads.  On a coarse grid (fewer than
// kChunkGridVoxels voxels, such as the 2^N grids of the paper's setting) a
// voxel's points are further split by index into chunks of kRankCap
// (s_shift = 10), as long as the buckets stay within kChunkBuckets, so that
// dense voxels keep their queries together instead of turning bucketing off.
constexpr int kOutShift = 6;
constexpr int64_t kOutChunk = (int64_t)1 << kOutShift;
constexpr uint32_t kRankCap = 1024;
constexpr int kRankShift = 10;                   // log2(kRankCap)
constexpr int64_t kChunkGridVoxels = 65536;
constexpr int64_t kChunkBuckets = (int64_t)1 << 20;

// Index chunking of a pair's voxel buckets: bucket of (voxel v, index i) is
// v * chunks + (i >> shift).
struct SrcChunks {
    int shift;
    int64_t chunks;
};
inline SrcChunks src_chunks(int64_t V, int64_t m)
{
    SrcChunks c{62, 1};
    if (V <= 0 || V >= kChunkGridVoxels || m <= (int64_t)kRankCap) return c;
    for (int s = kRankShift; s < 62; ++s) {
        const int64_t ch = (m + ((int64_t)1 << s) - 1) >> s;
        if (V * ch <= kChunkBuckets) return SrcChunks{s, ch};
    }
    return c;
}

// One pair: where its data lives and its grid (Sec. II.A Step 1).
struct PairDev {
    int64_t q_base;   // first target point (also first qs4 slot)
    int64_t n;        // target points
    int64_t v_base;   // first voxel in hist/off
    int64_t V;        // voxels
    int64_t p_base;   // first source point
    int64_t m;        // source points
    float ox, oy, oz, inv;  // origin and 1/voxel
    float fDx, fDy, fDz;    // dims as float32, for the inside test
    float cx, cy, cz;       // centre of the grid: reference point of the moment sums
    int32_t Dx, Dy, Dz;     // dims
    int32_t pad;
    int64_t s_base;   // first source bucket: V * s_chunks voxel buckets, then ceil(m / kOutChunk) "outside" buckets
    int64_t s_chunks; // index chunks per voxel bucket (1 on fine grids)
    int32_t s_shift;  // a source point's chunk is its index >> s_shift
    int32_t s_pad;
};

// A padded grid box whose coordinates all lie within +-kCoordLimit keeps
// every float32 difference and squared distance between two points inside it
// finite (|a - b| <= 2e18 per axis, 3 (2e18)^2 = 1.2e37 < FLT_MAX), so every
// local search has a finite best distance.
constexpr float kCoordLimit = 1e18f;
inline bool grid_box_fits(const float lo[3], const float hi[3])
{
    for (int a = 0; a < 3; ++a)
        if (!(lo[a] >= -kCoordLimit && lo[a] <= kCoordLimit && hi[a] >= -kCoordLimit && hi[a] <= kCoordLimit))
            return false;
    return true;
}

// Work items of the global search for F listed queries of a pair over its n
// targets: chunks of kFbQueries queries times tiles of kFbTargets targets.
// 64-bit: F n / 2^18 passes 2^31 at about 24M points per pair.
constexpr int kFbQueries = 256;
constexpr int kFbTargets = 1024;
constexpr int kFbMaxPairs = 4096;
__host__ __device__ inline int64_t fallback_items(int64_t F, int64_t n)
{
    return F > 0 ? ((F + kFbQueries - 1) / kFbQueries) * ((n + kFbTargets - 1) / kFbTargets) : 0;
}

// A block's work: the pair it serves and its first item within the pair.
struct BlockJob {
    int32_t pair;
    int32_t start;
};

// First-level fold of the search's moment records (one per search wave): up
// to kFoldChunk consecutive records [b0, b1) of one pair.
constexpr int kFoldChunk = 64;
struct FoldJob {
    int32_t pair;
    int32_t b0, b1;
    int32_t pad;
};

// Per-pair ICP state on the device.
struct PairState {
    double Rt[12];      // float64 pose, R row-major then t
    float Rtf[12];      // the pose rounded to float32, used by the search
    double prev_rmse;
    int32_t done;       // early stop reached (or nothing to do)
    int32_t iters;
    int32_t degenerate;
    int32_t status;     // latched device faults (bit 0: non-finite source)
    int32_t rot_ok;     // Rt's rotation is a solve's result (orthogonal to rounding)
};

// Pair p's registration state at pose rt (float64, R row-major then t) for a
// source of m points, with its global-search counts and fault flags zeroed.
__device__ __forceinline__ void init_pair_state(PairState* __restrict__ st, int p, const double* rt, int64_t m,
                                                int npairs, int32_t* __restrict__ fb_count,
                                                int32_t* __restrict__ flags)
{
    fb_count[p] = 0;
    fb_count[npairs + p] = 0;
    flags[p] = 0;
    PairState& S = st[p];
    S.done = m > 0 ? 0 : 1;
    for (int j = 0; j < 12; ++j) {
        S.Rt[j] = rt[j];
        S.Rtf[j] = (float)rt[j];
    }
    S.prev_rmse = 0.0;
    S.iters = 0;
    S.degenerate = 0;
    S.status = 0;
    S.rot_ok = 0;   // a caller's rotation: the first solve checks it
}

// The pose applied to a source point: s = R p + t (R row-major, then t).
__device__ __forceinline__ void transform(const float* __restrict__ R, float x, float y, float z, float& sx, float& sy,
                                          float& sz)
{
    sx = __builtin_fmaf(R[0], x, __builtin_fmaf(R[1], y, __builtin_fmaf(R[2], z, R[9])));
    sy = __builtin_fmaf(R[3], x, __builtin_fmaf(R[4], y, __builtin_fmaf(R[5], z, R[10])));
    sz = __builtin_fmaf(R[6], x, __builtin_fmaf(R[7], y, __builtin_fmaf(R[8], z, R[11])));
}

// Voxel of a transformed point, or false when it is outside the grid.
__device__ __forceinline__ bool voxel_of(const PairDev& P, float sx, float sy, float sz, uint32_t& v)
{
    const float fx = (sx - P.ox) * P.inv;
    const float fy = (sy - P.oy) * P.inv;
    const float fz = (sz - P.oz) * P.inv;
    // non-short-circuit: no branch waits on each bound's load in turn
    const bool in = (fx >= 0.0f) & (fx < P.fDx) & (fy >= 0.0f) & (fy < P.fDy) & (fz >= 0.0f) & (fz < P.fDz);
    if (in) v = (uint32_t)floorf(fx) + (uint32_t)P.Dx * ((uint32_t)floorf(fy) + (uint32_t)P.Dy * (uint32_t)floorf(fz));
    return in;
}


// --------------------------------------------------------------------------
// XCD-aware block order.  Workgroups are dealt to the 8 XCDs round-robin
// (block b runs on XCD b mod 8), and each XCD has its own L2.  xcd_job maps
// the launch index to a job index so that each XCD receives chunks of
// kXcdChunk consecutive jobs (jobs touching the same data, such as
// neighbouring queries of the bucketed source, then share one L2), while the
// chunks still rotate over the XCDs (a dense region does not land on one
// XCD).  A bijection on [0, n); the ragged tail keeps its order.
// --------------------------------------------------------------------------
constexpr int kXcds = 8;
#ifndef VICP_XCD_CHUNK
#define VICP_XCD_CHUNK 16
#endif
constexpr int kXcdChunk = VICP_XCD_CHUNK;

__device__ __forceinline__ int xcd_job(int b, int n)
{
    if (kXcdChunk <= 0) return b;
    constexpr int span = kXcds * kXcdChunk;
    const int full = (n / span) * span;
    if (b >= full) return b;
    const int x = b % kXcds, i = b / kXcds;
    return ((i / kXcdChunk) * kXcds + x) * kXcdChunk + (i % kXcdChunk);
}

// XCD slabs: XCD x receives the x-th eighth of the jobs as one contiguous
// range (block b runs on XCD b mod 8 and is its (b / 8)-th block).  For work
// of uniform cost whose neighbouring jobs share data (the dilation's voxel
// tiles and their halos), each XCD's L2 then holds one slab of the grid
// instead of a share of every part of it.  A bijection on [0, n); the
// n mod 8 jobs past the last whole round keep their index.
__device__ __forceinline__ int xcd_slab(int b, int n)
{
    const int per = n / kXcds, full = per * kXcds;
    if (b >= full) return b;
    return (b % kXcds) * per + b / kXcds;
}

// --------------------------------------------------------------------------
// wave64 reductions on DPP (no LDS round trips)
// --------------------------------------------------------------------------

// x + (x moved by the DPP control CTRL within the rows of ROW_MASK; lanes
// whose source is outside the row read 0).  Both 32-bit halves move.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROW_MASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROW_MASK, 0xF, true);
    return x + __hiloint2double(hi, lo);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_add_u32(uint32_t x)
{
    return x + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xF, true);
}

// Sum inside each row of 16 lanes (an inclusive scan) of values held in the
// lanes that are multiples of STRIDE (the others hold zero): steps of
// STRIDE, 2 STRIDE, ... 8; the row's total ends in lane 16 - STRIDE.
template <int STRIDE>
__device__ __forceinline__ uint32_t row_sum_u32(uint32_t x)
{
    if (STRIDE <= 1) x = dpp_add_u32<0x111, 0xF>(x);
    if (STRIDE <= 2) x = dpp_add_u32<0x112, 0xF>(x);
    if (STRIDE <= 4) x = dpp_add_u32<0x114, 0xF>(x);
    x = dpp_add_u32<0x118, 0xF>(x);
    return x;
}

// Sum over the 64 lanes in a fixed order (an inclusive scan inside each row
// of 16, then rows 0+1 and 2+3, then the two halves), returned to every lane.
__device__ __forceinline__ double wave_sum_f64(double x)
{
    x = dpp_add<0x111, 0xF>(x);   // row_shr:1
    x = dpp_add<0x112, 0xF>(x);   // row_shr:2
    x = dpp_add<0x114, 0xF>(x);   // row_shr:4
    x = dpp_add<0x118, 0xF>(x);   // row_shr:8
    x = dpp_add<0x142, 0xA>(x);   // row_bcast:15 into rows 1 and 3
    x = dpp_add<0x143, 0xC>(x);   // row_bcast:31 into rows 2 and 3
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), 63),
                            __builtin_amdgcn_readlane(__double2loint(x), 63));
}

// --------------------------------------------------------------------------
// Rank of e among the c values a[lo .. lo + c): how many are smaller.  Reads
// 16-byte aligned chunks, eight in flight per round; a must be allocated with
// at least 4 words of slack past its last element (a chunk may run over).
// --------------------------------------------------------------------------
__device__ __forceinline__ uint32_t rank_in(const uint32_t* __restrict__ a, int64_t lo, uint32_t c, uint32_t e)
{
    if (c == 0) return 0;
    const uint4* v4 = reinterpret_cast<const uint4*>(a + (lo & ~(int64_t)3));
    const int64_t first = lo & 3, end = first + c;   // positions relative to the aligned base
    const int64_t last_chunk = (end - 1) >> 2;
    uint32_t r = 0;
    for (int64_t k = 0; k <= last_chunk; k += 8) {
        uint4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = v4[min(k + u, last_chunk)];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t pos = 4 * (k + u);
            const bool live = k + u <= last_chunk;
            r += (live && pos >= first && pos < end && v[u].x < e) ? 1u : 0u;
            r += (live && pos + 1 >= first && pos + 1 < end && v[u].y < e) ? 1u : 0u;
            r += (live && pos + 2 >= first && pos + 2 < end && v[u].z < e) ? 1u : 0u;
            r += (live && pos + 3 >= first && pos + 3 < end && v[u].w < e) ? 1u : 0u;
        }
    }
    return r;
}

// The same rank taken by a whole wave whose 64 lanes all rank within the
// same c words (a long segment): the wave loads the words once, kCoopChunk
// at a time, into its own LDS slice `chunk`, and every lane compares its own
// e with each word there (broadcast reads).  Equal to rank_in for every
// lane (padding words are 0xFFFFFFFF, above any index), with O(c) global
// loads per wave instead of per lane.  The caller checks that all 64 lanes
// are active and share the segment.
constexpr int kCoopChunk = 256;
constexpr uint32_t kCoopMin = 256;   // segments at least this long take the wave-wide form
__device__ __forceinline__ uint32_t rank_in_wave(const uint32_t* __restrict__ a, int64_t lo, uint32_t c, uint32_t e,
                                                 uint32_t* chunk)
{
    const int lane = threadIdx.x & 63;
    uint32_t r = 0;
    for (uint32_t base = 0; base < c; base += kCoopChunk) {
        uint32_t v[kCoopChunk / 64];
#pragma unroll
        for (int j = 0; j < kCoopChunk / 64; ++j) {
            const uint32_t idx = base + (uint32_t)(j * 64 + lane);
            v[j] = idx < c ? a[lo + idx] : 0xFFFFFFFFu;
        }
#pragma unroll
        for (int j = 0; j < kCoopChunk / 64; ++j) chunk[j * 64 + lane] = v[j];
        // a wave's LDS accesses execute in order: the barriers only keep the
        // compiler from moving them across
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 8
        for (int i = 0; i < kCoopChunk; i += 4) {
            const uint4 q = *reinterpret_cast<const uint4*>(chunk + i);
            r += (q.x < e ? 1u : 0u) + (q.y < e ? 1u : 0u) + (q.z < e ? 1u : 0u) + (q.w < e ? 1u : 0u);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    return r;
}

// True when every lane of the wave is active and shares the value x.
__device__ __forceinline__ bool wave_full_and_uniform(int64_t x)
{
    const bool full = __ballot(1) == ~0ull;
    const int64_t x0 = __shfl(x, 0, 64);
    return full && __ballot(x == x0) == ~0ull;
}

// --------------------------------------------------------------------------
// Kernel timing.  While a timed scope of the runtime is open on this thread
// (and its stream is not being captured), launch_timed hands the scope's two
// events to the launch, and the runtime records them at the kernel's own
// start and end; otherwise it is a plain launch.
// --------------------------------------------------------------------------
bool prof_take_ext_events(hipEvent_t* start, hipEvent_t* stop);

template <typename F, typename... Args>
inline void launch_timed(F kernel, dim3 grid, dim3 block, hipStream_t s, Args... args)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (prof_take_ext_events(&a, &b))
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, a, b, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

// The same with `lds` bytes of dynamic LDS.
template <typename F, typename... Args>
inline void launch_timed_lds(F kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, Args... args)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (prof_take_ext_events(&a, &b))
        hipExtLaunchKernelGGL(kernel, grid, block, lds, s, a, b, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}

// --------------------------------------------------------------------------
// kernel launchers (one translation unit each; all asynchronous)
// --------------------------------------------------------------------------

// grid build
void launch_aabb(const float* qx, const float* qy, const float* qz, const PairDev* pd,
                 const BlockJob* jobs, int njobs, int items_per_block, uint32_t* box, uint32_t tag, hipStream_t s);
// block: target points per block (256, 512 or 1024; the packed-hash
// ablation always takes 256); jobs must hold `block` points per entry
// big_list / big_count (both or neither): every voxel whose count reaches
// kSegSortMin is appended once (its segment is then sorted by
// launch_sort_segments instead of ranked point by point)
void launch_count(const float* qx, const float* qy, const float* qz, const PairDev* pd,
                  const BlockJob* jobs, int njobs, int block, uint32_t* hist, uint32_t* vox, uint32_t* rank,
                  uint32_t* err, bool packed, hipStream_t s, uint32_t* big_list = nullptr,
                  uint32_t* big_count = nullptr);
bool count_packed_fits(int64_t voxels);
// VANICP's layout: counts every point of a voxel into cnt and copies it into
// the voxel's block of cap records when it fits
void launch_count_direct(const float* qx, const float* qy, const float* qz, const PairDev* pd,
                         const BlockJob* jobs, int njobs, uint32_t* cnt, uint32_t* err, float4* blk,
                         uint32_t cap, hipStream_t s);
void launch_seg_headers(const uint32_t* hist, const uint32_t* off, int64_t total, uint32_t* vm, uint2* dir,
                        hipStream_t s);
int scan_tiles(int64_t total);
void launch_scan(const uint32_t* hist, int64_t total, uint32_t* off, uint32_t* vm, uint2* dir,
                 unsigned long long* status, uint32_t* ticket, hipStream_t s);
void launch_place(const PairDev* pd, const BlockJob* jobs, int njobs, const uint32_t* vox,
                  const uint32_t* rank, const uint32_t* off, uint32_t* tmp, hipStream_t s);
// sort_min: segments of kSegSortMin to kSegSortMax points are left to
// launch_sort_segments (pass kSegSortMin when it runs, else UINT32_MAX)
void launch_rank_sort(const float* qx, const float* qy, const float* qz, const PairDev* pd,
                      const BlockJob* jobs, int njobs, const uint32_t* vox, const uint32_t* hist,
                      const uint32_t* off, const uint32_t* tmp, uint32_t* vm, float4* qs4,
                      hipStream_t s, uint32_t sort_min = 0xFFFFFFFFu);
// Long segments of a single-pair grid listed by the count: each sorted in
// LDS (ascending index) by one block, then written to vm and qs4.
constexpr uint32_t kSegSortMin = 512;
constexpr uint32_t kSegSortMax = 16384;
void launch_sort_segments(const float* qx, const float* qy, const float* qz, const PairDev* pd,
                          const uint32_t* big_list, const uint32_t* big_count, const uint32_t* hist,
                          const uint32_t* off, const uint32_t* tmp, uint32_t* vm, float4* qs4, hipStream_t s);
void launch_clear4(uint32_t* a, int64_t na, unsigned long long* b, int64_t nb, uint32_t* c, int64_t nc, uint32_t* d,
                   int64_t nd, hipStream_t s);
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s);
void launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t count, hipStream_t s);

// dilation: one ring over jobs of 256 consecutive voxels, block = 64, 128
// or 256 threads per job
void launch_dilate_ring(const PairDev* pd, const BlockJob* jobs, int njobs, int block,
                        const uint32_t* hist, const uint32_t* off, uint32_t* vm, uint2* dir,
                        const uint32_t* src, uint32_t* dst, int first, int last, hipStream_t s);
// all rings in one launch for rings <= kFusedRings, over a table of voxel
// tiles of one of kDilateShapes shapes (dilate_tiles per pair); returns false
// (nothing launched) otherwise.  Reads the search directory the offset scan
// wrote, writes Mask(root) count words and the dilated voxels' entries.
constexpr int kFusedRings = 4;
constexpr int kDilateShapes = 5;
int64_t dilate_tiles(int shape, int Dx, int Dy, int Dz);
bool launch_dilate_fused(const PairDev* pd, const BlockJob* jobs, int njobs, int rings, int shape, uint32_t* vm,
                         uint2* dir, hipStream_t s);
// VANICP's layout (single pair): copies each dilated voxel's root records
// into its block, from the ring state (own id, root id or none per voxel)
void launch_replicate(const PairDev* pd, int64_t V, const uint32_t* state, uint32_t* cnt, float4* blk,
                      uint32_t cap, hipStream_t s);

// search and moments; one_m >= 0: a single pair of one_m source points with
// jobs of block / lpq queries each (the table is not read), else -1
void launch_nns_local(const PairDev* pd, const BlockJob* jobs, int njobs, int block, int lpq, bool sorted, bool mom,
                      const float* px, const float* py, const float* pz, const float4* ps4,
                      const PairState* st, const uint2* dir, const float4* qs4, const float4* qsg,
                      int32_t* nn_idx, float* nn_d2, int32_t* fb_count, int32_t* fb_miss, uint32_t* fb_list,
                      unsigned long long* fb_key, unsigned long long* ctr, double* part, int all_global,
                      const uint32_t* dcnt, uint32_t cap, int mode, int64_t one_m, hipStream_t s);
void launch_src_bucket(const PairDev* pd, const BlockJob* jobs, int njobs, const float* px, const float* py,
                       const float* pz, const PairState* st, uint32_t* sh, uint32_t* skey, uint32_t* srank,
                       int32_t* sbig, int32_t* flags, hipStream_t s);
void launch_src_place(const PairDev* pd, const BlockJob* jobs, int njobs, const uint32_t* skey,
                      const uint32_t* srank, const uint32_t* soff, uint32_t* sidx, hipStream_t s);
void launch_src_rank(const PairDev* pd, const BlockJob* jobs, int njobs, const float* px, const float* py,
                     const float* pz, const uint32_t* skey, const uint32_t* soff, const uint32_t* sidx,
                     const int32_t* sbig, float4* ps4, hipStream_t s);
// The refill's count, scan, scatter and order passes each paired with the
// source plan's matching pass in one launch (blocks [0, nq) the refill's,
// the rest the plan's): k_count<false, 256> with k_src_bucket, the two
// look-back scans, k_place with k_src_place, k_rank_sort with k_src_rank.
void launch_count_bucket(const float* qx, const float* qy, const float* qz, const PairDev* pd,
                         const BlockJob* qjobs, int nq, uint32_t* hist, uint32_t* vox, uint32_t* rank, uint32_t* err,
                         const BlockJob* pjobs, int np, const float* px, const float* py, const float* pz,
                         const PairState* st, uint32_t* sh, uint32_t* skey, uint32_t* srank, int32_t* sbig,
                         int32_t* flags, hipStream_t s);
void launch_scan_pair(const uint32_t* hist, int64_t total, uint32_t* off, uint32_t* vm, uint2* dir,
                      unsigned long long* status, uint32_t* ticket, const uint32_t* sh, int64_t nb, uint32_t* soff,
                      unsigned long long* s_status, uint32_t* s_ticket, hipStream_t s);
void launch_place_pair(const PairDev* pd, const BlockJob* qjobs, int nq, const uint32_t* vox, const uint32_t* rank,
                       const uint32_t* off, uint32_t* tmp, const BlockJob* pjobs, int np, const uint32_t* skey,
                       const uint32_t* srank, const uint32_t* soff, uint32_t* sidx, hipStream_t s);
void launch_rank_pair(const float* qx, const float* qy, const float* qz, const PairDev* pd, const BlockJob* qjobs,
                      int nq, const uint32_t* vox, const uint32_t* hist, const uint32_t* off, const uint32_t* tmp,
                      uint32_t* vm, float4* qs4, const BlockJob* pjobs, int np, const float* px, const float* py,
                      const float* pz, const uint32_t* skey, const uint32_t* soff, const uint32_t* sidx,
                      const int32_t* sbig, float4* ps4, hipStream_t s);
// false (nothing launched) for npairs outside [1, kFbMaxPairs]
bool launch_fallback(const PairDev* pd, int npairs, int grid, const float* qx, const float* qy, const float* qz,
                     const float* px, const float* py, const float* pz, const PairState* st, const int32_t* fb_count,
                     const uint32_t* fb_list, unsigned long long* fb_key, const FoldJob* fjobs, int nunits,
                     const double* part, const unsigned long long* ctr, double* fpart,
                     unsigned long long* fctr, hipStream_t s);
void launch_fb_finalize(const PairDev* pd, const BlockJob* jobs, int njobs,
                        const unsigned long long* fb_key, int32_t* nn_idx, float* nn_d2,
                        int32_t* flags, hipStream_t s);
void launch_solve(const PairDev* pd, int npairs, const int32_t* fold_begin, int32_t nunits, const double* fpart,
                  const unsigned long long* fctr, PairState* st, int32_t* fb_count, const uint32_t* fb_list,
                  const unsigned long long* fb_key, const float* px, const float* py, const float* pz,
                  const float* qx, const float* qy, const float* qz, int32_t* flags, double* rmse_hist,
                  int32_t* fb_hist, int32_t* deg_hist, unsigned long long* ctr_hist, int k, int K, int early_stop,
                  double eps, int32_t* nn_idx, float* nn_d2, hipStream_t s);
// the same with the poses of up to kInlinePairs pairs passed in the launch
// itself (host array), so no upload precedes it
constexpr int kInlinePairs = 8;
void launch_set_state_inline(const PairDev* pd, PairState* st, const double* host_rt, int npairs,
                             int32_t* fb_count, int32_t* flags, hipStream_t s);
void launch_set_state(const PairDev* pd, PairState* st, const double* rt64, int npairs, int32_t* fb_count,
                      int32_t* flags, hipStream_t s);
void launch_check_finite(const PairDev* pd, const BlockJob* jobs, int njobs, const float* px, const float* py,
                         const float* pz, int32_t* flags, hipStream_t s);
void launch_copy_fb(const int32_t* fb_count, int32_t* out, int npairs, hipStream_t s);

// differentiable loss
void launch_se3(const double* xi, int npairs, PairState* st, double* jl6, int32_t* fb_count, int32_t* flags,
                hipStream_t s);
void launch_loss_terms(const PairDev* pd, const BlockJob* jobs, int njobs, const float* px,
                       const float* py, const float* pz, const float* qx, const float* qy,
                       const float* qz, const PairState* st, const unsigned long long* fb_key,
                       int32_t* nn_idx, const double* gloss, float* dpx, float* dpy, float* dpz,
                       double* part, int32_t* flags, hipStream_t s);
void launch_loss_finish(const PairDev* pd, int npairs, const int32_t* job_begin,
                        const double* part, const double* jl6, const double* gloss,
                        double* loss, double* dxi, hipStream_t s);

}  // namespace vicp
