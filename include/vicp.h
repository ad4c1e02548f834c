/*
 * vicp.h -- C ABI of libvicp: dilation-based ICP with segmented, offset-
 * addressed dilation memory on AMD Instinct MI355X (gfx950).
 *
 * The method is the one of Chang, Wang, Zhong and Miyazaki, "A dynamic memory
 * assignment strategy for dilation-based ICP algorithm on embedded GPUs"
 * (arXiv 2512.04996): align a source cloud P = {p_1..p_m} to a target cloud
 * Q = {q_1..q_n} by the rigid R, t that minimise Eq. 1 (sum_i |R p_i + t - q'_i|^2,
 * q'_i the correspondence of p_i), with correspondences found by a local search
 * inside voxels of a dilated target grid (Sec. II.A, Steps 1-3) whose per-voxel
 * memory is assigned from a histogram and its prefix offsets (Sec. III,
 * Algorithms 1-4).
 *
 * Conventions for every entry point
 * ---------------------------------
 * Layout     Point clouds are structure-of-arrays float32: three device arrays
 *            x[k], y[k], z[k], each contiguous.  Batched calls take the pairs'
 *            points concatenated in pair order, with per-pair counts in a HOST
 *            array.  Voxel ids are x-fastest: v = ix + Dx*(iy + Dy*iz).
 * Ownership  The caller owns every input and output buffer and keeps it alive
 *            until the work queued on the stream has finished.  A grid keeps a
 *            reference to the target arrays it was built from (not a copy of
 *            the coordinates' ownership): they must outlive the grid.  The grid
 *            owns its histogram, offsets, dilated voxel index and workspaces,
 *            allocated through the caller's vicp_allocator, or with
 *            hipMallocAsync on the given stream when that is NULL.
 * Streams    All device work is queued on the caller's stream in order.  Calls
 *            that must read a value back (grid sizing, registration results)
 *            wait for it, and say so: the grid sizing and the registration
 *            results arrive through pinned host memory that the device
 *            writes, with a tag the host waits for (every kernel that
 *            produced the value has finished by then; the stream may still
 *            be finishing the small kernel that wrote it).
 * Errors     Every call returns VICP_OK (0) or a negative VICP_ERR_* code and
 *            never aborts or prints; vicp_last_error() gives a message for the
 *            calling thread.  Faults found on the device (non-finite source
 *            coordinates, degenerate cross-covariance) are latched in the grid
 *            and returned by the next call that waits for the device.
 * Threads    A grid may be used by one host thread at a time.  Distinct grids
 *            are independent.
 */
#ifndef VICP_H
#define VICP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define VICP_OK 0
#define VICP_ERR_INVALID_ARG (-1)   /* bad size, pointer, voxel, ring count or pair count */
#define VICP_ERR_GRID_TOO_LARGE (-2) /* V >= 2^31 voxels or n + 2V >= 2^32 words */
#define VICP_ERR_OOM (-3)           /* the allocator returned NULL */
#define VICP_ERR_HIP (-4)           /* a HIP runtime call failed */
#define VICP_ERR_STATE (-5)         /* call out of order (e.g. dilating twice) */
#define VICP_ERR_NONFINITE (-6)     /* NaN or Inf in the input coordinates */
#define VICP_ERR_DEGENERATE (-7)    /* cross-covariance of rank < 2: pose kept */

/* Mask(root) of a dilated voxel's count word (Alg. 3): bit 31 set. */
#define VICP_MASK_BIT 0x80000000u

typedef struct vicp_grid vicp_grid;

/* Stream-ordered allocator supplied by the caller (e.g. a framework's caching
 * allocator).  alloc returns device memory of at least `bytes` usable on
 * `stream`, or NULL; free releases it after the stream's queued work. */
typedef struct vicp_allocator {
    void* (*alloc)(size_t bytes, hipStream_t stream, void* user);
    void (*free)(void* ptr, size_t bytes, hipStream_t stream, void* user);
    void* user;
} vicp_allocator;

/* Description of one pair's grid (Sec. II.A Step 1; Table 1 accounting). */
typedef struct vicp_grid_desc {
    float origin[3];       /* lower corner: target box minimum minus pad_rings voxels */
    float inv;             /* 1/voxel, rounded once to float32 */
    float voxel;           /* voxel edge */
    int32_t dims[3];       /* voxels per axis */
    int64_t V;             /* dims[0]*dims[1]*dims[2] */
    int64_t n;             /* target points */
    int32_t pad_rings;     /* padding the grid was built with */
    int32_t rings_applied; /* dilation rings applied so far (0 before vicp_dilate) */
    int64_t occupied;      /* voxels holding >= 1 target point */
    int64_t dilated;       /* empty voxels given a root by dilation */
    uint32_t max_count;    /* largest per-voxel count */
    int64_t static_bytes;  /* histogram + offsets: 8 V (Table 1, note 1) */
    int64_t dynamic_bytes; /* dilated voxel index: 4 (n + 2V) */
    int64_t vanicp_bytes;  /* fixed 64 KiB per voxel of the original VANICP (Sec. II.B) */
    int64_t extra_bytes;   /* device bytes this library holds beyond the two above */
} vicp_grid_desc;

/* ICP options (Sec. IV.A "Parameter": maximum iterations and RMSE difference). */
typedef struct vicp_icp_opts {
    int32_t max_iter;   /* K >= 0 */
    double rmse_eps;    /* stop when |RMSE_k - RMSE_{k-1}| < rmse_eps (k >= 1) ... */
    int32_t early_stop; /* ... only if non-zero; 0 runs exactly K iterations */
    int32_t use_graph;  /* non-zero: capture the K iterations once in a hipGraph and replay it */
    int32_t global_only; /* non-zero: every query takes the exact global search (ICP with exhaustive
                            NNS, the "Brute" comparator of Table 2); the grid is not consulted */
    int32_t layout;      /* 0: the segmented, offset-addressed layout (Alg. 2-4); 1: VANICP's
                            monolithic direct-addressed layout built by vicp_direct_build (the
                            comparator); excludes global_only */
    int32_t* nn_idx;     /* optional (NULL: not written): device int32[m] (batched: all pairs'
                            sources in pair order) receiving, for every source point, the target
                            index of its Alg. 4 correspondence in the last iteration the pair ran,
                            written by the registration's own search and solve kernels */
    float* nn_d2;        /* with nn_idx: device float32[m], the squared distances (float32) */
} vicp_icp_opts;

/* Per-pair registration statistics.  The arrays are caller-owned HOST arrays
 * of max_iter entries and may be NULL. */
typedef struct vicp_icp_stats {
    int32_t iters;            /* iterations run */
    int32_t degenerate;       /* iterations whose solve kept the previous pose */
    double* rmse;             /* RMSE_k = sqrt(mean nn_d2) of iteration k */
    int64_t* fallbacks;       /* queries that took the global search in iteration k */
    int64_t* candidates;      /* target points scanned by local searches in iteration k */
    int64_t* dilated_lookups; /* local searches redirected through Mask(root) in iteration k */
} vicp_icp_stats;

/* ---- build (Alg. 1 and Alg. 2) --------------------------------------------
 * Voxelises the target (qx, qy, qz; n points, device) with edge `voxel` on the
 * target's bounding box padded by `pad_rings` voxels, counts points per voxel,
 * exclusive-scans count + 2 into segment offsets, and scatters point indices
 * into their segments [lock = 0, count, indices ascending].  Waits once for
 * the device, for the bounding box that sizes the grid (per-block partials
 * written into pinned host memory; the stream itself is synchronised only
 * when that takes over a millisecond).
 * Errors: n <= 0, voxel <= 0 or non-finite, pad_rings < 0 -> INVALID_ARG;
 * non-finite target coordinates -> NONFINITE; grid too large -> GRID_TOO_LARGE;
 * a padded grid reaching beyond +-VICP_COORD_LIMIT on any axis (float32
 * squared distances inside it could overflow) -> INVALID_ARG. */
#define VICP_COORD_LIMIT 1e18f
int vicp_build_grid(const float* qx, const float* qy, const float* qz, int64_t n,
                    float voxel, int32_t pad_rings, const vicp_allocator* alloc,
                    hipStream_t stream, vicp_grid** out);

/* As vicp_build_grid for `npairs` independent targets concatenated in pair
 * order; n_per_pair and voxel_per_pair are HOST arrays of npairs entries. */
int vicp_build_grid_batched(const float* qx, const float* qy, const float* qz,
                            const int64_t* n_per_pair, int32_t npairs,
                            const float* voxel_per_pair, int32_t pad_rings,
                            const vicp_allocator* alloc, hipStream_t stream,
                            vicp_grid** out);

/* As vicp_build_grid on a given grid instead of the target's padded bounding
 * box: `dims` voxels of edge `voxel` from `origin` (HOST arrays of 3), i.e.
 * the setting of Sec. IV.A, 2^N voxels per axis over the unit sphere's cube
 * [-1, 1)^3 for clouds normalised to the unit sphere.  `max_rings` bounds the
 * rings a later vicp_dilate may apply (it plays the role of pad_rings; the
 * grid is not padded).  Voxel indices and 1/voxel follow the same float32
 * arithmetic as every grid.  A rebuild keeps the geometry.  Synchronises the
 * stream once, to check that every target point lies inside the grid.
 * Errors: n <= 0, voxel <= 0 or non-finite, non-finite origin, dims < 1,
 * max_rings < 0, or a target point outside the grid -> INVALID_ARG (the grid
 * then needs a successful rebuild before use); grid too large ->
 * GRID_TOO_LARGE. */
int vicp_build_grid_fixed(const float* qx, const float* qy, const float* qz, int64_t n,
                          const float origin[3], float voxel, const int32_t dims[3],
                          int32_t max_rings, const vicp_allocator* alloc,
                          hipStream_t stream, vicp_grid** out);

/* Refills an existing grid from a new target with the same per-pair point
 * counts (e.g. the next frame of a stream): the bounding box, grid
 * specification, counts, offsets and segments are recomputed exactly as by
 * vicp_build_grid, while allocations, work tables and captured graphs are
 * reused when the voxel counts are unchanged.  The grid is left undilated:
 * call vicp_dilate again.  Waits once for the device (bounding box).
 * Errors as vicp_build_grid; STATE for a grid that was never built.  After a
 * rebuild fails once the new bounding box is known (a target point outside a
 * given-geometry grid, an allocation or a launch failure), every other entry
 * point returns STATE for that grid until a rebuild succeeds. */
int vicp_grid_rebuild(vicp_grid* g, const float* qx, const float* qy, const float* qz,
                      hipStream_t stream);

/* The Alg. 1 ablation, for later builds and rebuilds of this grid:
 * host_offsets != 0 computes the offsets as the paper's CPU part does (the
 * histogram is copied to the host, scanned there serially, and the offsets
 * copied back; two synchronisations); packed_hash != 0 counts with the
 * paper's fused 32-bit LDS hash entry (voxel key and count in one word;
 * grids of 2^23 voxels or more per pair keep the default count).  The grid
 * built either way is identical.  The host scan's time is reported by
 * vicp_prof_read as "moc_host" while timing is enabled.
 * Errors: null grid -> INVALID_ARG. */
int vicp_set_build_options(vicp_grid* grid, int32_t host_offsets, int32_t packed_hash);

/* ---- VANICP's monolithic layout (the comparator) -------------------------
 * Sec. II.B describes the layout the paper replaces: a fixed memory block per
 * voxel (64 KiB) into which voxelisation copies the voxel's points and
 * dilation copies the root's points, so that the search addresses a voxel's
 * candidates directly; Sec. IV.B notes that points beyond a block's capacity
 * send the search to the global fallback.  vicp_direct_build builds that
 * layout for a built and dilated single-pair grid, on the same geometry and
 * with the same rings (roots as Alg. 3):
 *   - blocks: V * block_bytes device bytes, allocated here with hipMalloc and
 *     owned by the grid (about 21.8 GB for 332k voxels at 64 KiB); records of
 *     16 bytes (float32 x, y, z and the point index as 32 bits), so a block
 *     holds block_bytes / 16 points, in no particular order;
 *   - a count word per voxel: the voxel's own point count, or its root's
 *     count with bit 31 set for a dilated voxel;
 *   - a voxel whose count exceeds the capacity keeps only what fitted, and
 *     its queries, and those of voxels dilated from it, take the global
 *     search.
 * A registration with opts.layout = 1 then searches these blocks.  Without
 * overflow it returns exactly what the segmented layout returns (ties go to
 * the lowest index in both).  Asynchronous except when it (re)allocates.
 * Errors: null grid -> INVALID_ARG; grid not built, failed or not dilated ->
 * STATE; more than one pair, block_bytes not a positive multiple of 16 ->
 * INVALID_ARG; the device allocation fails -> OOM.  Any rebuild of the grid
 * invalidates the layout (STATE until it is built again). */
int vicp_direct_build(vicp_grid* g, int64_t block_bytes, hipStream_t stream);

/* Frees the blocks of vicp_direct_build (synchronises the device).  No-op
 * when there are none.  Errors: null grid -> INVALID_ARG. */
int vicp_direct_free(vicp_grid* g);

/* ---- dilation (Alg. 3) ----------------------------------------------------
 * Applies `rings` synchronous dilation rings (0 <= rings <= pad_rings) to every
 * pair: an empty voxel within L1 distance `rings` of an occupied voxel gets
 * Mask(root) in its count word, root = the nearest occupied voxel, lowest id
 * on ties.  May be called once per grid; again -> STATE.  Asynchronous. */
int vicp_dilate(vicp_grid* g, int32_t rings, hipStream_t stream);

/* ---- nearest-neighbour search (Alg. 4) ------------------------------------
 * For each source point (px, py, pz; m points, device) of a single-pair grid:
 * s = R p + t with Rt = 12 HOST floats (R row-major, then t); the voxel of s,
 * then its own segment, its root's segment when dilated, or an exact search
 * over all targets when the voxel is empty or s is outside the grid.  Writes
 * nn_idx[m] (target index, ties to the lowest) and nn_d2[m] (float32 squared
 * distance) to device memory, and the number of global searches to the device
 * int32 *n_fallback when it is not NULL.  m == 0 is a no-op.  Asynchronous. */
int vicp_nns(const vicp_grid* g, const float* px, const float* py, const float* pz,
             int64_t m, const float Rt[12], int32_t* nn_idx, float* nn_d2,
             int32_t* n_fallback, hipStream_t stream);

/* Batched form: m_per_pair HOST array, Rt HOST float[npairs*12], outputs
 * concatenated in pair order, n_fallback a device int32[npairs] or NULL. */
int vicp_nns_batched(const vicp_grid* g, const float* px, const float* py, const float* pz,
                     const int64_t* m_per_pair, const float* Rt, int32_t* nn_idx,
                     float* nn_d2, int32_t* n_fallback, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): vicp_nns
 * with every intermediate (the pose, the work tables, the global-search list
 * and its keys, the per-block counters) in one fixed device array that the
 * library holds on each GPU it runs on until the process ends
 * (14,713,600 bytes, sized for VICP_NOALLOC_MAX_QUERIES source points),
 * instead of the grid's workspace.  Same arguments, outputs and results as vicp_nns (bit for bit:
 * the same search kernels, over the source in index order); the grid must
 * have been built beforehand (building allocates).  Allocates nothing: no
 * hipMalloc, no hipFree, no allocating library routine.  Every call on one
 * GPU shares that GPU's array and overwrites what the last call left there,
 * so calls that overlap on one GPU (other streams or host threads) race:
 * the caller serialises them.  Asynchronous.  Errors: as vicp_nns;
 * m > VICP_NOALLOC_MAX_QUERIES -> INVALID_ARG; a HIP error while locating
 * the array on first use on a device -> HIP. */
#define VICP_NOALLOC_MAX_QUERIES (1 << 20)
int vicp_nns_noalloc(const vicp_grid* g, const float* px, const float* py, const float* pz,
                     int64_t m, const float Rt[12], int32_t* nn_idx, float* nn_d2,
                     int32_t* n_fallback, hipStream_t stream);

/* ---- registration (Sec. II.A loop, Eq. 1) ---------------------------------
 * Runs the ICP loop on a single-pair grid: correspondences by Alg. 4 at the
 * float32-rounded pose, then the closed-form rigid transform of Eq. 1 on
 * (original p_i, q_c(i)) in float64, repeated opts->max_iter times or until
 * the RMSE difference rule stops it.  Rt_io: 12 HOST doubles, initial pose in,
 * final pose out.  `stats` may be NULL.  Waits at the end until the results
 * are in host memory (written there by the device after every kernel of the
 * loop has finished).
 * Returns DEGENERATE (pose still valid) if any solve kept the previous pose. */
int vicp_register(const vicp_grid* g, const float* px, const float* py, const float* pz,
                  int64_t m, const vicp_icp_opts* opts, double Rt_io[12],
                  vicp_icp_stats* stats, hipStream_t stream);

/* Batched form: every pair runs its own loop inside one launch sequence.
 * m_per_pair HOST int64[npairs]; Rt_io HOST double[npairs*12]; stats HOST
 * array of npairs entries or NULL. */
int vicp_register_batched(const vicp_grid* g, const float* px, const float* py, const float* pz,
                          const int64_t* m_per_pair, const vicp_icp_opts* opts, double* Rt_io,
                          vicp_icp_stats* stats, hipStream_t stream);

/* The next frame in one call: vicp_grid_rebuild(qx, qy, qz), vicp_dilate(rings)
 * and vicp_register_batched(px, ...) in turn, with the same results, errors
 * and waits.  When the schedule buckets the source (Alg. 4's queries sorted
 * by target voxel), each of the refill's count, scan, scatter and order
 * passes (Alg. 1-2) shares one launch with the bucketing's matching pass, as
 * the two are independent; everything stays on `stream`.  Given-geometry
 * grids, host-side offsets, the packed-hash count, the direct layout,
 * global_only and searches over the source in index order take the three
 * calls' path.  Errors: as the three calls; STATE for a grid that was never
 * built.  A failure after the bounding box leaves the grid refusing every
 * call with STATE until a rebuild succeeds, as a failed rebuild does. */
int vicp_rebuild_register(vicp_grid* g, const float* qx, const float* qy, const float* qz,
                          int32_t rings, const float* px, const float* py, const float* pz,
                          const int64_t* m_per_pair, const vicp_icp_opts* opts, double* Rt_io,
                          vicp_icp_stats* stats, hipStream_t stream);

/* ---- differentiable point-to-point loss ------------------------------------
 * For pair b with pose xi_b = (rho, phi) in R^6 (device float64[npairs*6]),
 * T = Exp(xi_b) in SE(3), correspondences c_i from Alg. 4 at the float32-rounded
 * T, and L_b = (1/m_b) sum_i |T p_i - q_c(i)|^2 (the objective of Eq. 1 per
 * point).  Forward writes loss[npairs] (device float64).  Backward recomputes
 * the correspondences (never stored) and, given dL/dL_b in gloss (device
 * float64[npairs]), writes dP (device float32 SoA, same layout as p) and dxi
 * (device float64[npairs*6], through the SE(3) left Jacobian).  Asynchronous. */
int vicp_p2p_loss_fwd(const vicp_grid* g, const float* px, const float* py, const float* pz,
                      const int64_t* m_per_pair, const double* xi, double* loss,
                      hipStream_t stream);
int vicp_p2p_loss_bwd(const vicp_grid* g, const float* px, const float* py, const float* pz,
                      const int64_t* m_per_pair, const double* xi, const double* gloss,
                      float* dpx, float* dpy, float* dpz, double* dxi, hipStream_t stream);

/* ---- helpers ---------------------------------------------------------------- */
/* Number of pairs in a grid. */
int vicp_grid_npairs(const vicp_grid* g);
/* Description of pair `pair`; synchronises the stream the grid was last used on. */
int vicp_grid_describe(const vicp_grid* g, int32_t pair, vicp_grid_desc* out);
/* Copies pair `pair`'s histogram (uint32[V]), offsets (uint32[V+1], relative to
 * the pair's segment base) and dilated voxel index (uint32[n+2V]) into device
 * buffers (any may be NULL).  Asynchronous. */
int vicp_grid_export(const vicp_grid* g, int32_t pair, uint32_t* hist, uint32_t* off,
                     uint32_t* vm, hipStream_t stream);
/* Releases the grid and everything it owns (after its queued work). */
int vicp_grid_free(vicp_grid* g);

/* Autotuning: times schedules on this grid and source and keeps the fastest
 * in the grid:
 *   - the count's block size (vicp_get_build_schedule), re-running the count
 *     (the histogram it leaves is the same);
 *   - on a dilated grid of 1 to 4 rings, the dilation's form and tile shape,
 *     re-running the dilation (which leaves the same grid);
 *   - the search (see vicp_get_schedule) in its registration form at the
 *     identity pose; the source-bucketing pass serves `searches_per_plan`
 *     searches (1 for vicp_nns, the iteration count for vicp_register) and is
 *     charged at that rate;
 *   - the global search's block count on a load of listed queries (the
 *     first max(256, m/64) sources of each pair) charged once per
 *     `searches_per_plan` searches, beside the fold it also runs.
 * The chosen schedule is stored per shape (pairs' point counts, grid
 * dimensions, rings, source sizes); a later call on the same shape in this
 * process takes it without timing, and with the environment variable
 * VICP_AUTOTUNE_CACHE naming a file, schedules are read from and appended to
 * that file.  Correspondences, counts and grids never depend on the schedule;
 * a pose may differ in its last bits (see vicp_get_schedule).  Synchronises
 * the stream. */
int vicp_autotune(vicp_grid* g, const float* px, const float* py, const float* pz,
                  const int64_t* m_per_pair, int32_t searches_per_plan, hipStream_t stream);

/* The current search schedule of a grid: threads per block of the local
 * search (128, 256 or 512), lanes cooperating on one query (1, 2, 4 or 8),
 * whether the source is bucketed by target voxel before searching (0/1), the
 * number of blocks of the global search, and the candidate loop of a
 * registration's search (search_mode): 0 each lane keeps its best
 * candidate's index and coordinates; 1 (any lanes per query) each lane
 * keeps its best segment position and the winner's record is read once,
 * fewer instructions per candidate and one more dependent load per query.
 * No setting changes a correspondence or a count.  The lanes per query (a
 * search wave sums the moments of 64 / lanes-per-query queries) and the
 * source order group the float64 moment sums, so they can change the last
 * bits of a pose; the threads per block, the global-search grid and the
 * search mode do not.  INVALID_ARG for an unsupported value or
 * combination. */
int vicp_get_schedule(const vicp_grid* g, int32_t* nns_block, int32_t* lanes_per_query,
                      int32_t* sort_source, int32_t* fallback_grid, int32_t* search_mode);
int vicp_set_schedule(vicp_grid* g, int32_t nns_block, int32_t lanes_per_query, int32_t sort_source,
                      int32_t fallback_grid, int32_t search_mode);

/* The build schedule of a grid: threads per block of the count (256, 512 or
 * 1024 target points per block, which is also how many points share one LDS
 * hash), and the dilation's form for 1 to 4 rings: dilate_fused = 1 runs every
 * ring in one launch on LDS tiles of shape dilate_tile (0: 8x8x4 voxels,
 * 1: 16x8x4, 2: 8x8x8, 3: 32x8x4, 4: 16x16x4, plus a halo of L voxels),
 * 0 one launch per ring with ring_block threads per 256-voxel block (64, 128
 * or 256; also the form for more than 4 rings).  No setting changes a result.
 * INVALID_ARG for an unsupported value. */
int vicp_get_build_schedule(const vicp_grid* g, int32_t* count_block, int32_t* dilate_fused, int32_t* dilate_tile,
                            int32_t* ring_block);
int vicp_set_build_schedule(vicp_grid* g, int32_t count_block, int32_t dilate_fused, int32_t dilate_tile,
                            int32_t ring_block);

/* Forgets every schedule vicp_autotune stored in this process (the file
 * named by VICP_AUTOTUNE_CACHE is left as it is). */
int vicp_autotune_cache_clear(void);

/* Per-kernel timing with HIP events on the launch stream (0 = off).  While on,
 * every launch of a named kernel is bracketed by events; vicp_prof_read gives
 * the count and summed milliseconds, vicp_prof_samples the duration of each
 * launch in launch order (up to `cap` into the HOST array ms, the number
 * recorded in *count); both synchronise the events.  vicp_prof_reset clears
 * both. */
int vicp_prof_enable(int32_t on);
int vicp_prof_read(const char* kernel, int64_t* launches, double* total_ms);
int vicp_prof_samples(const char* kernel, double* ms, int64_t cap, int64_t* count);
int vicp_prof_reset(void);

const char* vicp_status_str(int code);
const char* vicp_last_error(void);
const char* vicp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* VICP_H */
