/*
 * ogvdb.h -- C-ABI of the MI355X occupancy-grid ray sampler.
 *
 * Kato & Tarashima, "Plug-and-Play Acceleration of Occupancy Grid-based NeRF
 * Rendering using VDB Grid and Hierarchical Ray Traversal" (2024).  The
 * library turns a trained dense binary occupancy grid into a VDB-style tree
 * (Sec. 3) and marches camera rays through it with a hierarchical DDA that
 * steps over a whole empty tile at once (Sec. 2.3), emitting the fixed-step
 * sample points that fall in occupied voxels (Sec. 3; Alg. 1 and Alg. 2 of
 * the supplementary material).  The dense-grid voxel DDA the paper compares
 * against is available behind the same calls.  On top of the sampler: a fused
 * volume-rendering composite with its backward pass, and a batched
 * multi-scene launch.
 *
 * Conventions for every call
 *  - Return value: OGV_OK (0) or a negative ogv_status; no call throws or
 *    aborts.  ogv_last_error() gives a message for the calling thread.
 *  - Pointers named *_dev are device pointers (HBM of the current HIP
 *    device); pointers named *_host are host pointers.  Ray, sample and
 *    gradient buffers are owned by the caller.  The library owns only what
 *    sits behind an opaque handle and frees it in the matching *_destroy.
 *  - Work is enqueued on the caller's stream (a hipStream_t passed as void*;
 *    NULL is the default stream) and returns without waiting, except where
 *    a call says it synchronizes.  A built grid is read-only, so several
 *    sample calls may use one grid concurrently.
 *  - Geometry is binary32 throughout.  For cascade level l with box
 *    [B, A] (per axis) and R voxels per axis: h = fl((A-B)/R), plane
 *    P(m) = fl(B + fl(m*h)), crossing T(m) = fl(fl(P(m)-o)*fl(1/d)).  A voxel
 *    owns the ray parameters (entry, exit] (a point on a face belongs to the
 *    voxel the ray leaves, the "<=" tests of Alg. 1); an axis with d == 0 or
 *    an infinite 1/d keeps the voxel holding o (floor rule).  The finest
 *    level holding a parameter decides its occupancy (Sec. 3, last
 *    paragraph).  Samples are the lattice points t_n <= far in occupied
 *    voxels, n >= 0, with t_n = fl(near + fl(n*dt)) (constant step) or
 *    t_0 = near, t_{n+1} = fl(t_n + max(fl(t_n*cone), dt_min)) (growing
 *    step, Sec. 3); each is emitted as (ray id, t0 = t_n, t1 = t_{n+1}),
 *    ray-major, t ascending.  Rays with a non-finite component get none.
 */
#ifndef OGVDB_H
#define OGVDB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ogv_status;
#define OGV_OK 0
#define OGV_ERR_INVALID (-1)     /* bad argument (null pointer, size, parameter) */
#define OGV_ERR_CAPACITY (-2)    /* workspace or output capacity too small */
#define OGV_ERR_HIP (-3)         /* a HIP runtime call failed */
#define OGV_ERR_OOM (-4)         /* device allocation failed */
#define OGV_ERR_UNSUPPORTED (-5) /* valid but outside what the library handles */

#define OGV_MAX_LEVELS 8
#define OGV_MAX_RES 1024

/* Loop structure of the sampler (supplementary material):
 *   OGV_BRANCH -- Alg. 1 "DDA branch": one cell per iteration, branch on its
 *                 occupancy (NerfAcc's structure);
 *   OGV_SKIP   -- Alg. 2 "DDA skip": pass over all leading empty cells, then
 *                 march the occupied run (Instant-NGP's structure).
 * OGV_VOXEL may be or-ed into either, for VDB grids only: the tree is then
 * walked one voxel per step, each voxel's occupancy looked up in the tree and
 * no tile skipped in one step (the "VDB + DDA" rows of Tab. 1-2, against the
 * default hierarchical steps of "VDB + HDDA").  OGV_SUBLEAF (VDB grids only,
 * not with OGV_VOXEL) makes the hierarchical steps go on below the leaf
 * level: a uniform 4^3 sub-block of a leaf (all 64 voxels empty or all
 * occupied) is passed in one step, so empty space is skipped by powers of two
 * (root tile, 8^3 tile, 4^3 sub-block) down to single voxels (Fig. 1).  A
 * sampling call rejects either on any other grid with OGV_ERR_INVALID;
 * batches take OGV_BRANCH or OGV_SKIP only.
 * Every variant gives identical samples. */
#define OGV_BRANCH 0
#define OGV_SKIP 1
#define OGV_VOXEL 2
#define OGV_SUBLEAF 4

/* Options of a sampling call (NULL means {OGV_BRANCH, 0}).  image_width > 0
 * says the rays are the row-major pixels of an image that wide; lanes then
 * take 8x8 pixel tiles so neighbouring rays walk together.  It changes only
 * speed, never the samples or their order. */
typedef struct {
    int32_t variant;      /* OGV_BRANCH or OGV_SKIP, optionally | OGV_VOXEL or | OGV_SUBLEAF */
    int32_t image_width;  /* >= 0 */
} ogv_sample_opts;

#define OGV_STEP_CONST 0 /* t_n = near + n*dt            (NeRF-Synthetic, Sec. 3) */
#define OGV_STEP_CONE 1  /* dt_n = max(t_n*cone, dt_min) (Mip-NeRF 360, Sec. 3) */

typedef struct {
    int32_t kind;  /* OGV_STEP_CONST or OGV_STEP_CONE */
    float dt;      /* constant step, > 0 */
    float cone;    /* growing step factor, >= 0 */
    float dt_min;  /* growing step floor, > 0 */
} ogv_step;

/* Opaque grid: a dense bitfield (the plain method) or a VDB tree. */
typedef struct ogv_grid ogv_grid;

typedef struct {
    int32_t kind;          /* 0 dense bitfield, 1 VDB tree */
    int32_t n_levels, res, internal_log2;
    int64_t bytes;         /* device bytes the representation occupies */
    int64_t n_nodes, n_leaves;
    int64_t n_tiles_full, n_tiles_empty;           /* internal-node slots */
    int64_t n_root_tiles_full, n_root_tiles_empty; /* root cells */
} ogv_grid_info;

/* Dense bitfield of the occupancy grid, 1 bit per voxel (the paper's OG,
 * Sec. 1 and Tab. 3: 256 KiB at 128^3).
 *   n_levels  1..OGV_MAX_LEVELS cascades, finest first; res 1..OGV_MAX_RES.
 *   boxes_host [n_levels][6] (min x,y,z, max x,y,z), each level's planes
 *             nested inside the next level's (checked).
 *   occ_dev   uint8 [n_levels][res][res][res], x slowest, z fastest, nonzero
 *             = occupied; read during the call's kernels only.
 *   *out      receives the handle.  The build's kernels run on `stream`,
 *             and the call synchronizes `stream` once before returning (the
 *             occupancy may be freed and the handle used on any stream as
 *             soon as the call returns). */
ogv_status ogv_dense_build(int32_t n_levels, int32_t res, const float *boxes_host, const uint8_t *occ_dev,
                           ogv_grid **out, void *stream);

/* The dense bitfield plus, per voxel, its Chebyshev (chessboard) distance to
 * the nearest occupied voxel of its level, capped at 16 (uint8 [L][R][R][R]).
 * Sampling on it skips, from an empty voxel at distance d >= 2, the whole
 * cube of voxels within d - 1 in one step: the distance-field skipping the
 * paper discusses as an alternative and does not evaluate (Sec. 2.3, Fig. 1;
 * it notes the memory cost, here one byte per voxel).  Its
 * samples are the dense and VDB grids' exactly.  Batches march it by its
 * bitfield.  Same arguments, errors and synchronization as ogv_dense_build
 * (the call synchronizes `stream` once before returning). */
ogv_status ogv_dist_build(int32_t n_levels, int32_t res, const float *boxes_host, const uint8_t *occ_dev,
                          ogv_grid **out, void *stream);

/* Copies a distance grid's capped distances (uint8 [L][R][R][R], 0 for an
 * occupied voxel) to out_dev; OGV_ERR_INVALID for other grids. */
ogv_status ogv_grid_distances(const ogv_grid *grid, uint8_t *out_dev, void *stream);

/* VDB tree of the occupancy grid (Sec. 3): per level a dense root table of
 * internal nodes, each covering 2^internal_log2 leaf blocks of 8^3 voxels
 * per axis, with child and value bitmasks; 8^3 leaves hold 512-bit masks.
 * Uniform blocks are pruned into tiles (all empty -> empty tile, all
 * occupied -> full tile), and the same one level up (a node whose slots are
 * all empty or all full tiles becomes a root tile).  Voxels outside the grid
 * count as empty.  internal_log2 in 1..5.  Other arguments as
 * ogv_dense_build.  Synchronizes `stream` once (to size the tree). */
ogv_status ogv_vdb_build(int32_t n_levels, int32_t res, const float *boxes_host, const uint8_t *occ_dev,
                         int32_t internal_log2, ogv_grid **out, void *stream);

/* Structure counts and bytes; synchronizes the grid's build stream. */
ogv_status ogv_grid_info_get(const ogv_grid *grid, ogv_grid_info *info_host);

/* Decodes the grid back into occ_out_dev (uint8 [L][R][R][R], 0/1). */
ogv_status ogv_grid_to_dense(const ogv_grid *grid, uint8_t *occ_out_dev, void *stream);

void ogv_grid_destroy(ogv_grid *grid);

/* Re-derives a grid from a new occupancy occ_dev of the same shape (levels,
 * resolution, boxes and, for a VDB, internal node size are kept), in place
 * and asynchronously on the stream: no allocation and no host
 * synchronization, so a training loop can refresh its grid every few steps
 * (the paper's GPU tree is read-only and left this as future work, Sec. 5).
 * A VDB is rebuilt by the build's own kernels into the storage it was given
 * for the worst case, re-classifying every 8^3 block (R^3 bytes read); the
 * build's scratch stays with the grid for this.  Sampling calls on the same
 * stream see the new grid; calls on other streams must be ordered by the
 * caller, and no other call may use the grid while a refresh runs.  After a
 * refresh, ogv_grid_info_get waits for this stream.  OGV_ERR_INVALID on null
 * arguments. */
ogv_status ogv_grid_refresh(ogv_grid *grid, const uint8_t *occ_dev, void *stream);

/* Refreshes a grid from a density cache (Sec. 2.1: the occupancy grid
 * caches the densities the field predicts during training, and samples come
 * from the voxels whose cached density exceeds a threshold; the paper's
 * training refreshes it every 16 iterations, Sec. 4.1, and names low-cost
 * pruning on the GPU as future work, Sec. 5).  In place and asynchronous on
 * the stream, no allocation and no host synchronization.
 *   cache_dev    float32 [n_levels][res][res][res] (the grid's layout),
 *                caller-owned.  With density_dev non-null every entry is
 *                first updated in place to max(decay*cache, density): one
 *                binary32 product, then density when it is larger, else the
 *                product.  Entries must not be NaN.
 *   density_dev  nullable float32, same layout: the field's new densities.
 *   decay        in [0, 1] (checked only when density_dev is given).
 *   threshold    a voxel is occupied when its (updated) cache value is
 *                greater than this.
 *   changed_dev  nullable int32 [2], written on the stream: [0] the number
 *                of voxels whose occupancy changed, [1] 1 if the VDB tree's
 *                structure changed (some 8^3 block became empty, full or
 *                mixed), else 0 (always 0 for other grids).
 * The threshold is fused into the pass that classifies the 8^3 blocks, which
 * also compares each block's bits with the previous ones.  A VDB tree is
 * renumbered and rewritten only when some block changed kind; otherwise
 * just the leaves whose bits changed are rewritten.  Ordering and the use of
 * ogv_grid_info_get afterwards as for ogv_grid_refresh.  OGV_ERR_INVALID on
 * null grid or cache, a decay outside [0, 1] or a NaN threshold. */
ogv_status ogv_grid_refresh_density(ogv_grid *grid, float *cache_dev, const float *density_dev, float decay,
                                    float threshold, int32_t *changed_dev, void *stream);

/* Workspace bytes a sample call needs for n_rays rays and this lattice.
 * With a growing step (OGV_STEP_CONE) the workspace also keeps the lattice's
 * point table between calls, beside a header with near, far, cone, dt_min,
 * the table's length and a 64-bit hash of its entries.  A call on the same
 * workspace whose parameters match the header, and whose table still hashes
 * to it, reuses the table; any other call rebuilds it (a sequential pass of
 * about 50 ns per lattice point).  The caller may overwrite the workspace
 * between calls (except between a count and its fill); it only costs the
 * rebuild. */
ogv_status ogv_sample_workspace_size(int64_t n_rays, float near_t, float far_t, const ogv_step *step_host,
                                     size_t *bytes_host);

/* Counting pass (Alg. 1/Alg. 2 without emission): per-ray sample counts and
 * their exclusive scan.
 *   origins_dev, dirs_dev  float32 [n_rays][3].
 *   near_t, far_t          the ray-parameter range [t_min, t_max]; finite,
 *                          near_t >= 0; far_t < near_t gives no samples.
 *   offsets_dev            int64 [n_rays + 1] out: offsets[i] = first
 *                          sample of ray i, offsets[n_rays] = total.
 *   ws_dev, ws_bytes       workspace of ogv_sample_workspace_size bytes.
 * Dense grids march voxels; VDB grids use the hierarchical DDA. */
ogv_status ogv_sample_count(const ogv_grid *grid, const ogv_sample_opts *opts, const float *origins_dev, const float *dirs_dev,
                            int64_t n_rays, float near_t, float far_t, const ogv_step *step_host,
                            int64_t *offsets_dev, void *ws_dev, size_t ws_bytes, void *stream);

/* The two halves of ogv_sample_count, for callers that time or schedule
 * them apart: ogv_sample_count_raw walks the rays and leaves the per-ray
 * counts and runs in the workspace (same arguments as ogv_sample_count,
 * without offsets); ogv_sample_scan then writes offsets_dev (int64
 * [n_rays + 1]) from those counts.  n_rays must equal the count call's, and
 * ws_bytes must be at least that call's workspace size. */
ogv_status ogv_sample_count_raw(const ogv_grid *grid, const ogv_sample_opts *opts, const float *origins_dev,
                                const float *dirs_dev, int64_t n_rays, float near_t, float far_t,
                                const ogv_step *step_host, void *ws_dev, size_t ws_bytes, void *stream);
ogv_status ogv_sample_scan(int64_t n_rays, int64_t *offsets_dev, void *ws_dev, size_t ws_bytes, void *stream);

/* Emission pass: writes ray i's samples at offsets[i] .. offsets[i+1]-1.
 *   offsets_dev       from ogv_sample_count with the same arguments.
 *   ws_dev            the workspace that ogv_sample_count filled, unchanged
 *                     since: it holds each ray's occupied runs (and the
 *                     growing-step table), which this pass expands.
 *   capacity          length of the sample arrays; samples at index >=
 *                     capacity are not written.
 *   ray_ids_dev int32 [capacity], t0_dev/t1_dev float32 [capacity].
 *   voxel_ids_dev     nullable int32 [capacity]: ((l*R+i)*R+j)*R+k of the
 *                     voxel owning t0 (debug/parity output, slower); needs
 *                     n_levels * res^3 <= 2^31, else OGV_ERR_UNSUPPORTED. */
ogv_status ogv_sample_fill(const ogv_grid *grid, const ogv_sample_opts *opts, const float *origins_dev, const float *dirs_dev,
                           int64_t n_rays, float near_t, float far_t, const ogv_step *step_host,
                           const int64_t *offsets_dev, int64_t capacity, int32_t *ray_ids_dev, float *t0_dev,
                           float *t1_dev, int32_t *voxel_ids_dev, void *ws_dev, size_t ws_bytes, void *stream);

/* Count + scan + emission in one asynchronous call with no host round trip
 * (capacity mode): offsets_dev as in ogv_sample_count; samples beyond
 * `capacity` are dropped and *overflow_dev (int32) is set to 1, else 0.
 * The caller reads offsets[n_rays] to learn the total. */
ogv_status ogv_sample_rays(const ogv_grid *grid, const ogv_sample_opts *opts, const float *origins_dev, const float *dirs_dev,
                           int64_t n_rays, float near_t, float far_t, const ogv_step *step_host,
                           int64_t *offsets_dev, int64_t capacity, int32_t *ray_ids_dev, float *t0_dev,
                           float *t1_dev, int32_t *voxel_ids_dev, int32_t *overflow_dev, void *ws_dev,
                           size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * ogv_sample_rays with the workspace taken from a static per-device array of
 * OGV_NOALLOC_SCRATCH_BYTES (64 MiB) inside the library instead of an
 * argument.  The call allocates nothing; the caller still passes every input
 * and output, with the meaning ogv_sample_rays gives them.  The array is
 * reserved on each device the library runs on and held until the process
 * ends.  A call whose workspace (ogv_sample_workspace_size) exceeds it --
 * about 440,000 rays at a constant step -- fails with OGV_ERR_CAPACITY and
 * does nothing.  All calls on one device share its array: calls that
 * overlap in time on one device (other host threads, other streams) race,
 * so the caller orders them, e.g. on one stream. */
#define OGV_NOALLOC_SCRATCH_BYTES (64u << 20)
ogv_status ogv_sample_rays_noalloc(const ogv_grid *grid, const ogv_sample_opts *opts, const float *origins_dev,
                                   const float *dirs_dev, int64_t n_rays, float near_t, float far_t,
                                   const ogv_step *step_host, int64_t *offsets_dev, int64_t capacity,
                                   int32_t *ray_ids_dev, float *t0_dev, float *t1_dev, int32_t *voxel_ids_dev,
                                   int32_t *overflow_dev, void *stream);

/* Volume-rendering composite over packed samples (the accumulation of
 * Sec. 1; emission-absorption quadrature): per ray, dt_i = t1_i - t0_i,
 * alpha_i = 1 - exp(-sigma_i dt_i), T_i = exp(-sum_{j<i} sigma_j dt_j),
 * w_i = T_i alpha_i, rgb = sum w_i c_i, opacity = sum w_i.
 *   offsets_dev int64 [n_rays+1]; t0/t1/sigma float32 [S]; rgb float32 [S][3].
 *   out_rgb_dev float32 [n_rays][3], out_opacity_dev float32 [n_rays]. */
ogv_status ogv_composite_fwd(const int64_t *offsets_dev, int64_t n_rays, const float *t0_dev, const float *t1_dev,
                             const float *sigma_dev, const float *rgb_dev, float *out_rgb_dev,
                             float *out_opacity_dev, void *stream);

/* Backward of ogv_composite_fwd: given g_rgb (float32 [n_rays][3]) and
 * g_opacity (float32 [n_rays], nullable = zero), writes
 * d_sigma_i = dt_i (g_rgb . (T_{i+1} c_i - sum_{k>i} w_k c_k) + g_opacity T_n)
 * and d_rgb_i = w_i g_rgb (float32 [S] and [S][3]), S = n_samples, the length
 * of the sample arrays (>= offsets[n_rays]).  Samples no ray owns (before
 * offsets[0] or from offsets[n_rays] on) get zero, so the outputs need no
 * clearing beforehand. */
ogv_status ogv_composite_bwd(const int64_t *offsets_dev, int64_t n_rays, int64_t n_samples, const float *t0_dev,
                             const float *t1_dev, const float *sigma_dev, const float *rgb_dev, const float *g_rgb_dev,
                             const float *g_opacity_dev, float *d_sigma_dev, float *d_rgb_dev, void *stream);

/* A synthetic radiance field: K Gaussian blobs (1 <= K <= OGV_MAX_BLOBS).
 * At a point x, g_k = exp(-|x - centre_k|^2 / (2 radius_k^2)),
 * sigma(x) = sum_k density_k g_k and colour(x) = sum_k density_k g_k
 * colour_k / sigma(x) (0 where sigma is 0).  It stands in for the trained
 * field that the sampler's points are fed to (Sec. 1); the paper's networks
 * and weights are not part of this library. */
#define OGV_MAX_BLOBS 16
typedef struct {
    int32_t n;
    float centre[OGV_MAX_BLOBS][3];
    float radius[OGV_MAX_BLOBS];   /* > 0 */
    float density[OGV_MAX_BLOBS];  /* >= 0 */
    float colour[OGV_MAX_BLOBS][3];
} ogv_blob_field;

/* Renders packed samples through a blob field in one pass: each sample's
 * field value is taken at its interval midpoint o + d (t0 + t1) / 2 and
 * composited as in ogv_composite_fwd (density and colour are never stored).
 *   offsets_dev int64 [n_rays+1]; origins_dev, dirs_dev float32 [n_rays][3];
 *   t0_dev, t1_dev float32 [S]; field_host read during the call only.
 *   out_rgb_dev float32 [n_rays][3], out_opacity_dev float32 [n_rays]
 *   (nullable).  Errors: OGV_ERR_INVALID on null pointers, n_rays < 0, a
 *   blob count outside 1..OGV_MAX_BLOBS, a radius <= 0 or a density < 0. */
ogv_status ogv_render_blobs(const int64_t *offsets_dev, int64_t n_rays, const float *origins_dev,
                            const float *dirs_dev, const float *t0_dev, const float *t1_dev,
                            const ogv_blob_field *field_host, float *out_rgb_dev, float *out_opacity_dev,
                            void *stream);

/* ---------------------------------------------------------------- batches
 * Many scenes, uneven grids and ray counts, in one graph-captured pass: a
 * persistent counting kernel pulls chunks of rays from a queue that spans
 * all scenes, one scan numbers every sample, and one expansion kernel
 * writes them.  Not in the paper (it renders one scene at a time); the
 * per-ray result is exactly ogv_sample_rays's. */
typedef struct {
    const ogv_grid *grid;                /* dense or VDB, built on this device */
    const float *origins_dev, *dirs_dev; /* float32 [n_rays][3] */
    int64_t n_rays;
    float near_t, far_t;
    ogv_step step;
    int32_t image_width;                 /* as in ogv_sample_opts */
} ogv_scene;

typedef struct {
    int32_t chunk;          /* rays per queue item, a multiple of 256 */
    int32_t blocks_per_cu;  /* persistent workgroups (256 threads) per compute unit */
} ogv_tune;

typedef struct ogv_batch ogv_batch;

typedef struct {
    int64_t n_rays;         /* all scenes' rays; scene s starts at ray_base[s] */
    int32_t n_scenes;
    ogv_tune tune;          /* the choice in use */
    int32_t tuned;          /* 1 if chosen by the autotuner */
    float tune_ms;          /* counting time of the chosen tune when tuned */
} ogv_batch_info;

/* Plans a batched pass over scenes_host[0..n_scenes-1] (1..64 scenes; the
 * descriptors are copied, the grids and ray buffers must stay alive and
 * unchanged while the batch is used).  tune_host NULL runs the autotuner:
 * every candidate queue chunk and persistent grid size is timed on `stream`
 * (this synchronizes) and the fastest kept.  The batch owns its workspace. */
ogv_status ogv_batch_create(const ogv_scene *scenes_host, int32_t n_scenes, int32_t variant,
                            const ogv_tune *tune_host, ogv_batch **out, void *stream);

ogv_status ogv_batch_info_get(const ogv_batch *batch, ogv_batch_info *info_host, int64_t *ray_base_host);

/* One pass, replayed from a captured HIP graph (captured on first use and
 * again whenever the output pointers or capacity change).  Outputs form one
 * CSR over the scenes' rays concatenated in scene order: offsets_dev int64
 * [n_rays + 1]; ray_ids are global ray indices (scene s, ray i ->
 * ray_base[s] + i); capacity and overflow_dev as in ogv_sample_rays. */
ogv_status ogv_batch_launch(ogv_batch *batch, int64_t *offsets_dev, int64_t capacity, int32_t *ray_ids_dev,
                            float *t0_dev, float *t1_dev, int32_t *overflow_dev, void *stream);

/* The same pass as plain kernel launches, no graph (for comparison). */
ogv_status ogv_batch_launch_eager(ogv_batch *batch, int64_t *offsets_dev, int64_t capacity, int32_t *ray_ids_dev,
                                  float *t0_dev, float *t1_dev, int32_t *overflow_dev, void *stream);

void ogv_batch_destroy(ogv_batch *batch);

/* Message for the last non-OK status returned on the calling thread. */
const char *ogv_last_error(void);

/* Library version string. */
const char *ogv_version(void);

#ifdef __cplusplus
}
#endif

#endif /* OGVDB_H */
