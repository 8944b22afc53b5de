// Batched sampling of many scenes in one pass (not in the paper, which
// renders one scene at a time): uneven grids and ray counts share
//   reset    the queue head (a kernel, so the pass can be graph-captured)
//   count    a persistent kernel: each workgroup pulls the next chunk of
//            rays from a queue spanning every scene and counts them
//   scan     one exclusive scan over all rays
//   expand   coalesced expansion of the kept runs, each on its scene's lattice
//   fill     traversal fill of rays with more runs than the count pass keeps
// The queue chunk and persistent grid size come from an autotuner that times
// the candidates; the pass is captured into a HIP graph and replayed.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "geometry.hpp"
#include "internal.hpp"
#include "scan.hpp"
#include "trace.hpp"

namespace ogv {
namespace {

constexpr int kMaxScenes = 64;
static_assert(kMaxScenes <= kBlock, "the expansion stages every scene's lattice, one per thread");

struct SceneDesc {
    GridView g;
    const float *o, *d;
    int64_t n;       // rays of the scene
    int64_t nt;      // threads walking them (more than n when image-tiled)
    int64_t first;   // its first global ray
    int64_t item0;   // its first queue item
    Lattice lat;
    int32_t width;   // image width for 8x8 tiling, 0 for none
    int32_t lds;     // 1: the walk stages its tree's tables in LDS (they fit the launch's share)
};

// LDS a walk block may give a scene's staged tree tables: eight such blocks
// fit a compute unit's 160 KiB (the autotuner tries up to eight per CU).
// A 128^3 grid with 16^3-slot nodes needs 16 KiB and a few bytes; larger
// trees are read from global memory.
constexpr size_t kBatchTreeLds = 19 * 1024;

// zeroes the queue head, the run-pool head and the lost-ray count
// (queue[0], queue[1], queue[2])
__global__ void batch_reset_kernel(int32_t *queue) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        queue[0] = 0;
        queue[1] = 0;
        queue[2] = 0;
    }
}

__device__ __forceinline__ int scene_of_item(const SceneDesc *scenes, int n, int64_t item) {
    int s = 0;
    while (s + 1 < n && scenes[s + 1].item0 <= item) ++s;
    return s;
}

// The descriptors are in queue order, not in ray order: search them all.
__device__ __forceinline__ int scene_of_ray(const SceneDesc *scenes, int n, int64_t gr) {
    for (int s = 0; s < n; ++s)
        if (gr >= scenes[s].first && gr < scenes[s].first + scenes[s].n) return s;
    return 0;
}

// Threads tr in [r0, r1) of one queue item walk their rays with `tree`.
template <bool kSkip>
__device__ __forceinline__ void count_item(const SceneDesc *sc, const Tree &tree, int64_t r0, int64_t r1,
                                           int32_t *__restrict__ counts, int32_t *__restrict__ nruns,
                                           const RunPool &pool) {
    const Lattice lat = sc->lat;
    const GridView g = sc->g;
    const CountCtx ctx{lat, pool};
    for (int64_t tr = r0 + threadIdx.x; tr < r1; tr += kBlock) {
        const int64_t r = ray_of_thread(tr, sc->n, sc->width);
        if (r < 0) continue;
        float o[3], d[3];
        load_ray(sc->o, sc->d, r, o, d);
        const int64_t gr = sc->first + r;
        CountVis vis = make_count_vis(gr, pool);
        // batches march a distance grid (kind 2) by its bitfield, as a dense grid
        if (g.kind == 1) trace_ray<1, kSkip>(g, tree, o, d, lat, vis, ctx);
        else trace_ray<0, kSkip>(g, tree, o, d, lat, vis, ctx);
        vis.finish(ctx);
        counts[gr] = vis.n;
        nruns[gr] = vis.nr;
    }
}

// Persistent: every workgroup loops pulling items until the queue runs dry,
// so every wave reaches the exit once n_items items are handed out.  The
// queue hands out a scene's items one after another, so a block mostly takes
// several items of one scene in a row: a scene whose tree fits (lds) has its
// tables staged in LDS when a block's item is its first of that scene, and
// read from there.  The block's barrier after taking an item means every
// thread has finished the previous item before the tables are overwritten.
// The Alg. 1 loop asks for at least 5 waves per SIMD (at -O3 the compiler
// would settle at 4 with 108 VGPRs; 5 spilled 20 registers and measured 4.8%
// faster on the 16-scene pass).  This file's -O1 build fits the walk in 80
// VGPRs with no spills, six waves per SIMD.
template <bool kSkip>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kSkip ? 1 : 5)))
batch_count_kernel(const SceneDesc *__restrict__ scenes, int n_scenes, int64_t n_items, int chunk,
                   int32_t *__restrict__ queue, int32_t *__restrict__ counts, int32_t *__restrict__ nruns,
                   RunPool pool) {
    extern __shared__ __align__(16) uint32_t smem[];
    __shared__ int32_t s_item;
    int staged = -1;   // scene whose tables are in smem (the same in every thread)
    while (true) {
        if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
        __syncthreads();
        const int64_t item = s_item;
        __syncthreads();
        if (item >= n_items) return;
        const int si = scene_of_item(scenes, n_scenes, item);
        const SceneDesc *sc = scenes + si;
        const int64_t r0 = (item - sc->item0) * (int64_t)chunk;
        const int64_t r1 = min(r0 + (int64_t)chunk, sc->nt);
        if (sc->lds) {
            if (si != staged) {
                stage_tree(sc->g, smem);
                staged = si;
            }
            count_item<kSkip>(sc, tree_in_lds(sc->g, smem), r0, r1, counts, nruns, pool);
        } else {
            count_item<kSkip>(sc, load_tree<false>(sc->g, nullptr), r0, r1, counts, nruns, pool);
        }
    }
}

// Traversal fill of the rays whose runs were lost, each on its scene's grid
// and lattice; the blocks of the launch stride through the list.
template <bool kSkip>
__device__ __forceinline__ void batch_fill_lost(const SceneDesc *__restrict__ scenes, int n_scenes,
                                                const int32_t *__restrict__ lost, const int32_t *__restrict__ n_lost,
                                                const int64_t *__restrict__ offsets, int64_t capacity,
                                                int32_t *__restrict__ ray_ids, float *__restrict__ t0,
                                                float *__restrict__ t1) {
    const int64_t m = *n_lost;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < m; k += (int64_t)gridDim.x * kBlock) {
        const int64_t gr = lost[k];
        const int64_t first_out = offsets[gr];
        if (first_out >= capacity) continue;
        const SceneDesc *sc = scenes + scene_of_ray(scenes, n_scenes, gr);
        const Lattice lat = sc->lat;
        const GridView g = sc->g;
        const Tree tree = load_tree<false>(g, nullptr);
        float o[3], d[3];
        load_ray(sc->o, sc->d, gr - sc->first, o, d);
        const FillCtx ctx{lat, capacity, ray_ids, t0, t1, nullptr, g.R};
        FillVis<false> vis;
        vis.idx = first_out;
        vis.ray = (int32_t)gr;
        vis.lev = 0;
        if (g.kind == 1) trace_ray<1, kSkip>(g, tree, o, d, lat, vis, ctx);
        else trace_ray<0, kSkip>(g, tree, o, d, lat, vis, ctx);
    }
}

// Expansion of the kept runs, then, in the same launch, the traversal fill of
// the lost rays (their outputs are disjoint from the expansion's).
template <bool kSkip>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kExpandWaves))) batch_expand_kernel(const int64_t *__restrict__ offsets, int64_t n_total,
                                                              const int32_t *__restrict__ nruns, RunReader rd,
                                                              const Lattice *__restrict__ lats,
                                                              const int64_t *__restrict__ first, int n_scenes,
                                                              int64_t capacity, int32_t *__restrict__ ray_ids,
                                                              float *__restrict__ t0, float *__restrict__ t1, int vec4,
                                                              const SceneDesc *__restrict__ scenes,
                                                              const int32_t *__restrict__ lost,
                                                              const int32_t *__restrict__ n_lost) {
    // the offsets are read only (no scan inside the expansion)
    expand_block(const_cast<int64_t *>(offsets), ChunkScan{}, n_total, nruns, rd, SceneLattices{lats, first, n_scenes},
                 capacity, ray_ids, t0, t1, vec4 != 0);
    batch_fill_lost<kSkip>(scenes, n_scenes, lost, n_lost, offsets, capacity, ray_ids, t0, t1);
}


// growing-step lattice of one scene (one thread), padded past its length
__global__ void batch_cone_table_kernel(float tmin, float tmax, float cone, float dt_min, float *tab, int32_t cap) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    float t = tmin;
    int32_t k = 0;
    while (k < cap) {
        tab[k++] = t;
        if (t > tmax) break;
        float grow = __fmul_rn(t, cone);
        float step = grow > dt_min ? grow : dt_min;
        t = __fadd_rn(t, step);
    }
    const float last = tab[k - 1];
    for (int32_t j = k; j < cap; ++j) tab[j] = last;
}

}  // namespace
}  // namespace ogv

using namespace ogv;

struct ogv_batch {
    int n_scenes = 0, variant = 0, n_cu = 0;
    std::vector<SceneDesc> desc;   // host copy (item0 depends on the chunk)
    std::vector<int64_t> ray_base;
    int64_t n_total = 0, n_items = 0, n_tiles = 0;
    size_t tree_lds = 0;   // dynamic LDS of the walk: the largest staged tree
    ogv_tune tune{0, 0};
    bool tuned = false;
    float tune_ms = 0.0f;
    void *mem = nullptr;
    SceneDesc *desc_dev = nullptr;
    Lattice *lats_dev = nullptr;
    int64_t *first_dev = nullptr;
    int32_t *counts = nullptr, *nruns = nullptr, *queue = nullptr;
    RunPool pool{};
    int64_t *tiles = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // outputs the captured graph writes
    int64_t *g_offsets = nullptr;
    int64_t g_capacity = -1;
    int32_t *g_ids = nullptr, *g_overflow = nullptr;
    float *g_t0 = nullptr, *g_t1 = nullptr;
};

namespace {

hipError_t upload_desc(ogv_batch *b, int chunk, hipStream_t s) {
    int64_t item = 0;
    for (SceneDesc &d : b->desc) {
        d.item0 = item;
        item += (d.nt + chunk - 1) / chunk;
    }
    b->n_items = item;
    hipError_t e = hipMemcpyAsync(b->desc_dev, b->desc.data(), sizeof(SceneDesc) * b->n_scenes,
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

void enqueue_count(ogv_batch *b, const ogv_tune &t, hipStream_t s) {
    batch_reset_kernel<<<1, 64, 0, s>>>(b->queue);
    unsigned grid = (unsigned)std::max(1, b->n_cu * t.blocks_per_cu);
    if (b->variant == OGV_SKIP)
        batch_count_kernel<true><<<grid, kBlock, b->tree_lds, s>>>(b->desc_dev, b->n_scenes, b->n_items, t.chunk,
                                                                   b->queue, b->counts, b->nruns, b->pool);
    else
        batch_count_kernel<false><<<grid, kBlock, b->tree_lds, s>>>(b->desc_dev, b->n_scenes, b->n_items, t.chunk,
                                                                    b->queue, b->counts, b->nruns, b->pool);
}

hipError_t enqueue_pass(ogv_batch *b, int64_t *offsets, int64_t capacity, int32_t *ids, float *t0, float *t1,
                        int32_t *overflow, hipStream_t s) {
    enqueue_count(b, b->tune, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_excl_scan(b->counts, b->n_total, offsets, b->tiles, capacity, overflow, s);
    if (e != hipSuccess || capacity == 0) return e;
    const unsigned blocks = (unsigned)min(expand_items(b->n_total), (int64_t)INT32_MAX);
    const RunReader rd{b->pool.slots, b->pool.stride, b->pool.ray_next, b->pool.chunks, b->pool.chunk_next};
    const int vec4 = (((uintptr_t)ids | (uintptr_t)t0 | (uintptr_t)t1) & 15) == 0;
    if (b->variant == OGV_SKIP)
        batch_expand_kernel<true><<<blocks, kBlock, 0, s>>>(offsets, b->n_total, b->nruns, rd, b->lats_dev,
                                                            b->first_dev, b->n_scenes, capacity, ids, t0, t1, vec4,
                                                            b->desc_dev, b->pool.lost, b->pool.n_lost);
    else
        batch_expand_kernel<false><<<blocks, kBlock, 0, s>>>(offsets, b->n_total, b->nruns, rd, b->lats_dev,
                                                             b->first_dev, b->n_scenes, capacity, ids, t0, t1, vec4,
                                                             b->desc_dev, b->pool.lost, b->pool.n_lost);
    return hipGetLastError();
}

void release(ogv_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->mem) (void)hipFree(b->mem);
    delete b;
}

// time the counting stage of one tune: best of `reps` after one warm-up
ogv_status time_tune(ogv_batch *b, const ogv_tune &t, hipStream_t s, float *ms_out) {
    OGV_CHECK_HIP(upload_desc(b, t.chunk, s));
    hipEvent_t e0, e1;
    OGV_CHECK_HIP(hipEventCreate(&e0));
    OGV_CHECK_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
        (void)hipEventRecord(e0, s);
        enqueue_count(b, t, s);
        (void)hipEventRecord(e1, s);
        hipError_t e = hipEventSynchronize(e1);
        if (e != hipSuccess) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            OGV_FAIL(OGV_ERR_HIP, std::string("autotune run failed: ") + hipGetErrorString(e));
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) best = std::min(best, ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_out = best;
    return OGV_OK;
}

}  // namespace

extern "C" ogv_status ogv_batch_create(const ogv_scene *scenes, int32_t n, int32_t variant, const ogv_tune *tune,
                                       ogv_batch **out, void *stream) {
    if (!out) OGV_FAIL(OGV_ERR_INVALID, "out is null");
    *out = nullptr;
    if (!scenes || n < 1 || n > kMaxScenes) OGV_FAIL(OGV_ERR_INVALID, "need 1..64 scenes");
    if (variant != OGV_BRANCH && variant != OGV_SKIP) OGV_FAIL(OGV_ERR_INVALID, "variant must be 0 or 1");
    if (tune && (tune->chunk < kBlock || tune->chunk % kBlock != 0 || tune->blocks_per_cu < 1 ||
                 tune->blocks_per_cu > 64))
        OGV_FAIL(OGV_ERR_INVALID, "tune: chunk must be a positive multiple of 256, blocks_per_cu in 1..64");
    hipStream_t s = (hipStream_t)stream;
    ogv_batch *b = new ogv_batch();
    b->n_scenes = n;
    b->variant = variant;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        release(b);
        OGV_FAIL(OGV_ERR_HIP, "cannot query the device");
    }
    // validate every scene and size the workspace
    std::vector<int32_t> tab_cap(n, 0);
    size_t tab_words = 0;
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
        const ogv_scene &sc = scenes[i];
        std::string pre = "scene " + std::to_string(i) + ": ";
        ogv_status st = validate_sampling(sc.grid, variant, sc.origins_dev, sc.dirs_dev, sc.n_rays, sc.near_t,
                                          sc.far_t, &sc.step, pre.c_str());
        if (st != OGV_OK) {
            release(b);
            return st;
        }
        if (sc.image_width < 0) {
            release(b);
            OGV_FAIL(OGV_ERR_INVALID, pre + "image_width < 0");
        }
        tab_cap[i] = cone_table_capacity(sc.near_t, sc.far_t, &sc.step);
        tab_words += (size_t)std::max(tab_cap[i], 0);
        b->ray_base.push_back(total);
        total += sc.n_rays;
    }
    if (total > (int64_t)INT32_MAX) {
        release(b);
        OGV_FAIL(OGV_ERR_UNSUPPORTED, "more than 2^31-1 rays in one batch");
    }
    b->n_total = total;
    b->n_tiles = scan_tiles(total);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    size_t o_desc = take(sizeof(SceneDesc) * n);
    size_t o_lats = take(sizeof(Lattice) * n);
    size_t o_first = take(sizeof(int64_t) * (n + 1));
    size_t o_queue = take(sizeof(int32_t) * 4);
    size_t o_counts = take(sizeof(int32_t) * (size_t)total);
    size_t o_nruns = take(sizeof(int32_t) * (size_t)total);
    size_t o_runs = take(sizeof(int2) * (size_t)total * kMaxRuns);
    size_t o_next = take(sizeof(int32_t) * (size_t)total);
    const int32_t pool_cap = (int32_t)std::min<int64_t>(std::max<int64_t>(256, total / 16), 1 << 24);
    size_t o_chunks = take(sizeof(int2) * (size_t)pool_cap * kMaxRuns);
    size_t o_cnext = take(sizeof(int32_t) * (size_t)pool_cap);
    size_t o_lost = take(sizeof(int32_t) * (size_t)total);
    size_t o_tiles = take(sizeof(int64_t) * (size_t)(b->n_tiles + 1));
    size_t o_tabs = take(sizeof(float) * tab_words);
    if (hipMalloc(&b->mem, off) != hipSuccess) {
        b->mem = nullptr;
        release(b);
        OGV_FAIL(OGV_ERR_OOM, "device allocation of " + std::to_string(off) + " bytes failed");
    }
    char *m = (char *)b->mem;
    b->desc_dev = (SceneDesc *)(m + o_desc);
    b->lats_dev = (Lattice *)(m + o_lats);
    b->first_dev = (int64_t *)(m + o_first);
    b->queue = (int32_t *)(m + o_queue);
    b->counts = (int32_t *)(m + o_counts);
    b->nruns = (int32_t *)(m + o_nruns);
    b->pool.slots = (int2 *)(m + o_runs);
    b->pool.stride = total;
    b->pool.ray_next = (int32_t *)(m + o_next);
    b->pool.chunks = (int2 *)(m + o_chunks);
    b->pool.chunk_next = (int32_t *)(m + o_cnext);
    b->pool.head = b->queue + 1;
    b->pool.cap = pool_cap;
    b->pool.lost = (int32_t *)(m + o_lost);
    b->pool.n_lost = b->queue + 2;
    b->tiles = (int64_t *)(m + o_tiles);
    float *tabs = (float *)(m + o_tabs);
    std::vector<Lattice> lats(n);
    std::vector<int64_t> first(n + 1);
    size_t tab_at = 0;
    for (int i = 0; i < n; ++i) {
        const ogv_scene &sc = scenes[i];
        SceneDesc d;
        std::memset(&d, 0, sizeof(d));
        d.g = sc.grid->view;
        d.o = sc.origins_dev;
        d.d = sc.dirs_dev;
        d.n = sc.n_rays;
        d.width = sc.image_width;
        d.nt = tiled_threads(sc.n_rays, sc.image_width);
        d.first = b->ray_base[i];
        const size_t tb = d.g.kind == 1 ? tree_lds_bytes(d.g.L, d.g.NR, d.g.S) : 0;
        d.lds = d.g.kind == 1 && tb <= kBatchTreeLds ? 1 : 0;
        if (d.lds) b->tree_lds = std::max(b->tree_lds, tb);
        Lattice &L = d.lat;
        L.tmin = sc.near_t;
        L.tmax = sc.far_t;
        L.dt = sc.step.dt;
        L.cone = sc.step.kind == OGV_STEP_CONE;
        L.tab = nullptr;
        L.n_tab = 0;
        if (L.cone && tab_cap[i] > 0) {
            L.tab = tabs + tab_at;
            L.n_tab = tab_cap[i];
            batch_cone_table_kernel<<<1, 64, 0, s>>>(sc.near_t, sc.far_t, sc.step.cone, sc.step.dt_min,
                                                     tabs + tab_at, tab_cap[i]);
            tab_at += (size_t)tab_cap[i];
        }
        b->desc.push_back(d);
        lats[i] = L;
        first[i] = d.first;
    }
    first[n] = total;
    // The queue hands out the scenes' chunks in order of decreasing per-ray
    // cost (resolution times levels: the cells a ray can cross), so the
    // scenes whose waves run longest start first instead of forming the
    // launch's tail; the output stays in scene order (each descriptor keeps
    // its first global ray).
    std::stable_sort(b->desc.begin(), b->desc.end(), [](const SceneDesc &x, const SceneDesc &y) {
        const int64_t cx = (int64_t)x.g.R * x.g.L, cy = (int64_t)y.g.R * y.g.L;
        return cx != cy ? cx > cy : x.n > y.n;
    });
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(b->lats_dev, lats.data(), sizeof(Lattice) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->first_dev, first.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipStreamCreate(&b->cap_stream);
    if (e != hipSuccess) {
        release(b);
        OGV_FAIL(OGV_ERR_HIP, std::string("batch setup failed: ") + hipGetErrorString(e));
    }
    if (tune) {
        b->tune = *tune;
        e = upload_desc(b, b->tune.chunk, s);
        if (e != hipSuccess) {
            release(b);
            OGV_FAIL(OGV_ERR_HIP, std::string("batch setup failed: ") + hipGetErrorString(e));
        }
    } else if (total > 0) {
        // autotune: queue chunk x persistent workgroups per compute unit
        const int chunks[] = {256, 512, 1024, 2048, 4096};
        const int per_cu[] = {2, 4, 8};
        float best = 1e30f;
        ogv_tune best_t{1024, 4};
        for (int c : chunks)
            for (int p : per_cu) {
                ogv_tune t{c, p};
                float ms = 0.0f;
                ogv_status st = time_tune(b, t, s, &ms);
                if (st != OGV_OK) {
                    release(b);
                    return st;
                }
                if (ms < best) {
                    best = ms;
                    best_t = t;
                }
            }
        b->tune = best_t;
        b->tuned = true;
        b->tune_ms = best;
        e = upload_desc(b, b->tune.chunk, s);
        if (e != hipSuccess) {
            release(b);
            OGV_FAIL(OGV_ERR_HIP, std::string("batch setup failed: ") + hipGetErrorString(e));
        }
    } else {
        b->tune = ogv_tune{1024, 4};
        (void)upload_desc(b, b->tune.chunk, s);
    }
    *out = b;
    return OGV_OK;
}

extern "C" ogv_status ogv_batch_info_get(const ogv_batch *b, ogv_batch_info *info, int64_t *ray_base) {
    if (!b || !info) OGV_FAIL(OGV_ERR_INVALID, "null argument");
    info->n_rays = b->n_total;
    info->n_scenes = b->n_scenes;
    info->tune = b->tune;
    info->tuned = b->tuned ? 1 : 0;
    info->tune_ms = b->tune_ms;
    if (ray_base)
        for (int i = 0; i < b->n_scenes; ++i) ray_base[i] = b->ray_base[i];
    return OGV_OK;
}

static ogv_status check_outputs(const ogv_batch *b, const int64_t *offsets, int64_t capacity, const int32_t *ids,
                                const float *t0, const float *t1, const int32_t *overflow) {
    if (!b) OGV_FAIL(OGV_ERR_INVALID, "batch is null");
    if (!offsets || !overflow) OGV_FAIL(OGV_ERR_INVALID, "offsets/overflow is null");
    if (capacity < 0) OGV_FAIL(OGV_ERR_INVALID, "capacity < 0");
    if (capacity > 0 && (!ids || !t0 || !t1)) OGV_FAIL(OGV_ERR_INVALID, "null sample array");
    return OGV_OK;
}

extern "C" ogv_status ogv_batch_launch_eager(ogv_batch *b, int64_t *offsets, int64_t capacity, int32_t *ids,
                                             float *t0, float *t1, int32_t *overflow, void *stream) {
    ogv_status st = check_outputs(b, offsets, capacity, ids, t0, t1, overflow);
    if (st != OGV_OK) return st;
    OGV_CHECK_HIP(enqueue_pass(b, offsets, capacity, ids, t0, t1, overflow, (hipStream_t)stream));
    return OGV_OK;
}

extern "C" ogv_status ogv_batch_launch(ogv_batch *b, int64_t *offsets, int64_t capacity, int32_t *ids, float *t0,
                                       float *t1, int32_t *overflow, void *stream) {
    ogv_status st = check_outputs(b, offsets, capacity, ids, t0, t1, overflow);
    if (st != OGV_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (!b->exec || b->g_offsets != offsets || b->g_capacity != capacity || b->g_ids != ids || b->g_t0 != t0 ||
        b->g_t1 != t1 || b->g_overflow != overflow) {
        if (b->exec) {
            (void)hipGraphExecDestroy(b->exec);
            b->exec = nullptr;
        }
        if (b->graph) {
            (void)hipGraphDestroy(b->graph);
            b->graph = nullptr;
        }
        OGV_CHECK_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_pass(b, offsets, capacity, ids, t0, t1, overflow, b->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            OGV_FAIL(OGV_ERR_HIP, std::string("graph capture failed: ") +
                                      hipGetErrorString(e != hipSuccess ? e : e2));
        }
        b->graph = g;
        OGV_CHECK_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->g_offsets = offsets;
        b->g_capacity = capacity;
        b->g_ids = ids;
        b->g_t0 = t0;
        b->g_t1 = t1;
        b->g_overflow = overflow;
    }
    OGV_CHECK_HIP(hipGraphLaunch(b->exec, s));
    return OGV_OK;
}

extern "C" void ogv_batch_destroy(ogv_batch *b) {
    if (b) release(b);
}
