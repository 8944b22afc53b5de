// Single-scene sampler: the count -> exclusive scan -> fill pipeline that
// packs every ray's samples into one CSR, over the ray walk of trace.hpp.
//
//   count   one ray per lane; per-ray sample count and occupied runs
//   scan    counts -> int64 offsets
//   fill    expansion of the kept runs with coalesced stores, plus a
//           traversal fill for rays with too many runs to keep (or for every
//           ray when voxel ids are requested)
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <mutex>
#include <string>

#include "geometry.hpp"
#include "internal.hpp"
#include "scan.hpp"
#include "count.hpp"
#include "trace.hpp"

namespace ogv {

// The Alg. 2 (skip) walks over a tree (hierarchical, voxel and sub-leaf
// steps) are instantiated in count_skip.hip.
#define OGV_COUNT_SKIP(V, L, L1)                                                                               \
    extern template __global__ void count_kernel<V, true, L, L1>(GridView, const float *, const float *, int64_t, \
                                                                 Lattice, int32_t *, int32_t *, RunPool, int,  \
                                                                 int64_t *, int64_t *);
OGV_COUNT_SKIP_ALL
#undef OGV_COUNT_SKIP

// ------------------------------------------------------------------ kernels

// Traversal fill: re-walks every ray and writes its samples from offsets[i]
// (used when voxel ids are requested; the expansion fill writes the rest).
template <int kGrid, bool kSkip, bool kVox, bool kLds>
__global__ void __launch_bounds__(kBlock) fill_kernel(GridView g, const float *__restrict__ origins,
                                                      const float *__restrict__ dirs, int64_t n_rays, Lattice lat,
                                                      const int64_t *__restrict__ offsets, int64_t capacity,
                                                      int32_t *__restrict__ ray_ids, float *__restrict__ t0,
                                                      float *__restrict__ t1, int32_t *__restrict__ vox) {
    extern __shared__ __align__(16) uint32_t smem[];
    Tree tree = reads_tree(kGrid) ? load_tree<kLds>(g, smem) : Tree{};
    const FillCtx ctx{lat, capacity, ray_ids, t0, t1, vox, g.R};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n_rays; i += (int64_t)gridDim.x * kBlock) {
        const int64_t first = offsets[i];
        if (first >= capacity) continue;
        float o[3], d[3];
        load_ray(origins, dirs, i, o, d);
        FillVis<kVox> vis;
        vis.idx = first;
        vis.ray = (int32_t)i;
        vis.lev = 0;
        trace_ray<kGrid, kSkip>(g, tree, o, d, lat, vis, ctx);
    }
}

// zeroes the pool head and the lost-ray count (head[0], head[1]) and the
// scan tile and chunk sums the count pass accumulates
__global__ void pool_reset_kernel(int32_t *head, int64_t *tile_sums, int64_t n_tiles, int64_t *chunk_sums,
                                  int64_t n_chunks) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        head[0] = 0;
        head[1] = 0;
    }
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_tiles; k += (int64_t)gridDim.x * blockDim.x)
        tile_sums[k] = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_chunks; k += (int64_t)gridDim.x * blockDim.x)
        chunk_sums[k] = 0;
}

// Expansion of the kept runs, then, in the same launch, the traversal fill
// of the rays whose runs the pool could not hold: after the expansion the
// blocks stride through their list, reading the tree from global memory.
// Those outputs are disjoint from the expansion's (it skips them, and a
// 16-byte group they share is written with 4-byte stores).
// kScan: the offsets are not given but written here (ChunkScan), from the
// count pass's counts and group sums: a one-call pass then needs no scan
// launch.  The lost rays' first outputs then come from the sums too (the
// offsets array is being written by other blocks of the same launch).
template <int kGrid, bool kSkip, bool kScan>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kExpandWaves))) expand_kernel(GridView g, const float *__restrict__ origins,
                                                        const float *__restrict__ dirs,
                                                        int64_t *__restrict__ offsets, ChunkScan cs, int64_t n_rays,
                                                        const int32_t *__restrict__ nruns, RunReader rd, Lattice lat,
                                                        int64_t capacity, int32_t *__restrict__ ray_ids,
                                                        float *__restrict__ t0, float *__restrict__ t1, int vec4,
                                                        const int32_t *__restrict__ lost,
                                                        const int32_t *__restrict__ n_lost) {
    expand_block<kScan>(offsets, cs, n_rays, nruns, rd, OneLattice{lat}, capacity, ray_ids, t0, t1, vec4 != 0);
    const int64_t m = *n_lost;
    if (m == 0) return;
    const Tree tree = reads_tree(kGrid) ? load_tree<false>(g, nullptr) : Tree{};
    const FillCtx ctx{lat, capacity, ray_ids, t0, t1, nullptr, g.R};
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < m; k += (int64_t)gridDim.x * kBlock) {
        const int64_t i = lost[k];
        const int64_t first = kScan ? offset_of_ray(i, cs) : offsets[i];
        if (first >= capacity) continue;
        float o[3], d[3];
        load_ray(origins, dirs, i, o, d);
        FillVis<false> vis;
        vis.idx = first;
        vis.ray = (int32_t)i;
        vis.lev = 0;
        trace_ray<kGrid, kSkip>(g, tree, o, d, lat, vis, ctx);
    }
}

// Growing-step lattice: t_0 = near, t_{k+1} = fl(t_k + max(fl(t_k*cone),
// dt_min)), stored up to and including the first value past far, then padded
// to the capacity with that value so binary searches over the whole capacity
// stay on written entries.  n_tab = -1 if the capacity ran out first.
//
// The recurrence is sequential (one lane, about 50 ns a point), so the table
// is kept in the workspace between calls: a header beside it holds the four
// parameters, the capacity, the length and a 64-bit hash of every entry.  A
// call whose parameters match a header whose hash matches the table as it
// stands returns at once; anything else (a new workspace, other parameters,
// an overwritten table) rebuilds it.
struct TableHeader {
    uint64_t magic;
    float tmin, tmax, cone, dt_min;
    int32_t cap, n_tab;
    uint64_t hash;
};
constexpr uint64_t kTableMagic = 0x314e4f4356474f00ull;
constexpr int kTableThreads = 256;

// SplitMix64's output function (Steele, Lea and Flood, 2014) of (index, bits):
// summed with wrapping over the entries, so the order of the sum is free.
__device__ __forceinline__ uint64_t entry_mix(int32_t k, float v) {
    uint64_t z = ((uint64_t)(uint32_t)k << 32 | (uint64_t)__float_as_uint(v)) + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ uint64_t table_hash(const float *tab, int32_t cap, uint64_t *s_part) {
    uint64_t h = 0;
    for (int32_t k = threadIdx.x; k < cap; k += kTableThreads) h += entry_mix(k, tab[k]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) h += __shfl_xor(h, off, 64);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = h;
    __syncthreads();
    uint64_t t = 0;
#pragma unroll
    for (int w = 0; w < kTableThreads / 64; ++w) t += s_part[w];
    __syncthreads();
    return t;
}

__device__ __forceinline__ bool same_float(float a, float b) { return __float_as_uint(a) == __float_as_uint(b); }

__global__ void __launch_bounds__(kTableThreads) cone_table_kernel(float tmin, float tmax, float cone, float dt_min,
                                                                  float *tab, int32_t cap, int32_t *n_tab,
                                                                  TableHeader *hdr) {
    __shared__ uint64_t s_part[kTableThreads / 64];
    __shared__ int32_t s_n;
    const uint64_t h_now = table_hash(tab, cap, s_part);
    if (threadIdx.x == 0) {
        const TableHeader H = *hdr;
        const bool same = H.magic == kTableMagic && same_float(H.tmin, tmin) && same_float(H.tmax, tmax) &&
                          same_float(H.cone, cone) && same_float(H.dt_min, dt_min) && H.cap == cap &&
                          H.n_tab > 0 && H.n_tab == *n_tab && H.hash == h_now;
        s_n = same ? 0 : -2;
        if (!same) {
            hdr->magic = 0;   // invalid until rebuilt
            float t = tmin;
            int32_t k = 0;
            while (k < cap) {
                tab[k++] = t;
                if (t > tmax) break;
                float grow = __fmul_rn(t, cone);
                float step = grow > dt_min ? grow : dt_min;
                t = __fadd_rn(t, step);
            }
            s_n = (k > 0 && tab[k - 1] > tmax) ? k : -1;
            *n_tab = s_n;
        }
    }
    __syncthreads();
    const int32_t n = s_n;
    if (n == 0 || n == -1) return;   // reused, or the capacity ran out (left invalid)
    const float last = tab[n - 1];
    for (int32_t k = n + threadIdx.x; k < cap; k += kTableThreads) tab[k] = last;
    __syncthreads();
    const uint64_t h_new = table_hash(tab, cap, s_part);
    if (threadIdx.x == 0) {
        hdr->tmin = tmin;
        hdr->tmax = tmax;
        hdr->cone = cone;
        hdr->dt_min = dt_min;
        hdr->cap = cap;
        hdr->n_tab = n;
        hdr->hash = h_new;
        hdr->magic = kTableMagic;
    }
}

__global__ void zero_kernel(int64_t *p, int32_t *q) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (p) *p = 0;
        if (q) *q = 0;
    }
}

// ------------------------------------------------------------------ host

// Entries the growing-step table needs up to the first point past far (an
// upper bound; 0 for a constant step or an empty range, -1 if too long):
// every step adds at least dt_min less half an ulp of far, and past
// dt_min/cone each step multiplies t by at least (1 + cone) up to rounding.
int32_t cone_table_capacity(float near_t, float far_t, const ogv_step *step) {
    if (step->kind != OGV_STEP_CONE || !(far_t >= near_t)) return 0;
    double ulp = (double)std::nextafter(far_t, INFINITY) - (double)far_t;
    double inc = (double)step->dt_min - 0.5 * ulp;
    if (!(inc > 0.0)) return -1;
    double n_lin = std::ceil(((double)far_t - (double)near_t) / inc) + 2.0;
    double n = n_lin;
    if (step->cone > 1e-6f) {
        double knee = (double)step->dt_min / (double)step->cone;
        double n_floor = knee > near_t ? std::ceil((knee - (double)near_t) / inc) + 2.0 : 0.0;
        double t_s = knee > near_t ? knee : (double)near_t;
        double rate = std::log1p((double)step->cone) - 4.0 * std::ldexp(1.0, -24);
        double n_geo = far_t > t_s && t_s > 0 ? std::ceil(std::log((double)far_t / t_s) / rate) + 2.0 : 0.0;
        if (t_s > 0) n = std::min(n_lin, n_floor + n_geo);
    }
    n += 16.0;
    if (!(n <= (double)(1 << 22))) return -1;
    return (int32_t)n;
}

ogv_status validate_sampling(const ogv_grid *grid, int32_t variant, const float *o, const float *d, int64_t n_rays,
                    float near_t, float far_t, const ogv_step *step, const char *fn) {
    std::string f(fn);
    if (!grid) OGV_FAIL(OGV_ERR_INVALID, f + ": grid is null");
    if (variant < 0 || variant > (OGV_SKIP | OGV_VOXEL | OGV_SUBLEAF))
        OGV_FAIL(OGV_ERR_INVALID, f + ": variant must be 0..7");
    if ((variant & OGV_VOXEL) && (variant & OGV_SUBLEAF))
        OGV_FAIL(OGV_ERR_INVALID, f + ": OGV_VOXEL and OGV_SUBLEAF exclude each other");
    if ((variant & (OGV_VOXEL | OGV_SUBLEAF)) && grid->view.kind != 1)
        OGV_FAIL(OGV_ERR_INVALID, f + ": OGV_VOXEL and OGV_SUBLEAF walk a VDB grid; this grid is not one");
    if (n_rays < 0 || n_rays > (int64_t)INT32_MAX) OGV_FAIL(OGV_ERR_INVALID, f + ": n_rays out of range");
    if (n_rays > 0 && (!o || !d)) OGV_FAIL(OGV_ERR_INVALID, f + ": null ray pointer");
    if (!step) OGV_FAIL(OGV_ERR_INVALID, f + ": step is null");
    if (!std::isfinite(near_t) || !std::isfinite(far_t) || near_t < 0.0f)
        OGV_FAIL(OGV_ERR_INVALID, f + ": near/far must be finite with near >= 0");
    if (step->kind == OGV_STEP_CONST) {
        if (!(step->dt > 0.0f) || !std::isfinite(step->dt)) OGV_FAIL(OGV_ERR_INVALID, f + ": dt must be > 0");
        if (far_t >= near_t && ((double)far_t - (double)near_t) / (double)step->dt > 16777000.0)
            OGV_FAIL(OGV_ERR_UNSUPPORTED, f + ": more than 2^24 lattice points");
    } else if (step->kind == OGV_STEP_CONE) {
        if (!(step->dt_min > 0.0f) || !std::isfinite(step->dt_min) || !(step->cone >= 0.0f) ||
            !std::isfinite(step->cone))
            OGV_FAIL(OGV_ERR_INVALID, f + ": growing step needs dt_min > 0 and cone >= 0");
        float next = far_t + step->dt_min;
        double ulp = (double)std::nextafter(far_t, INFINITY) - (double)far_t;
        if (!(next > far_t) || (double)step->dt_min < 2.0 * ulp)
            OGV_FAIL(OGV_ERR_UNSUPPORTED, f + ": dt_min below two ulps of far");
    } else {
        OGV_FAIL(OGV_ERR_INVALID, f + ": unknown step kind");
    }
    return OGV_OK;
}

namespace {

struct Plan {
    int64_t n_rays;
    size_t off_counts, off_nruns, off_runs, off_next, off_chunks, off_cnext, off_lost, off_tiles, off_csums, off_tab,
        off_ntab, off_thdr,
        total;
    int32_t pool_cap;
    int64_t n_tiles;
    int32_t tab_cap;
};

bool make_plan(int64_t n_rays, float near_t, float far_t, const ogv_step *step, Plan *p, std::string *why) {
    p->n_rays = n_rays;
    p->n_tiles = scan_tiles(n_rays);
    p->tab_cap = cone_table_capacity(near_t, far_t, step);
    if (p->tab_cap < 0) {
        *why = "growing-step lattice longer than 2^22 points";
        return false;
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    p->off_counts = take(sizeof(int32_t) * (size_t)n_rays);
    p->off_nruns = take(sizeof(int32_t) * (size_t)n_rays);
    p->off_runs = take(sizeof(int2) * (size_t)n_rays * kMaxRuns);
    p->off_next = take(sizeof(int32_t) * (size_t)n_rays);
    p->pool_cap = (int32_t)std::min<int64_t>(std::max<int64_t>(256, n_rays / 16), 1 << 24);
    p->off_chunks = take(sizeof(int2) * (size_t)p->pool_cap * kMaxRuns);
    p->off_cnext = take(sizeof(int32_t) * (size_t)p->pool_cap);
    p->off_lost = take(sizeof(int32_t) * (size_t)n_rays);
    p->off_tiles = take(sizeof(int64_t) * (size_t)(p->n_tiles + 1));
    p->off_csums = take(sizeof(int64_t) * (size_t)((n_rays + kBlock - 1) / kBlock));
    p->off_tab = take(sizeof(float) * (size_t)p->tab_cap);
    p->off_ntab = take(sizeof(int32_t) * 4);
    p->off_thdr = take(sizeof(TableHeader));
    p->total = off;
    return true;
}

Lattice make_lattice(float near_t, float far_t, const ogv_step *step, void *ws, const Plan &p) {
    Lattice lat;
    lat.tmin = near_t;
    lat.tmax = far_t;
    lat.dt = step->dt;
    lat.cone = step->kind == OGV_STEP_CONE;
    lat.tab = lat.cone ? (const float *)((char *)ws + p.off_tab) : nullptr;
    lat.n_tab = p.tab_cap;
    return lat;
}

size_t lds_bytes(const GridView &g) {
    return g.kind == 1 ? tree_lds_bytes(g.L, g.NR, g.S) : 0;
}

constexpr size_t kLdsTreeBytes = 32768;


struct Bufs {
    int32_t *counts, *nruns;
    RunPool pool;
    int64_t *tiles;
    int64_t *csums;   // per 256-ray chunk
};

Bufs bufs_of(void *ws, const Plan &p) {
    char *w = (char *)ws;
    Bufs b;
    b.counts = (int32_t *)(w + p.off_counts);
    b.nruns = (int32_t *)(w + p.off_nruns);
    b.pool.slots = (int2 *)(w + p.off_runs);
    b.pool.stride = p.n_rays;
    b.pool.ray_next = (int32_t *)(w + p.off_next);
    b.pool.chunks = (int2 *)(w + p.off_chunks);
    b.pool.chunk_next = (int32_t *)(w + p.off_cnext);
    // [0] n_tab, [1] pool head, [2] lost rays
    b.pool.head = (int32_t *)(w + p.off_ntab) + 1;
    b.pool.cap = p.pool_cap;
    b.pool.lost = (int32_t *)(w + p.off_lost);
    b.pool.n_lost = (int32_t *)(w + p.off_ntab) + 2;
    b.tiles = (int64_t *)(w + p.off_tiles);
    b.csums = (int64_t *)(w + p.off_csums);
    return b;
}

RunReader reader_of(const Bufs &b) {
    return RunReader{b.pool.slots, b.pool.stride, b.pool.ray_next, b.pool.chunks, b.pool.chunk_next};
}

template <int kGrid, bool kSkip, bool kLds>
void launch_count(const GridView &g, const float *o, const float *d, int64_t n, const Lattice &lat, const Bufs &b,
                  int width, hipStream_t s) {
    unsigned blocks = (unsigned)((tiled_threads(n, width) + kBlock - 1) / kBlock);
    size_t shm = kLds ? lds_bytes(g) : 0;
    const int64_t nt = scan_tiles(n), nc = (n + kBlock - 1) / kBlock;
    pool_reset_kernel<<<(unsigned)std::min<int64_t>((nc + 255) / 256 + 1, 64), 256, 0, s>>>(b.pool.head, b.tiles, nt,
                                                                                         b.csums, nc);
    if (g.L == 1)
        count_kernel<kGrid, kSkip, kLds, true>
            <<<blocks, kBlock, shm, s>>>(g, o, d, n, lat, b.counts, b.nruns, b.pool, width, b.tiles, b.csums);
    else
        count_kernel<kGrid, kSkip, kLds, false>
            <<<blocks, kBlock, shm, s>>>(g, o, d, n, lat, b.counts, b.nruns, b.pool, width, b.tiles, b.csums);
}

template <int kGrid, bool kSkip, bool kLds>
void launch_fill(const GridView &g, const float *o, const float *d, int64_t n, const Lattice &lat,
                 const int64_t *offsets, int64_t cap, int32_t *ids, float *t0, float *t1, int32_t *vox,
                 hipStream_t s) {
    const unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
    const size_t shm = kLds ? lds_bytes(g) : 0;
    if (vox)
        fill_kernel<kGrid, kSkip, true, kLds><<<blocks, kBlock, shm, s>>>(g, o, d, n, lat, offsets, cap, ids, t0, t1, vox);
    else
        fill_kernel<kGrid, kSkip, false, kLds><<<blocks, kBlock, shm, s>>>(g, o, d, n, lat, offsets, cap, ids, t0, t1,
                                                                          vox);
}

// Traversal of a call (the CursorOf index): the grid's kind, or 3 for a VDB
// grid walked one voxel per step.
int traversal_of(const GridView &g, int variant) {
    return (variant & OGV_VOXEL) ? 3 : (variant & OGV_SUBLEAF) ? 4 : g.kind;
}

// Calls OGV_LAUNCH(traversal, skip, tree in LDS) with the instantiation that
// serves (g, variant).
#define OGV_DISPATCH(g, variant)                                         \
    do {                                                                 \
        const bool sk_ = ((variant) & OGV_SKIP) != 0;                    \
        const bool lds_ = lds_bytes(g) <= kLdsTreeBytes;                 \
        switch (traversal_of(g, variant)) {                              \
        case 0:                                                          \
            if (sk_) OGV_LAUNCH(0, true, false);                         \
            else OGV_LAUNCH(0, false, false);                            \
            break;                                                       \
        case 2:                                                          \
            if (sk_) OGV_LAUNCH(2, true, false);                         \
            else OGV_LAUNCH(2, false, false);                            \
            break;                                                       \
        case 3:                                                          \
            if (sk_ && lds_) OGV_LAUNCH(3, true, true);                  \
            else if (sk_) OGV_LAUNCH(3, true, false);                    \
            else if (lds_) OGV_LAUNCH(3, false, true);                   \
            else OGV_LAUNCH(3, false, false);                            \
            break;                                                       \
        case 4:                                                          \
            if (sk_ && lds_) OGV_LAUNCH(4, true, true);                  \
            else if (sk_) OGV_LAUNCH(4, true, false);                    \
            else if (lds_) OGV_LAUNCH(4, false, true);                   \
            else OGV_LAUNCH(4, false, false);                            \
            break;                                                       \
        default:                                                         \
            if (sk_ && lds_) OGV_LAUNCH(1, true, true);                  \
            else if (sk_) OGV_LAUNCH(1, true, false);                    \
            else if (lds_) OGV_LAUNCH(1, false, true);                   \
            else OGV_LAUNCH(1, false, false);                            \
        }                                                                \
    } while (0)

void dispatch_count(const GridView &g, int variant, const float *o, const float *d, int64_t n, const Lattice &lat,
                    const Bufs &b, int width, hipStream_t s) {
#define OGV_LAUNCH(V, K, L) launch_count<V, K, reads_tree(V) && L>(g, o, d, n, lat, b, width, s)
    OGV_DISPATCH(g, variant);
#undef OGV_LAUNCH
}

void dispatch_fill(const GridView &g, int variant, const float *o, const float *d, int64_t n, const Lattice &lat,
                   const int64_t *offsets, int64_t cap, int32_t *ids, float *t0, float *t1, int32_t *vox,
                   hipStream_t s) {
#define OGV_LAUNCH(V, K, L) launch_fill<V, K, reads_tree(V) && L>(g, o, d, n, lat, offsets, cap, ids, t0, t1, vox, s)
    OGV_DISPATCH(g, variant);
#undef OGV_LAUNCH
}

ogv_status build_table(float near_t, float far_t, const ogv_step *step, void *ws, const Plan &p, hipStream_t s) {
    if (step->kind != OGV_STEP_CONE || p.tab_cap == 0) return OGV_OK;
    float *tab = (float *)((char *)ws + p.off_tab);
    int32_t *n_tab = (int32_t *)((char *)ws + p.off_ntab);
    TableHeader *hdr = (TableHeader *)((char *)ws + p.off_thdr);
    cone_table_kernel<<<1, kTableThreads, 0, s>>>(near_t, far_t, step->cone, step->dt_min, tab, p.tab_cap, n_tab, hdr);
    OGV_CHECK_LAUNCH();
    return OGV_OK;
}

// count + exclusive scan; offsets[n] = total; overflow (nullable) = total > capacity
ogv_status count_and_scan(const ogv_grid *grid, int32_t variant, int width, const float *o, const float *d,
                          int64_t n, const Lattice &lat, int64_t *offsets, void *ws, const Plan &p, int64_t capacity,
                          int32_t *overflow, hipStream_t s) {
    if (n == 0) {
        zero_kernel<<<1, 64, 0, s>>>(offsets, overflow);
        OGV_CHECK_LAUNCH();
        return OGV_OK;
    }
    Bufs b = bufs_of(ws, p);
    dispatch_count(grid->view, variant, o, d, n, lat, b, width, s);
    OGV_CHECK_LAUNCH();
    OGV_CHECK_HIP(launch_excl_scan_from_sums(b.counts, n, offsets, b.tiles, capacity, overflow, s));
    return OGV_OK;
}

// fill from the runs the count pass left in the workspace: the expansion
// kernel writes every ray whose runs were kept, the traversal fill the rest;
// with voxel ids every ray is re-walked instead
ogv_status fill_all(const ogv_grid *grid, int32_t variant, const float *o, const float *d, int64_t n,
                    const Lattice &lat, const int64_t *offsets, int64_t cap, int32_t *ids, float *t0, float *t1,
                    int32_t *vox, void *ws, const Plan &p, hipStream_t s) {
    if (n == 0 || cap == 0) return OGV_OK;
    Bufs b = bufs_of(ws, p);
    if (vox) {
        dispatch_fill(grid->view, variant, o, d, n, lat, offsets, cap, ids, t0, t1, vox, s);
        OGV_CHECK_LAUNCH();
        return OGV_OK;
    }
    const unsigned blocks = (unsigned)min(expand_items(n), (int64_t)INT32_MAX);
    const int vec4 = (((uintptr_t)ids | (uintptr_t)t0 | (uintptr_t)t1) & 15) == 0;
    const GridView &g = grid->view;
    // the expansion's lost-ray walk reads the tree from global memory (the
    // LDS flag is ignored)
#define OGV_LAUNCH(V, K, L)                                                                                          \
    expand_kernel<V, K, false><<<blocks, kBlock, 0, s>>>(g, o, d, const_cast<int64_t *>(offsets), ChunkScan{}, n,    \
                                                          b.nruns, reader_of(b), lat, cap, ids, t0, t1, vec4,        \
                                                          b.pool.lost, b.pool.n_lost)
    OGV_DISPATCH(g, variant);
#undef OGV_LAUNCH
    OGV_CHECK_LAUNCH();
    return OGV_OK;
}

// Rays a one-call pass scans inside the expansion: each expansion block sums
// the tile sums before its chunk.  That prologue delays its stores; against a
// separate scan launch it pays up to about 200 tiles (measured: the
// 640,000-ray object workload, 157 tiles, 0.271 -> 0.264 ms a step; the
// 1,064,960-ray cascades, 260 tiles, 0.503 -> 0.510 ms).
constexpr int64_t kScanInExpandTiles = 192;

// scan and fill of a one-call pass in one launch: the expansion writes the
// offsets (and the overflow flag) itself from the count pass's sums
ogv_status scan_fill_fused(const ogv_grid *grid, int32_t variant, const float *o, const float *d, int64_t n,
                           const Lattice &lat, int64_t *offsets, int64_t cap, int32_t *ids, float *t0, float *t1,
                           int32_t *overflow, void *ws, const Plan &p, hipStream_t s) {
    Bufs b = bufs_of(ws, p);
    const unsigned blocks = (unsigned)min(expand_items(n), (int64_t)INT32_MAX);
    const int vec4 = (((uintptr_t)ids | (uintptr_t)t0 | (uintptr_t)t1) & 15) == 0;
    const GridView &g = grid->view;
    const ChunkScan cs{b.counts, b.tiles, b.csums, overflow};
#define OGV_LAUNCH(V, K, L)                                                                                          \
    expand_kernel<V, K, true><<<blocks, kBlock, 0, s>>>(g, o, d, offsets, cs, n, b.nruns, reader_of(b), lat, cap,    \
                                                         ids, t0, t1, vec4, b.pool.lost, b.pool.n_lost)
    OGV_DISPATCH(g, variant);
#undef OGV_LAUNCH
    OGV_CHECK_LAUNCH();
    return OGV_OK;
}

// Voxel ids are int32: every id of the grid, ((l*R+i)*R+j)*R+k, must fit.
ogv_status check_voxel_ids(const ogv_grid *grid, const int32_t *vox, const char *fn) {
    const GridView &g = grid->view;
    if (vox && (int64_t)g.L * g.R * g.R * g.R - 1 > (int64_t)INT32_MAX)
        OGV_FAIL(OGV_ERR_UNSUPPORTED, std::string(fn) + ": voxel ids need n_levels * res^3 <= 2^31");
    return OGV_OK;
}

ogv_status prepare(const ogv_grid *grid, const ogv_sample_opts &opts, const float *o, const float *d, int64_t n,
                   float near_t, float far_t, const ogv_step *step, void *ws, size_t ws_bytes, Plan *p,
                   const char *fn) {
    ogv_status st = validate_sampling(grid, opts.variant, o, d, n, near_t, far_t, step, fn);
    if (st != OGV_OK) return st;
    if (opts.image_width < 0) OGV_FAIL(OGV_ERR_INVALID, std::string(fn) + ": image_width < 0");
    std::string why;
    if (!make_plan(n, near_t, far_t, step, p, &why)) OGV_FAIL(OGV_ERR_UNSUPPORTED, why);
    if (!ws || ws_bytes < p->total)
        OGV_FAIL(OGV_ERR_CAPACITY, std::string(fn) + ": workspace smaller than ogv_sample_workspace_size");
    return OGV_OK;
}

}  // namespace
}  // namespace ogv

using namespace ogv;

extern "C" ogv_status ogv_sample_workspace_size(int64_t n_rays, float near_t, float far_t, const ogv_step *step,
                                                size_t *bytes) {
    if (!step || !bytes) OGV_FAIL(OGV_ERR_INVALID, "null argument");
    if (n_rays < 0) OGV_FAIL(OGV_ERR_INVALID, "n_rays < 0");
    Plan p;
    std::string why;
    if (!make_plan(n_rays, near_t, far_t, step, &p, &why)) OGV_FAIL(OGV_ERR_UNSUPPORTED, why);
    *bytes = p.total;
    return OGV_OK;
}

static ogv_sample_opts opts_of(const ogv_sample_opts *o) { return o ? *o : ogv_sample_opts{OGV_BRANCH, 0}; }

extern "C" ogv_status ogv_sample_count(const ogv_grid *grid, const ogv_sample_opts *opts_p, const float *o,
                                       const float *d, int64_t n, float near_t, float far_t, const ogv_step *step,
                                       int64_t *offsets, void *ws, size_t ws_bytes, void *stream) {
    const ogv_sample_opts opts = opts_of(opts_p);
    Plan p;
    ogv_status st = prepare(grid, opts, o, d, n, near_t, far_t, step, ws, ws_bytes, &p, "ogv_sample_count");
    if (st != OGV_OK) return st;
    if (!offsets) OGV_FAIL(OGV_ERR_INVALID, "offsets is null");
    hipStream_t s = (hipStream_t)stream;
    if ((st = build_table(near_t, far_t, step, ws, p, s)) != OGV_OK) return st;
    Lattice lat = make_lattice(near_t, far_t, step, ws, p);
    return count_and_scan(grid, opts.variant, opts.image_width, o, d, n, lat, offsets, ws, p, 0, nullptr, s);
}

extern "C" ogv_status ogv_sample_count_raw(const ogv_grid *grid, const ogv_sample_opts *opts_p, const float *o,
                                           const float *d, int64_t n, float near_t, float far_t,
                                           const ogv_step *step, void *ws, size_t ws_bytes, void *stream) {
    const ogv_sample_opts opts = opts_of(opts_p);
    Plan p;
    ogv_status st = prepare(grid, opts, o, d, n, near_t, far_t, step, ws, ws_bytes, &p, "ogv_sample_count_raw");
    if (st != OGV_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if ((st = build_table(near_t, far_t, step, ws, p, s)) != OGV_OK) return st;
    if (n == 0) return OGV_OK;
    Lattice lat = make_lattice(near_t, far_t, step, ws, p);
    dispatch_count(grid->view, opts.variant, o, d, n, lat, bufs_of(ws, p), opts.image_width, s);
    OGV_CHECK_LAUNCH();
    return OGV_OK;
}

extern "C" ogv_status ogv_sample_scan(int64_t n, int64_t *offsets, void *ws, size_t ws_bytes, void *stream) {
    if (n < 0 || n > (int64_t)INT32_MAX) OGV_FAIL(OGV_ERR_INVALID, "n_rays out of range");
    if (!offsets) OGV_FAIL(OGV_ERR_INVALID, "offsets is null");
    // counts and scan tiles sit at offsets that depend on n_rays alone
    const ogv_step unit{OGV_STEP_CONST, 1.0f, 0.0f, 0.0f};
    Plan p;
    std::string why;
    if (!make_plan(n, 0.0f, 0.0f, &unit, &p, &why)) OGV_FAIL(OGV_ERR_UNSUPPORTED, why);
    if (!ws || ws_bytes < p.off_tab) OGV_FAIL(OGV_ERR_CAPACITY, "workspace smaller than the count call's");
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        zero_kernel<<<1, 64, 0, s>>>(offsets, nullptr);
        OGV_CHECK_LAUNCH();
        return OGV_OK;
    }
    Bufs b = bufs_of(ws, p);
    OGV_CHECK_HIP(launch_excl_scan_from_sums(b.counts, n, offsets, b.tiles, 0, nullptr, s));
    return OGV_OK;
}

extern "C" ogv_status ogv_sample_fill(const ogv_grid *grid, const ogv_sample_opts *opts_p, const float *o,
                                      const float *d, int64_t n, float near_t, float far_t, const ogv_step *step,
                                      const int64_t *offsets, int64_t capacity, int32_t *ray_ids, float *t0,
                                      float *t1, int32_t *vox, void *ws, size_t ws_bytes, void *stream) {
    const ogv_sample_opts opts = opts_of(opts_p);
    Plan p;
    ogv_status st = prepare(grid, opts, o, d, n, near_t, far_t, step, ws, ws_bytes, &p, "ogv_sample_fill");
    if (st != OGV_OK) return st;
    if (!offsets) OGV_FAIL(OGV_ERR_INVALID, "offsets is null");
    if (capacity < 0) OGV_FAIL(OGV_ERR_INVALID, "capacity < 0");
    if (capacity > 0 && (!ray_ids || !t0 || !t1)) OGV_FAIL(OGV_ERR_INVALID, "null sample array");
    if ((st = check_voxel_ids(grid, vox, "ogv_sample_fill")) != OGV_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    Lattice lat = make_lattice(near_t, far_t, step, ws, p);
    return fill_all(grid, opts.variant, o, d, n, lat, offsets, capacity, ray_ids, t0, t1, vox, ws, p, s);
}

extern "C" ogv_status ogv_sample_rays(const ogv_grid *grid, const ogv_sample_opts *opts_p, const float *o,
                                      const float *d, int64_t n, float near_t, float far_t, const ogv_step *step,
                                      int64_t *offsets, int64_t capacity, int32_t *ray_ids, float *t0, float *t1,
                                      int32_t *vox, int32_t *overflow, void *ws, size_t ws_bytes, void *stream) {
    const ogv_sample_opts opts = opts_of(opts_p);
    Plan p;
    ogv_status st = prepare(grid, opts, o, d, n, near_t, far_t, step, ws, ws_bytes, &p, "ogv_sample_rays");
    if (st != OGV_OK) return st;
    if (!offsets || !overflow) OGV_FAIL(OGV_ERR_INVALID, "offsets/overflow is null");
    if (capacity < 0) OGV_FAIL(OGV_ERR_INVALID, "capacity < 0");
    if (capacity > 0 && (!ray_ids || !t0 || !t1)) OGV_FAIL(OGV_ERR_INVALID, "null sample array");
    if ((st = check_voxel_ids(grid, vox, "ogv_sample_rays")) != OGV_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if ((st = build_table(near_t, far_t, step, ws, p, s)) != OGV_OK) return st;
    Lattice lat = make_lattice(near_t, far_t, step, ws, p);
    if (n > 0 && !vox && p.n_tiles <= kScanInExpandTiles) {
        // walk, then one launch that scans and fills
        dispatch_count(grid->view, opts.variant, o, d, n, lat, bufs_of(ws, p), opts.image_width, s);
        OGV_CHECK_LAUNCH();
        return scan_fill_fused(grid, opts.variant, o, d, n, lat, offsets, capacity, ray_ids, t0, t1, overflow, ws, p,
                               s);
    }
    if ((st = count_and_scan(grid, opts.variant, opts.image_width, o, d, n, lat, offsets, ws, p, capacity, overflow,
                             s)) != OGV_OK)
        return st;
    return fill_all(grid, opts.variant, o, d, n, lat, offsets, capacity, ray_ids, t0, t1, vox, ws, p, s);
}

// ------------------------------------------------------------------ no allocation

// Workspace of ogv_sample_rays_noalloc: one file-scope array per device,
// which the device holds until the process ends.  In host code `scratch`
// names a host-side stand-in, not device memory: only the address
// hipGetSymbolAddress returns for it (kept per device below) is passed to
// kernels.  Every call on a device shares that device's copy.  Nothing in it
// needs clearing between calls: the count pass zeroes its counters and scan
// sums itself, every per-ray entry is written before it is read, and the
// growing-step table is only reused when its header and hash match.
static __device__ __align__(256) unsigned char scratch[OGV_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices];   // address of `scratch` on each device, once looked up

// The current device's copy of `scratch`, looked up once per device (with
// that device current, as it is for the caller's launches).
ogv_status scratch_of_current_device(void **ptr) {
    int dev = -1;
    OGV_CHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) OGV_FAIL(OGV_ERR_UNSUPPORTED, "device index beyond the library's table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        OGV_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) OGV_FAIL(OGV_ERR_HIP, "hipGetSymbolAddress returned a null address for the scratch array");
        g_scratch_dev[dev] = p;
    }
    *ptr = g_scratch_dev[dev];
    return OGV_OK;
}
}  // namespace

extern "C" ogv_status ogv_sample_rays_noalloc(const ogv_grid *grid, const ogv_sample_opts *opts_p, const float *o,
                                              const float *d, int64_t n, float near_t, float far_t,
                                              const ogv_step *step, int64_t *offsets, int64_t capacity,
                                              int32_t *ray_ids, float *t0, float *t1, int32_t *vox,
                                              int32_t *overflow, void *stream) {
    if (!step) OGV_FAIL(OGV_ERR_INVALID, "ogv_sample_rays_noalloc: step is null");
    if (n < 0) OGV_FAIL(OGV_ERR_INVALID, "ogv_sample_rays_noalloc: n_rays < 0");
    Plan p;
    std::string why;
    if (!make_plan(n, near_t, far_t, step, &p, &why)) OGV_FAIL(OGV_ERR_UNSUPPORTED, why);
    if (p.total > (size_t)OGV_NOALLOC_SCRATCH_BYTES)
        OGV_FAIL(OGV_ERR_CAPACITY, "ogv_sample_rays_noalloc: the call needs " + std::to_string(p.total) +
                                       " bytes of workspace, more than the " +
                                       std::to_string((size_t)OGV_NOALLOC_SCRATCH_BYTES) +
                                       "-byte static scratch; use ogv_sample_rays with a workspace");
    void *ws = nullptr;
    ogv_status st = scratch_of_current_device(&ws);
    if (st != OGV_OK) return st;
    return ogv_sample_rays(grid, opts_p, o, d, n, near_t, far_t, step, offsets, capacity, ray_ids, t0, t1, vox,
                           overflow, ws, (size_t)OGV_NOALLOC_SCRATCH_BYTES, stream);
}
