// The counting pass of the sampler: one ray per lane walks the grid, counts
// its lattice samples, keeps its occupied runs and adds its count to the scan
// tile and expansion chunk sums.  Shared by the sampler's two sources: the
// Alg. 2 walks over a tree are instantiated in count_skip.hip, built at a
// different optimisation level; the rest in sample.hip.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cstdint>

#include "geometry.hpp"
#include "internal.hpp"
#include "scan.hpp"
#include "trace.hpp"

namespace ogv {

// The wave adds its rays' counts to the sums of the groups of 2^kShift
// consecutive rays it touches: one wave reduction and one atomic per group.
// Groups of kScanTile rays are the scan tiles (so the scan needs no reduce
// launch of its own); groups of kBlock rays are the expansion's chunks (so a
// one-call pass needs no scan launch at all).
template <int kShift>
__device__ __forceinline__ void add_group_sums(int64_t ray, int32_t n, int64_t *__restrict__ tile_sums) {
    const int lane = threadIdx.x & 63;
    const int32_t key = ray >= 0 ? (int32_t)(ray >> kShift) : -1;
    uint64_t todo = __ballot(key >= 0);
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int32_t k = __shfl(key, leader, 64);
        const bool mine = key == k;
        int32_t v = mine ? n : 0;   // a wave's 64 rays hold < 2^31 samples (2^24 lattice points each)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == leader) atomicAdd((unsigned long long *)&tile_sums[k], (unsigned long long)(int64_t)v);
        todo &= ~__ballot(mine);
    }
}

// The chunk sums (kBlock consecutive rays each).  Every 8 consecutive lanes
// walk consecutive rays (a pixel row of a tile, or 8 of a row-major range),
// so their chunks form at most two contiguous segments: a segmented scan over
// the 8 lanes leaves each segment's total in its last lane, which adds it.
__device__ __forceinline__ void add_chunk_sums(int64_t ray, int32_t n, int64_t *__restrict__ chunk_sums) {
    const int32_t key = ray >= 0 ? (int32_t)(ray / kBlock) : -1;
    const int l8 = threadIdx.x & 7;
    int32_t v = n;
#pragma unroll
    for (int off = 1; off < 8; off <<= 1) {
        const int32_t y = __shfl_up(v, off, 8);
        const int32_t ky = __shfl_up(key, off, 8);
        if (l8 >= off && ky == key) v += y;
    }
    const int32_t kn = __shfl_down(key, 1, 8);
    const bool last = l8 == 7 || kn != key;
    if (last && key >= 0 && v != 0) atomicAdd((unsigned long long *)&chunk_sums[key], (unsigned long long)(int64_t)v);
}

// counts[i] = samples of ray i; nruns[i] = its occupied runs (kRunsLost: the
// run pool ran dry, the traversal fill writes the ray); the runs themselves
// go to the pool's slots and chunks; tile_sums[k] gains the counts of rays
// k*kScanTile .. (k+1)*kScanTile-1.  Single-level walks of the Alg. 1 loop
// ask for 7 waves per SIMD (8 for the dense march): the prioritised long
// waves then share their SIMD with more short ones (the compiler would
// otherwise settle at 6 once the span is computed before the walk).  So do
// the single-level Alg. 2 walks over a tree, which count_skip.hip builds at
// -O2 (at -O1 their nested loops took 14-40% longer).  The single-level
// Alg. 2 chessboard walk asks for 5 (83 VGPRs, no spills).  The cascade walks of
// the Alg. 1 loop over the dense grid, the hierarchical and the sub-leaf
// steps ask for 5 (70 to 87 VGPRs at -O1, no spills; the compiler would
// settle at 4).
constexpr int count_waves_per_eu(int kGrid, bool kSkip, bool kL1) {
    return kL1 ? (kGrid == 0 ? 8 : kSkip && kGrid == 2 ? 5 : 7)
               : (!kSkip && (kGrid == 0 || kGrid == 1 || kGrid == 4) ? 5 : 1);
}

// The instantiations count_skip.hip holds: X(traversal, tree in LDS, single level).
#define OGV_COUNT_SKIP_ALL                                                                                     \
    OGV_COUNT_SKIP(1, true, true) OGV_COUNT_SKIP(1, true, false) OGV_COUNT_SKIP(1, false, true)                \
    OGV_COUNT_SKIP(1, false, false) OGV_COUNT_SKIP(3, true, true) OGV_COUNT_SKIP(3, true, false)               \
    OGV_COUNT_SKIP(3, false, true) OGV_COUNT_SKIP(3, false, false) OGV_COUNT_SKIP(4, true, true)               \
    OGV_COUNT_SKIP(4, true, false) OGV_COUNT_SKIP(4, false, true) OGV_COUNT_SKIP(4, false, false)

template <int kGrid, bool kSkip, bool kLds, bool kL1>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(count_waves_per_eu(kGrid, kSkip, kL1))))
count_kernel(GridView g, const float *__restrict__ origins, const float *__restrict__ dirs, int64_t n_rays,
             Lattice lat, int32_t *__restrict__ counts, int32_t *__restrict__ nruns, RunPool pool, int image_width,
             int64_t *__restrict__ tile_sums, int64_t *__restrict__ chunk_sums) {
    extern __shared__ __align__(16) uint32_t smem[];
    Tree tree = reads_tree(kGrid) ? load_tree<kLds>(g, smem) : Tree{};
    const int64_t i = ray_of_thread((int64_t)blockIdx.x * kBlock + threadIdx.x, n_rays, image_width);
    int32_t n = 0;
    if constexpr (kL1) {
        // the span first, so the wave's priority can follow its longest ray
        float o[3] = {0.f, 0.f, 0.f}, d[3] = {0.f, 0.f, 0.f};
        L1Span s{};
        if (i >= 0) {
            load_ray(origins, dirs, i, o, d);
            s = l1_span(g, o, d, lat);
        }
        set_wave_priority(s.hit ? (fminf(s.X, lat.tmax) - fmaxf(s.E, lat.tmin)) *
                                      (fabsf(d[0]) * g.geom[6] + fabsf(d[1]) * g.geom[7] + fabsf(d[2]) * g.geom[8])
                                : 0.0f,
                          g.R);
        if (i >= 0) {
            const CountCtx ctx{lat, pool};
            CountVis vis = make_count_vis(i, pool);
            if (s.hit) march_segment<kGrid, kSkip>(g, tree, 0, s.ray, s.E, s.X, lat, vis, ctx);
            vis.finish(ctx);
            n = vis.n;
            counts[i] = n;
            nruns[i] = vis.nr;
        }
    } else if (i >= 0) {
        float o[3], d[3];
        load_ray(origins, dirs, i, o, d);
        const CountCtx ctx{lat, pool};
        CountVis vis = make_count_vis(i, pool);
        trace_ray<kGrid, kSkip, kL1>(g, tree, o, d, lat, vis, ctx);
        vis.finish(ctx);
        n = vis.n;
        counts[i] = n;
        nruns[i] = vis.nr;
    }
    static_assert(kScanTile == 1 << 12 && kBlock == 1 << 8, "group sums assume 4096-ray tiles, 256-ray chunks");
    add_group_sums<12>(i, n, tile_sums);
    add_chunk_sums(i, n, chunk_sums);
}

}  // namespace ogv
