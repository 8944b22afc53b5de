// Ray sampler kernels: dense-grid voxel DDA (the plain method) and VDB +
// hierarchical DDA (Sec. 2.3, Sec. 3), each in the loop structure of Alg. 1
// ("DDA branch") or Alg. 2 ("DDA skip") of the supplementary material, plus
// the count -> exclusive scan -> fill pipeline that packs the samples.
//
// One ray per lane.  A ray is split into segments owned by one cascade level
// each (finest level wins, Sec. 3); within a segment a cursor walks cells in
// ray order -- voxels for the dense grid; root tiles, internal-node tiles or
// leaf voxels for the VDB tree -- and the driver turns maximal runs of
// occupied cells into parameter intervals (lo, hi].  A visitor converts an
// interval into its lattice points: the count pass adds their number, the
// fill pass writes them.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "geometry.hpp"
#include "internal.hpp"
#include "scan.hpp"

namespace ogv {

constexpr int kBlock = 256;

// ------------------------------------------------------------------ cursors

// Dense bitfield: every cell is a voxel; one bit lookup per voxel.
struct DenseCursor {
    const uint32_t *bits;
    uint64_t level_base;  // bit index of the level's voxel (0,0,0)
    int R;
    Axis A0, A1, A2;
    int u0, u1, u2;       // ray-order voxel per moving axis
    int v0, v1, v2;       // voxel index per axis
    float tn0, tn1, tn2;  // next plane crossing per axis (+inf for zero axes)

    __device__ __forceinline__ bool occupied() const {
        uint64_t idx = level_base + ((uint64_t)((uint32_t)v0 * (uint32_t)R + (uint32_t)v1) * (uint32_t)R + (uint32_t)v2);
        return (bits[idx >> 5] >> (idx & 31)) & 1u;
    }
    __device__ __forceinline__ float exit(int &axis) const {
        float hi = tn0;
        axis = 0;
        if (tn1 < hi) { hi = tn1; axis = 1; }
        if (tn2 < hi) { hi = tn2; axis = 2; }
        return hi;
    }
    __device__ __forceinline__ bool step(int axis, float) {
        if (axis == 0) {
            if (++u0 >= R) return false;
            v0 = A0.voxel(u0);
            tn0 = A0.Tk(u0 + 1);
        } else if (axis == 1) {
            if (++u1 >= R) return false;
            v1 = A1.voxel(u1);
            tn1 = A1.Tk(u1 + 1);
        } else {
            if (++u2 >= R) return false;
            v2 = A2.voxel(u2);
            tn2 = A2.Tk(u2 + 1);
        }
        return true;
    }
};

// VDB tree: the current cell is the largest uniform cell holding the current
// voxel -- a root tile (D = 8*S voxels per axis), an internal-node tile
// (D = 8) or a leaf voxel (D = 1).  Leaving a tile moves the stepping axis
// past the tile and re-locates the other axes at the exit parameter.
struct VdbCursor {
    const GridView *g;
    int lev, R;
    Axis A0, A1, A2;
    int u0, u1, u2;
    int v0, v1, v2;
    float tn0, tn1, tn2;   // voxel-level next crossings (valid when D == 1 && tn_ok)
    bool tn_ok;
    int D;                 // current cell size in voxels
    bool occ;
    const uint64_t *leaf;  // cached leaf (nullptr if none)
    int lb0, lb1, lb2;     // voxel base of the cached leaf block
    uint64_t word;         // cached leaf word for x = v0
    int word_x;

    __device__ __forceinline__ void load_word() {
        word_x = v0 & 7;
        word = leaf[word_x];
    }

    __device__ __forceinline__ void classify() {
        if (leaf != nullptr && (v0 & ~7) == lb0 && (v1 & ~7) == lb1 && (v2 & ~7) == lb2) {
            if ((v0 & 7) != word_x) load_word();
            D = 1;
            occ = (word >> (((v1 & 7) << 3) | (v2 & 7))) & 1ull;
            return;
        }
        const int sh = 3 + g->ilog2;
        const int NR = g->NR;
        int ri = ((lev * NR + (v0 >> sh)) * NR + (v1 >> sh)) * NR + (v2 >> sh);
        int node = g->root[ri];
        if (node < 0) {
            D = 8 << g->ilog2;
            occ = node == -2;
            leaf = nullptr;
            tn_ok = false;
            return;
        }
        const int S = g->S, m = S - 1;
        int s = (((v0 >> 3) & m) * S + ((v1 >> 3) & m)) * S + ((v2 >> 3) & m);
        int w = node * g->W + (s >> 6);
        uint64_t cm = g->child[w];
        uint64_t bit = 1ull << (s & 63);
        if (cm & bit) {
            uint32_t li = g->rank[w] + (uint32_t)__popcll(cm & (bit - 1));
            leaf = g->leaves + (uint64_t)li * 8;
            lb0 = v0 & ~7;
            lb1 = v1 & ~7;
            lb2 = v2 & ~7;
            load_word();
            D = 1;
            occ = (word >> (((v1 & 7) << 3) | (v2 & 7))) & 1ull;
            return;
        }
        D = 8;
        occ = (g->value[w] & bit) != 0;
        leaf = nullptr;
        tn_ok = false;
    }

    __device__ __forceinline__ bool occupied() {
        classify();
        return occ;
    }

    // exit plane (ray order) of the D-cell on one axis
    __device__ __forceinline__ static int exit_plane(const Axis &A, int v, int D) {
        int base = v & ~(D - 1);
        return A.pos ? base + D : A.R - base;
    }

    __device__ __forceinline__ float exit(int &axis) {
        const float inf = __builtin_huge_valf();
        if (D == 1) {
            if (!tn_ok) {
                tn0 = A0.zero ? inf : A0.Tk(u0 + 1);
                tn1 = A1.zero ? inf : A1.Tk(u1 + 1);
                tn2 = A2.zero ? inf : A2.Tk(u2 + 1);
                tn_ok = true;
            }
            float hi = tn0;
            axis = 0;
            if (tn1 < hi) { hi = tn1; axis = 1; }
            if (tn2 < hi) { hi = tn2; axis = 2; }
            return hi;
        }
        float e0 = A0.zero ? inf : A0.Tk(exit_plane(A0, v0, D));
        float e1 = A1.zero ? inf : A1.Tk(exit_plane(A1, v1, D));
        float e2 = A2.zero ? inf : A2.Tk(exit_plane(A2, v2, D));
        float hi = e0;
        axis = 0;
        if (e1 < hi) { hi = e1; axis = 1; }
        if (e2 < hi) { hi = e2; axis = 2; }
        return hi;
    }

    __device__ __forceinline__ bool step(int axis, float t) {
        if (D == 1) {
            if (axis == 0) {
                if (++u0 >= R) return false;
                v0 = A0.voxel(u0);
                tn0 = A0.Tk(u0 + 1);
            } else if (axis == 1) {
                if (++u1 >= R) return false;
                v1 = A1.voxel(u1);
                tn1 = A1.Tk(u1 + 1);
            } else {
                if (++u2 >= R) return false;
                v2 = A2.voxel(u2);
                tn2 = A2.Tk(u2 + 1);
            }
            return true;
        }
        // leave a tile: the stepping axis goes to the first voxel past it,
        // the others to the voxel holding t+ inside the tile's range
        int k0 = A0.zero ? 0 : exit_plane(A0, v0, D);
        int k1 = A1.zero ? 0 : exit_plane(A1, v1, D);
        int k2 = A2.zero ? 0 : exit_plane(A2, v2, D);
        if (axis == 0) {
            if (k0 >= R) return false;
            u0 = k0;
        } else if (!A0.zero) {
            u0 = A0.advance_to(u0, t, min(k0, R) - 1);
        }
        if (axis == 1) {
            if (k1 >= R) return false;
            u1 = k1;
        } else if (!A1.zero) {
            u1 = A1.advance_to(u1, t, min(k1, R) - 1);
        }
        if (axis == 2) {
            if (k2 >= R) return false;
            u2 = k2;
        } else if (!A2.zero) {
            u2 = A2.advance_to(u2, t, min(k2, R) - 1);
        }
        if (!A0.zero) v0 = A0.voxel(u0);
        if (!A1.zero) v1 = A1.voxel(u1);
        if (!A2.zero) v2 = A2.voxel(u2);
        tn_ok = false;
        return true;
    }
};

// ------------------------------------------------------------------ driver

// Walks cells from the segment start a to its end b (or t_max) and reports
// maximal occupied runs (lo, hi] to the visitor.  kSkip = false is Alg. 1
// (every cell visited with a branch on occupancy); kSkip = true is Alg. 2
// (an inner loop passes all leading empty cells, then the occupied run is
// marched).
template <bool kSkip, class Cursor, class Vis>
__device__ __forceinline__ void drive(Cursor &c, float a, float b, float tmax, Vis &vis) {
    float lo = a;
    if (!kSkip) {
        bool in_run = false;
        float run_lo = 0.0f;
        while (true) {
            bool occ = c.occupied();
            int axis;
            float hi = c.exit(axis);
            if (occ && !in_run) {
                run_lo = lo;
                in_run = true;
            } else if (!occ && in_run) {
                vis.run(run_lo, lo);
                in_run = false;
            }
            if (hi >= b || hi >= tmax) {
                if (in_run) vis.run(run_lo, fminf(hi, b));
                return;
            }
            lo = hi;
            if (!c.step(axis, hi)) {
                if (in_run) vis.run(run_lo, lo);
                return;
            }
        }
    } else {
        while (true) {
            while (!c.occupied()) {
                int axis;
                float hi = c.exit(axis);
                if (hi >= b || hi >= tmax) return;
                lo = hi;
                if (!c.step(axis, hi)) return;
            }
            float run_lo = lo;
            while (true) {
                int axis;
                float hi = c.exit(axis);
                if (hi >= b || hi >= tmax) {
                    vis.run(run_lo, fminf(hi, b));
                    return;
                }
                lo = hi;
                if (!c.step(axis, hi)) {
                    vis.run(run_lo, lo);
                    return;
                }
                if (!c.occupied()) break;
            }
            vis.run(run_lo, lo);
        }
    }
}

// ------------------------------------------------------------------ visitors

struct CountVis {
    const Lattice *lat;
    int32_t n;
    __device__ __forceinline__ void begin_level(int, const Axis &, const Axis &, const Axis &) {}
    __device__ __forceinline__ void run(float lo, float hi) {
        int n0 = lat->first_above(lo);
        int n1 = lat->first_above(fminf(hi, lat->tmax));
        if (n1 > n0) n += n1 - n0;
    }
};

template <bool kVox>
struct FillVis {
    const Lattice *lat;
    int64_t idx, capacity;
    int32_t ray;
    int32_t *ray_ids;
    float *t0, *t1;
    int32_t *vox;       // nullable
    int lev, R;
    Axis A0, A1, A2;    // level geometry, for voxel ids only

    __device__ __forceinline__ void begin_level(int l, const Axis &a0, const Axis &a1, const Axis &a2) {
        lev = l;
        if (kVox) {
            A0 = a0;
            A1 = a1;
            A2 = a2;
        }
    }
    __device__ __forceinline__ int vcoord(const Axis &A, float t) const {
        return A.zero ? A.zero_voxel() : A.voxel(A.locate(t, false));
    }
    __device__ __forceinline__ void run(float lo, float hi) {
        int n0 = lat->first_above(lo);
        int n1 = lat->first_above(fminf(hi, lat->tmax));
        float tn = lat->t(n0);
        for (int n = n0; n < n1; ++n) {
            float tnext = lat->t(n + 1);
            if (idx < capacity) {
                ray_ids[idx] = ray;
                t0[idx] = tn;
                t1[idx] = tnext;
                if (kVox) {
                    int i = vcoord(A0, tn), j = vcoord(A1, tn), k = vcoord(A2, tn);
                    vox[idx] = ((lev * R + i) * R + j) * R + k;
                }
            }
            ++idx;
            tn = tnext;
        }
    }
};

// ------------------------------------------------------------------ ray

template <bool kVdb, bool kSkip, class Vis>
__device__ __forceinline__ void march_segment(const GridView &g, int lev, const float o[3], const float d[3],
                                              float a, float b, const Lattice &lat, Vis &vis) {
    if (!(b >= lat.tmin) || !(a < lat.tmax)) return;   // no lattice point in (a, b]
    const float *box = g.boxes + 6 * lev;
    const int R = g.R;
    Axis A0 = make_axis(box, 0, R, o[0], d[0]);
    Axis A1 = make_axis(box, 1, R, o[1], d[1]);
    Axis A2 = make_axis(box, 2, R, o[2], d[2]);
    vis.begin_level(lev, A0, A1, A2);
    // start at the voxel owning t_min when it lies inside the segment,
    // else at the voxel owning the parameters just after a
    const bool after = lat.tmin > a;
    const float ts = after ? lat.tmin : a;
    int u0 = 0, u1 = 0, u2 = 0, v0, v1, v2;
    if (A0.zero) v0 = A0.zero_voxel(); else { u0 = A0.locate(ts, !after); v0 = A0.voxel(u0); }
    if (A1.zero) v1 = A1.zero_voxel(); else { u1 = A1.locate(ts, !after); v1 = A1.voxel(u1); }
    if (A2.zero) v2 = A2.zero_voxel(); else { u2 = A2.locate(ts, !after); v2 = A2.voxel(u2); }
    if (v0 < 0 || v0 >= R || v1 < 0 || v1 >= R || v2 < 0 || v2 >= R) return;
    const float inf = __builtin_huge_valf();
    if (!kVdb) {
        DenseCursor c;
        c.bits = g.bits;
        c.level_base = (uint64_t)lev * R * R * R;
        c.R = R;
        c.A0 = A0; c.A1 = A1; c.A2 = A2;
        c.u0 = u0; c.u1 = u1; c.u2 = u2;
        c.v0 = v0; c.v1 = v1; c.v2 = v2;
        c.tn0 = A0.zero ? inf : A0.Tk(u0 + 1);
        c.tn1 = A1.zero ? inf : A1.Tk(u1 + 1);
        c.tn2 = A2.zero ? inf : A2.Tk(u2 + 1);
        drive<kSkip>(c, a, b, lat.tmax, vis);
    } else {
        VdbCursor c;
        c.g = &g;
        c.lev = lev;
        c.R = R;
        c.A0 = A0; c.A1 = A1; c.A2 = A2;
        c.u0 = u0; c.u1 = u1; c.u2 = u2;
        c.v0 = v0; c.v1 = v1; c.v2 = v2;
        c.tn_ok = false;
        c.leaf = nullptr;
        c.word_x = -1;
        c.D = 1;
        drive<kSkip>(c, a, b, lat.tmax, vis);
    }
}

__device__ __forceinline__ bool span_of(const GridView &g, int lev, const float o[3], const float d[3], float &E,
                                        float &X) {
    const float *box = g.boxes + 6 * lev;
    Axis A0 = make_axis(box, 0, g.R, o[0], d[0]);
    Axis A1 = make_axis(box, 1, g.R, o[1], d[1]);
    Axis A2 = make_axis(box, 2, g.R, o[2], d[2]);
    return level_span(A0, A1, A2, E, X);
}

// All samples of one ray, in increasing t.  The cascade boxes are nested
// (checked when the grid is built), so level l holds exactly (E_l, X_l] and
// these intervals nest; with f the finest level the ray meets, the owner of
// t runs l = L-1 .. f+1 on (E_l, E_{l-1}], f on (E_f, X_f], then
// l = f+1 .. L-1 on (X_{l-1}, X_l].
template <bool kVdb, bool kSkip, class Vis>
__device__ void trace_ray(const GridView &g, const float o[3], const float d[3], const Lattice &lat, Vis &vis) {
    if (!(lat.tmin <= lat.tmax)) return;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (!__builtin_isfinite(o[a]) || !__builtin_isfinite(d[a])) return;
    const int L = g.L;
    int f = -1;
    float Ef = 0.0f, Xf = 0.0f;
    for (int lev = 0; lev < L; ++lev) {
        if (span_of(g, lev, o, d, Ef, Xf)) {
            f = lev;
            break;
        }
    }
    if (f < 0) return;
    // coarse levels on the way in
    if (f + 1 < L) {
        float E_outer, X_unused;
        span_of(g, L - 1, o, d, E_outer, X_unused);
        for (int lev = L - 1; lev > f; --lev) {
            float E_inner = Ef, X_tmp;
            if (lev - 1 > f) span_of(g, lev - 1, o, d, E_inner, X_tmp);
            march_segment<kVdb, kSkip>(g, lev, o, d, E_outer, E_inner, lat, vis);
            E_outer = E_inner;
        }
    }
    march_segment<kVdb, kSkip>(g, f, o, d, Ef, Xf, lat, vis);
    // coarse levels on the way out
    float X_inner = Xf;
    for (int lev = f + 1; lev < L; ++lev) {
        float E_tmp, X_outer;
        span_of(g, lev, o, d, E_tmp, X_outer);
        if (X_inner >= lat.tmax) break;
        march_segment<kVdb, kSkip>(g, lev, o, d, X_inner, X_outer, lat, vis);
        X_inner = X_outer;
    }
}

// ------------------------------------------------------------------ kernels

__device__ __forceinline__ void load_ray(const float *origins, const float *dirs, int64_t i, float o[3], float d[3]) {
    o[0] = origins[3 * i + 0];
    o[1] = origins[3 * i + 1];
    o[2] = origins[3 * i + 2];
    d[0] = dirs[3 * i + 0];
    d[1] = dirs[3 * i + 1];
    d[2] = dirs[3 * i + 2];
}

template <bool kVdb, bool kSkip>
__global__ void __launch_bounds__(kBlock) count_kernel(GridView g, const float *__restrict__ origins,
                                                       const float *__restrict__ dirs, int64_t n_rays, Lattice lat,
                                                       int32_t *__restrict__ counts) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_rays) return;
    float o[3], d[3];
    load_ray(origins, dirs, i, o, d);
    CountVis vis{&lat, 0};
    trace_ray<kVdb, kSkip>(g, o, d, lat, vis);
    counts[i] = vis.n;
}

template <bool kVdb, bool kSkip, bool kVox>
__global__ void __launch_bounds__(kBlock) fill_kernel(GridView g, const float *__restrict__ origins,
                                                      const float *__restrict__ dirs, int64_t n_rays, Lattice lat,
                                                      const int64_t *__restrict__ offsets, int64_t capacity,
                                                      int32_t *__restrict__ ray_ids, float *__restrict__ t0,
                                                      float *__restrict__ t1, int32_t *__restrict__ vox) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_rays) return;
    int64_t first = offsets[i];
    if (first >= capacity) return;
    float o[3], d[3];
    load_ray(origins, dirs, i, o, d);
    FillVis<kVox> vis;
    vis.lat = &lat;
    vis.idx = first;
    vis.capacity = capacity;
    vis.ray = (int32_t)i;
    vis.ray_ids = ray_ids;
    vis.t0 = t0;
    vis.t1 = t1;
    vis.vox = vox;
    vis.lev = 0;
    vis.R = g.R;
    trace_ray<kVdb, kSkip>(g, o, d, lat, vis);
}

// Growing-step lattice, one thread: t_0 = near, t_{k+1} = fl(t_k +
// max(fl(t_k*cone), dt_min)), stored up to and including the first value
// past far.  n_tab = -1 if the capacity ran out first.
__global__ void cone_table_kernel(float tmin, float tmax, float cone, float dt_min, float *tab, int32_t cap,
                                  int32_t *n_tab) {
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
    *n_tab = (k > 0 && tab[k - 1] > tmax) ? k : -1;
}

__global__ void zero_kernel(int64_t *p, int32_t *q) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (p) *p = 0;
        if (q) *q = 0;
    }
}

// ------------------------------------------------------------------ host

namespace {

struct Plan {
    int64_t n_rays;
    size_t off_counts, off_tiles, off_tab, off_ntab, total;
    int64_t n_tiles;
    int32_t tab_cap;
};

bool make_plan(int64_t n_rays, float near_t, float far_t, const ogv_step *step, Plan *p, std::string *why) {
    p->n_rays = n_rays;
    p->n_tiles = scan_tiles(n_rays);
    p->tab_cap = 0;
    if (step->kind == OGV_STEP_CONE && far_t >= near_t) {
        // Upper bound on the growing-step lattice length up to the first
        // point past far: every step adds at least dt_min less half an ulp
        // of far, and past dt_min/cone each step multiplies t by at least
        // (1 + cone) up to rounding.
        double ulp = (double)std::nextafter(far_t, INFINITY) - (double)far_t;
        double inc = (double)step->dt_min - 0.5 * ulp;
        double n_lin = std::ceil(((double)far_t - (double)near_t) / inc) + 2.0;
        double n = n_lin;
        if (step->cone > 0.0f && step->cone > 1e-6f) {
            double knee = (double)step->dt_min / (double)step->cone;
            double n_floor = knee > near_t ? std::ceil((knee - (double)near_t) / inc) + 2.0 : 0.0;
            double t_s = knee > near_t ? knee : (double)near_t;
            double rate = std::log1p((double)step->cone) - 4.0 * ldexp(1.0, -24);
            double n_geo = far_t > t_s && t_s > 0 ? std::ceil(std::log((double)far_t / t_s) / rate) + 2.0 : 0.0;
            if (t_s > 0) n = std::min(n_lin, n_floor + n_geo);
        }
        n += 16.0;
        if (!(n <= (double)(1 << 22))) {
            *why = "growing-step lattice longer than 2^22 points";
            return false;
        }
        p->tab_cap = (int32_t)n;
    }
    size_t off = 0;
    p->off_counts = off;
    off = align_up(off + sizeof(int32_t) * (size_t)n_rays, 256);
    p->off_tiles = off;
    off = align_up(off + sizeof(int64_t) * (size_t)(p->n_tiles + 1), 256);
    p->off_tab = off;
    off = align_up(off + sizeof(float) * (size_t)p->tab_cap, 256);
    p->off_ntab = off;
    off = align_up(off + sizeof(int32_t) * 4, 256);
    p->total = off;
    return true;
}

ogv_status validate(const ogv_grid *grid, int32_t variant, const float *o, const float *d, int64_t n_rays,
                    float near_t, float far_t, const ogv_step *step, const char *fn) {
    std::string f(fn);
    if (!grid) OGV_FAIL(OGV_ERR_INVALID, f + ": grid is null");
    if (variant != OGV_BRANCH && variant != OGV_SKIP) OGV_FAIL(OGV_ERR_INVALID, f + ": variant must be 0 or 1");
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

template <bool kVdb, bool kSkip>
void launch_count(const GridView &g, const float *o, const float *d, int64_t n, const Lattice &lat, int32_t *counts,
                  hipStream_t s) {
    unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
    count_kernel<kVdb, kSkip><<<blocks, kBlock, 0, s>>>(g, o, d, n, lat, counts);
}

template <bool kVdb, bool kSkip>
void launch_fill(const GridView &g, const float *o, const float *d, int64_t n, const Lattice &lat,
                 const int64_t *offsets, int64_t cap, int32_t *ids, float *t0, float *t1, int32_t *vox,
                 hipStream_t s) {
    unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
    if (vox) fill_kernel<kVdb, kSkip, true><<<blocks, kBlock, 0, s>>>(g, o, d, n, lat, offsets, cap, ids, t0, t1, vox);
    else fill_kernel<kVdb, kSkip, false><<<blocks, kBlock, 0, s>>>(g, o, d, n, lat, offsets, cap, ids, t0, t1, vox);
}

void dispatch_count(const GridView &g, int variant, const float *o, const float *d, int64_t n, const Lattice &lat,
                    int32_t *counts, hipStream_t s) {
    if (g.kind == 0) {
        if (variant == OGV_SKIP) launch_count<false, true>(g, o, d, n, lat, counts, s);
        else launch_count<false, false>(g, o, d, n, lat, counts, s);
    } else {
        if (variant == OGV_SKIP) launch_count<true, true>(g, o, d, n, lat, counts, s);
        else launch_count<true, false>(g, o, d, n, lat, counts, s);
    }
}

void dispatch_fill(const GridView &g, int variant, const float *o, const float *d, int64_t n, const Lattice &lat,
                   const int64_t *offsets, int64_t cap, int32_t *ids, float *t0, float *t1, int32_t *vox,
                   hipStream_t s) {
    if (g.kind == 0) {
        if (variant == OGV_SKIP) launch_fill<false, true>(g, o, d, n, lat, offsets, cap, ids, t0, t1, vox, s);
        else launch_fill<false, false>(g, o, d, n, lat, offsets, cap, ids, t0, t1, vox, s);
    } else {
        if (variant == OGV_SKIP) launch_fill<true, true>(g, o, d, n, lat, offsets, cap, ids, t0, t1, vox, s);
        else launch_fill<true, false>(g, o, d, n, lat, offsets, cap, ids, t0, t1, vox, s);
    }
}

// Growing-step table into the workspace, padded past its true length with
// its last value (> far) so binary searches over the whole capacity stay on
// written entries.
__global__ void cone_pad_kernel(float *tab, int32_t cap, const int32_t *n_tab) {
    int32_t n = *n_tab;
    if (n <= 0) return;
    float last = tab[n - 1];
    for (int32_t k = n + blockIdx.x * blockDim.x + threadIdx.x; k < cap; k += gridDim.x * blockDim.x) tab[k] = last;
}

ogv_status build_table(float near_t, float far_t, const ogv_step *step, void *ws, const Plan &p, hipStream_t s) {
    if (step->kind != OGV_STEP_CONE || p.tab_cap == 0) return OGV_OK;
    float *tab = (float *)((char *)ws + p.off_tab);
    int32_t *n_tab = (int32_t *)((char *)ws + p.off_ntab);
    cone_table_kernel<<<1, 64, 0, s>>>(near_t, far_t, step->cone, step->dt_min, tab, p.tab_cap, n_tab);
    OGV_CHECK_LAUNCH();
    cone_pad_kernel<<<8, 256, 0, s>>>(tab, p.tab_cap, n_tab);
    OGV_CHECK_LAUNCH();
    return OGV_OK;
}

// count + exclusive scan; offsets[n] = total; overflow (nullable) = total > capacity
ogv_status count_and_scan(const ogv_grid *grid, int32_t variant, const float *o, const float *d, int64_t n,
                          const Lattice &lat, int64_t *offsets, void *ws, const Plan &p, int64_t capacity,
                          int32_t *overflow, hipStream_t s) {
    if (n == 0) {
        zero_kernel<<<1, 64, 0, s>>>(offsets, overflow);
        OGV_CHECK_LAUNCH();
        return OGV_OK;
    }
    int32_t *counts = (int32_t *)((char *)ws + p.off_counts);
    int64_t *tiles = (int64_t *)((char *)ws + p.off_tiles);
    dispatch_count(grid->view, variant, o, d, n, lat, counts, s);
    OGV_CHECK_LAUNCH();
    OGV_CHECK_HIP(launch_excl_scan(counts, n, offsets, tiles, capacity, overflow, s));
    return OGV_OK;
}

ogv_status prepare(const ogv_grid *grid, int32_t variant, const float *o, const float *d, int64_t n, float near_t,
                   float far_t, const ogv_step *step, void *ws, size_t ws_bytes, Plan *p, const char *fn) {
    ogv_status st = validate(grid, variant, o, d, n, near_t, far_t, step, fn);
    if (st != OGV_OK) return st;
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

extern "C" ogv_status ogv_sample_count(const ogv_grid *grid, int32_t variant, const float *o, const float *d,
                                       int64_t n, float near_t, float far_t, const ogv_step *step, int64_t *offsets,
                                       void *ws, size_t ws_bytes, void *stream) {
    Plan p;
    ogv_status st = prepare(grid, variant, o, d, n, near_t, far_t, step, ws, ws_bytes, &p, "ogv_sample_count");
    if (st != OGV_OK) return st;
    if (!offsets) OGV_FAIL(OGV_ERR_INVALID, "offsets is null");
    hipStream_t s = (hipStream_t)stream;
    if ((st = build_table(near_t, far_t, step, ws, p, s)) != OGV_OK) return st;
    Lattice lat = make_lattice(near_t, far_t, step, ws, p);
    return count_and_scan(grid, variant, o, d, n, lat, offsets, ws, p, 0, nullptr, s);
}

extern "C" ogv_status ogv_sample_fill(const ogv_grid *grid, int32_t variant, const float *o, const float *d,
                                      int64_t n, float near_t, float far_t, const ogv_step *step,
                                      const int64_t *offsets, int64_t capacity, int32_t *ray_ids, float *t0,
                                      float *t1, int32_t *vox, void *ws, size_t ws_bytes, void *stream) {
    Plan p;
    ogv_status st = prepare(grid, variant, o, d, n, near_t, far_t, step, ws, ws_bytes, &p, "ogv_sample_fill");
    if (st != OGV_OK) return st;
    if (!offsets) OGV_FAIL(OGV_ERR_INVALID, "offsets is null");
    if (capacity < 0) OGV_FAIL(OGV_ERR_INVALID, "capacity < 0");
    if (capacity > 0 && (!ray_ids || !t0 || !t1)) OGV_FAIL(OGV_ERR_INVALID, "null sample array");
    if (n == 0) return OGV_OK;
    hipStream_t s = (hipStream_t)stream;
    // rebuilt so that fill does not depend on what count left in the workspace
    if ((st = build_table(near_t, far_t, step, ws, p, s)) != OGV_OK) return st;
    Lattice lat = make_lattice(near_t, far_t, step, ws, p);
    dispatch_fill(grid->view, variant, o, d, n, lat, offsets, capacity, ray_ids, t0, t1, vox, s);
    OGV_CHECK_LAUNCH();
    return OGV_OK;
}

extern "C" ogv_status ogv_sample_rays(const ogv_grid *grid, int32_t variant, const float *o, const float *d,
                                      int64_t n, float near_t, float far_t, const ogv_step *step, int64_t *offsets,
                                      int64_t capacity, int32_t *ray_ids, float *t0, float *t1, int32_t *vox,
                                      int32_t *overflow, void *ws, size_t ws_bytes, void *stream) {
    Plan p;
    ogv_status st = prepare(grid, variant, o, d, n, near_t, far_t, step, ws, ws_bytes, &p, "ogv_sample_rays");
    if (st != OGV_OK) return st;
    if (!offsets || !overflow) OGV_FAIL(OGV_ERR_INVALID, "offsets/overflow is null");
    if (capacity < 0) OGV_FAIL(OGV_ERR_INVALID, "capacity < 0");
    if (capacity > 0 && (!ray_ids || !t0 || !t1)) OGV_FAIL(OGV_ERR_INVALID, "null sample array");
    hipStream_t s = (hipStream_t)stream;
    if ((st = build_table(near_t, far_t, step, ws, p, s)) != OGV_OK) return st;
    Lattice lat = make_lattice(near_t, far_t, step, ws, p);
    if ((st = count_and_scan(grid, variant, o, d, n, lat, offsets, ws, p, capacity, overflow, s)) != OGV_OK) return st;
    if (n == 0) return OGV_OK;
    dispatch_fill(grid->view, variant, o, d, n, lat, offsets, capacity, ray_ids, t0, t1, vox, s);
    OGV_CHECK_LAUNCH();
    return OGV_OK;
}
