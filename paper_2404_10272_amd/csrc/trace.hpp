// Device-side ray walk shared by the single-scene and batched samplers:
// dense-grid voxel DDA (the plain method) and VDB + hierarchical DDA
// (Sec. 2.3, Sec. 3), each in the loop structure of Alg. 1 ("DDA branch")
// or Alg. 2 ("DDA skip") of the supplementary material.
//
// One ray per lane.  A ray is split into segments owned by one cascade level
// each (finest level wins, Sec. 3); within a segment a cursor walks cells in
// ray order -- voxels for the dense grid; root tiles, internal-node tiles or
// leaf voxels for the VDB tree -- and the driver turns maximal runs of
// occupied cells into parameter intervals (lo, hi].  A visitor converts an
// interval into its lattice points: the count pass adds their number and
// keeps the runs, the traversal fill writes the samples.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cstdint>

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

// The parts of a VDB tree a walk reads: the root table and the nodes' slot
// tables (staged in LDS when they fit), and the leaves (global memory).
struct Tree {
    const int32_t *root;
    const int32_t *slot;
    const uint64_t *leaves;
    const uint64_t *sub;   // [leaves]: uniform 4^3 sub-blocks
    int ilog2, S, NR;
};

__host__ __device__ inline size_t tree_lds_bytes(int L, int NR, int S) {
    const size_t n_root = (size_t)L * NR * NR * NR;
    return n_root * 4 + n_root * (size_t)S * S * S * 4;
}

// Copies n4 >= 1 16-byte words from global memory to LDS.  A thread issues
// the loads of a batch together and only then stores them, so the block waits
// for one memory round trip per batch rather than one per word.  Indices past
// the end are clamped to the last word, which such lanes load and store again
// with its own value: no branch lets the compiler sink a load to its store.
__device__ __forceinline__ void stage_to_lds(int4 *dst, const int4 *__restrict__ src, int n4) {
    constexpr int kBatch = 4;
    const int nt = (int)blockDim.x, t = (int)threadIdx.x;
    for (int base = 0; base < n4; base += kBatch * nt) {
        int4 r[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) r[u] = src[min(base + u * nt + t, n4 - 1)];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) dst[min(base + u * nt + t, n4 - 1)] = r[u];
    }
}

// The tree's view with its slot and root tables at smem (slot table first,
// then the root table: tree_lds_bytes), as stage_tree leaves them.  Node
// slots exist for every root cell (the worst case the build sizes for).
__device__ __forceinline__ Tree tree_in_lds(const GridView &g, uint32_t *smem) {
    Tree t;
    t.ilog2 = g.ilog2;
    t.S = g.S;
    t.NR = g.NR;
    t.leaves = g.leaves;
    t.sub = g.sub;
    const int ns = g.L * g.NR * g.NR * g.NR * g.S * g.S * g.S;
    t.slot = (const int32_t *)smem;
    t.root = (const int32_t *)smem + ns;
    return t;
}

// Copies the slot and root tables to smem.  Every thread of the block must
// call this (it synchronizes).  smem must be 16-byte aligned; the slot table
// is (the build aligns every table to 256 bytes, and a table holds S^3
// entries per root cell, a multiple of 4).
__device__ __forceinline__ void stage_tree(const GridView &g, uint32_t *smem) {
    const int n_root = g.L * g.NR * g.NR * g.NR;
    const int ns = n_root * g.S * g.S * g.S;
    int32_t *slot = (int32_t *)smem;
    int32_t *root = slot + ns;
    stage_to_lds(reinterpret_cast<int4 *>(slot), reinterpret_cast<const int4 *>(g.slot), ns >> 2);
    for (int i = threadIdx.x; i < n_root; i += blockDim.x) root[i] = g.root[i];
    __syncthreads();
}

// The tree a walk reads: its tables staged in LDS (kLds; every thread of the
// block must call this), or read from global memory.
template <bool kLds>
__device__ __forceinline__ Tree load_tree(const GridView &g, uint32_t *smem) {
    if (kLds) {
        stage_tree(g, smem);
        return tree_in_lds(g, smem);
    }
    Tree t;
    t.ilog2 = g.ilog2;
    t.S = g.S;
    t.NR = g.NR;
    t.leaves = g.leaves;
    t.sub = g.sub;
    t.root = g.root;
    t.slot = g.slot;
    return t;
}

// VDB tree: the current cell is the largest uniform cell holding the current
// voxel -- a root tile (D = 8*S voxels per axis), an internal-node tile
// (D = 8) or a leaf voxel (D = 1); with kSub, inside a leaf also a uniform
// 4^3 sub-block (D = 4: all its 64 voxels empty, or all occupied), so that
// the cells nest as aligned cubes of 8S, 8, 4 and 1 voxels a side and a step
// passes empty space by powers of two down to single voxels (Fig. 1).
// The cell's exit is the first crossing of its far planes (for D = 1 the
// ordinary voxel step).
//
// The walk is incremental, as in a plain DDA: a step moves the stepping axis
// into the next cell and looks that cell up; when it has the same size as the
// cell left, only the stepping axis's exit plane moves (D planes further).
// The other axes stay inside their D-aligned blocks while tiles are crossed,
// so their voxels are only re-located (exactly, at the exit parameter) when
// the walk descends into a finer cell; a change of size recomputes all three
// exits.  Cell sequence and exit parameters equal those of a walk that
// re-locates every axis at every exit.
//
// kTiles = false walks the same tree one voxel per step (the paper's
// "VDB + DDA" rows, Tab. 1-2): a voxel inside a tile takes the tile's value
// and the walk moves on to the next voxel, so the tree only changes how
// occupancy is looked up, not which cells are visited.
//
// kSub trades steps for dearer ones: it takes a fifth to a quarter fewer steps, but
// the cell size changes more often inside leaves, and each change recomputes
// all exits (and, going down, re-locates the other axes and looks the cell up
// again), in some lane of most steps of a wave.  Only 4^3 sub-blocks are
// cells: adding the 2^3 ones (D = 2) saves a few more steps but changes the
// size about twice as often again, which costs more than it saves (object
// walk 0.230 against 0.209 ms, four cascades the same).
template <bool kTiles, bool kSub = false>
struct VdbWalk {
    Tree t;
    int lev, R, sh;
    Axis A0, A1, A2;
    int u0, u1, u2;        // ray-order voxel per moving axis (inside the current cell's block)
    int v0, v1, v2;        // voxel index per axis
    int k0, k1, k2;        // ray-order exit plane of the current cell per moving axis
    float e0, e1, e2;      // their crossing parameters (+inf for zero axes)
    int kx;                // exit plane of the axis exit() chose
    int D;                 // current cell size in voxels
    bool occ;              // current cell occupied
    int lblk;              // cached leaf block (packed block coordinates), -1 if none
    int lbase;             // its first word in the leaf array
    uint32_t lu4;          // its uniform 4^3 sub-blocks (its Tree::sub entry)

    // Size of the largest uniform cell holding voxel (v0, v1, v2) and its
    // occupancy.  A voxel in the cached leaf block (most voxel steps) needs
    // only its word and bit; otherwise the root and slot tables are read and
    // a leaf found there becomes the cached one.  The word is read on every
    // leaf voxel: keeping the last one costs a divergent branch per step,
    // which is dearer than the (cached) load.
    __device__ __forceinline__ int classify(bool &o) {
        const int blk = ((v0 >> 3) << 20) | ((v1 >> 3) << 10) | (v2 >> 3);
        int D = 1;
        if (blk != lblk) {
            const int NR = t.NR;
            const int ri = NR == 1 ? lev : ((lev * NR + (v0 >> sh)) * NR + (v1 >> sh)) * NR + (v2 >> sh);
            const int node = t.root[ri];
            const int lg = t.ilog2, m = t.S - 1;
            const int s = (((v0 >> 3) & m) << (2 * lg)) | (((v1 >> 3) & m) << lg) | ((v2 >> 3) & m);
            const int c = t.slot[(max(node, 0) << (3 * lg)) | s];
            const bool root_tile = node < 0;
            const bool slot_tile = !root_tile && c < 0;
            if (!root_tile && !slot_tile) {
                lblk = blk;
                lbase = c * 8;
                if (kSub) lu4 = (uint32_t)t.sub[c];
            } else {
                o = root_tile ? node == -2 : c == -2;
                return kTiles ? (root_tile ? (8 << t.ilog2) : 8) : 1;
            }
        }
        const uint64_t word = t.leaves[lbase + (v0 & 7)];
        const int bit = ((v1 & 7) << 3) | (v2 & 7);
        const uint32_t half = bit < 32 ? (uint32_t)word : (uint32_t)(word >> 32);
        o = ((half >> (bit & 31)) & 1u) != 0;
        if (kSub) {
            // a uniform 4^3 sub-block takes the voxel's value and is the cell
            const int s4 = (((v0 >> 2) & 1) << 2) | (((v1 >> 2) & 1) << 1) | ((v2 >> 2) & 1);
            D = ((lu4 >> s4) & 1u) != 0 ? 4 : 1;
        }
        return D;
    }

    // exit planes and parameters of every moving axis for cells of size D.
    // Every axis is computed and a zero axis's parameter replaced by +inf
    // afterwards: a per-axis branch here costs more than the arithmetic.
    __device__ __forceinline__ void exits_all() {
        const float inf = __builtin_huge_valf();
        const int msk = ~(D - 1);
        const int b0 = v0 & msk, b1 = v1 & msk, b2 = v2 & msk;
        k0 = A0.pos ? b0 + D : R - b0;
        k1 = A1.pos ? b1 + D : R - b1;
        k2 = A2.pos ? b2 + D : R - b2;
        e0 = A0.zero ? inf : A0.Tk(k0);
        e1 = A1.zero ? inf : A1.Tk(k1);
        e2 = A2.zero ? inf : A2.Tk(k2);
    }

    // the cell holding the current voxels becomes current
    __device__ __forceinline__ void enter() {
        bool o;
        D = classify(o);
        occ = o;
        exits_all();
    }

    __device__ __forceinline__ bool occupied() const { return occ; }

    // first exit crossing; also keeps that axis's exit plane for step()
    __device__ __forceinline__ float exit(int &axis) {
        float hi = e0;
        int k = k0;
        axis = 0;
        if (e1 < hi) { hi = e1; k = k1; axis = 1; }
        if (e2 < hi) { hi = e2; k = k2; axis = 2; }
        kx = k;
        return hi;
    }

    // moves into the next cell across the exit found by exit(); false when
    // that leaves the grid
    __device__ __forceinline__ bool step(int axis, float t) {
        const int ka = kx;
        if (ka >= R) return false;
        if (axis == 0) { u0 = ka; v0 = A0.voxel(ka); }
        if (axis == 1) { u1 = ka; v1 = A1.voxel(ka); }
        if (axis == 2) { u2 = ka; v2 = A2.voxel(ka); }
        bool o;
        int Dn = classify(o);
        if (Dn == D) {
            // same cell size: the next exit along the stepping axis is D planes on
            if (axis == 0) { k0 += D; e0 = A0.Tk(k0); }
            if (axis == 1) { k1 += D; e1 = A1.Tk(k1); }
            if (axis == 2) { k2 += D; e2 = A2.Tk(k2); }
        } else {
            if (Dn < D) {
                // descending out of a tile: voxels of the other axes at t, inside their blocks
                if (axis != 0 && !A0.zero) { u0 = A0.advance_to(u0, t, min(k0, R) - 1); v0 = A0.voxel(u0); }
                if (axis != 1 && !A1.zero) { u1 = A1.advance_to(u1, t, min(k1, R) - 1); v1 = A1.voxel(u1); }
                if (axis != 2 && !A2.zero) { u2 = A2.advance_to(u2, t, min(k2, R) - 1); v2 = A2.voxel(u2); }
                Dn = classify(o);
            }
            D = Dn;
            exits_all();
        }
        occ = o;
        return true;
    }
};

// ------------------------------------------------------------------ driver

// Walks cells from the segment start a to its end b (or t_max) and reports
// maximal occupied runs (lo, hi] to the visitor, from a single call site.
// kSkip = false is Alg. 1 (every cell visited, branch on occupancy);
// kSkip = true is Alg. 2 (an inner loop passes all leading empty cells, then
// the occupied run is marched).
template <bool kSkip, class Cursor, class Vis, class Ctx>
__device__ __forceinline__ void drive(Cursor &c, float a, float b, float tmax, Vis &vis, const Ctx &ctx) {
    float lo = a;
    if (!kSkip) {
        bool in_run = false;
        float run_lo = a;
        while (true) {
            bool occ = c.occupied();
            int axis;
            float hi = c.exit(axis);
            if (occ && !in_run) {
                in_run = true;
                run_lo = lo;
            }
            bool end = hi >= b || hi >= tmax;
            if (!end) end = !c.step(axis, hi);
            // a run closes at lo on an empty cell, or at this cell's end when the ray ends
            if (in_run && (!occ || end)) {
                vis.run(ctx, run_lo, occ ? fminf(hi, b) : lo);
                in_run = false;
            }
            if (end) return;
            lo = hi;
        }
    } else {
        while (true) {
            bool end = false;
            while (!c.occupied()) {
                int axis;
                float hi = c.exit(axis);
                if (hi >= b || hi >= tmax || !c.step(axis, hi)) return;
                lo = hi;
            }
            float run_lo = lo, run_hi;
            while (true) {
                int axis;
                float hi = c.exit(axis);
                end = hi >= b || hi >= tmax;
                if (!end) end = !c.step(axis, hi);
                run_hi = fminf(hi, b);
                lo = hi;
                if (end || !c.occupied()) break;
            }
            vis.run(ctx, run_lo, run_hi);
            if (end) return;
        }
    }
}

// ------------------------------------------------------------------ visitors

// Count pass: number of lattice points in each occupied run, and the runs
// themselves as lattice-index ranges [n0, n1) (adjacent ranges merged) for
// the expansion fill.  A ray keeps its first kMaxRuns runs in fixed slots;
// further runs go to chunks of kMaxRuns slots taken from a shared pool and
// chained (ray_next -> pool_next -> ...).  If the pool runs dry the ray is
// marked kRunsLost, listed, and the traversal fill writes it instead.
//
// During the walk a run is only recorded, as the bits of its parameter
// interval (lo, hi]; its lattice range is found once the walk has ended, in
// a loop over the ray's recorded runs that also merges adjacent ranges and
// rewrites them in place.  Lanes close runs at different steps, so doing the
// lattice arithmetic at the close would run it, masked, in most steps of a
// wave; after the walk the lanes of a wave do it together.
constexpr int kMaxRuns = 16;
constexpr int32_t kRunsLost = 0x7fffffff;

struct RunPool {
    int2 *slots;          // [kMaxRuns][stride]: slot k of ray r at k * stride + r (reads of one slot coalesce)
    int64_t stride;       // rays the slot array is laid out for
    int32_t *ray_next;    // [rays]: first pool chunk of the ray, -1 if none
    int2 *chunks;         // [cap][kMaxRuns]
    int32_t *chunk_next;  // [cap]
    int32_t *head;        // chunks handed out so far
    int32_t cap;
    int32_t *lost;        // [rays]: rays marked kRunsLost, in no particular order
    int32_t *n_lost;      // their number
};

// Uniform context of the count pass.
struct CountCtx {
    Lattice lat;
    RunPool pool;
};

// Per-lane state of the count pass.
struct CountVis {
    int32_t n;            // samples
    int32_t nr;           // runs recorded (kRunsLost: pool exhausted); after finish(), runs kept
    int32_t kept;         // runs recorded before the pool ran dry
    int64_t ray;
    int32_t first;        // first pool chunk of the ray, -1 if none
    int32_t chunk;        // last pool chunk taken

    __device__ __forceinline__ void begin_level(int, const Axis &, const Axis &, const Axis &) {}

    // slot k of the ray (k >= kMaxRuns: slot k % kMaxRuns of pool chunk c)
    __device__ __forceinline__ int2 *slot(const RunPool &pool, int k, int32_t c) const {
        return k < kMaxRuns ? pool.slots + (int64_t)k * pool.stride + ray : pool.chunks + (int64_t)c * kMaxRuns + k % kMaxRuns;
    }
    // records run nr; false (and the ray marked lost) if the pool is dry
    __device__ __forceinline__ bool record(const RunPool &pool, int2 v) {
        if (nr >= kMaxRuns && nr % kMaxRuns == 0) {
            const int32_t c = atomicAdd(pool.head, 1);
            if (c >= pool.cap) {
                kept = nr;
                nr = kRunsLost;
                return false;
            }
            pool.chunk_next[c] = -1;
            if (nr == kMaxRuns) {
                pool.ray_next[ray] = c;
                first = c;
            } else {
                pool.chunk_next[chunk] = c;
            }
            chunk = c;
        }
        *slot(pool, nr, chunk) = v;
        ++nr;
        return true;
    }
    // lattice points of (lo, hi] up to t_max: [n0, n1), empty when n1 <= n0
    __device__ __forceinline__ static int2 lattice_range(const Lattice &lat, float lo, float hi) {
        return make_int2(lat.first_above(lo), lat.first_above(fminf(hi, lat.tmax)));
    }
    __device__ __forceinline__ void run(const CountCtx &x, float lo, float hi) {
        if (nr != kRunsLost && record(x.pool, make_int2(__float_as_int(lo), __float_as_int(hi)))) return;
        // the pool is dry: this ray is re-walked by the fill, only its count is needed
        const int2 q = lattice_range(x.lat, lo, hi);
        n += max(q.y - q.x, 0);
    }
    // Lattice ranges of the recorded runs, merged where one ends at the next's
    // start and written back over the recorded runs (the write index never
    // passes the read index).
    __device__ __forceinline__ void finish(const CountCtx &x) {
        const bool lost = nr == kRunsLost;
        const int m = lost ? kept : nr;
        int w = 0;
        int32_t c0 = 0, c1 = 0;          // merged range held back (c1 > c0 when held)
        int32_t rc = first, wc = first;  // pool chunks of the read and write positions
        for (int k = 0; k < m; ++k) {
            if (k > kMaxRuns && k % kMaxRuns == 0) rc = x.pool.chunk_next[rc];
            const int2 raw = *slot(x.pool, k, rc);
            const int2 q = lattice_range(x.lat, __int_as_float(raw.x), __int_as_float(raw.y));
            if (q.y <= q.x) continue;
            n += q.y - q.x;
            if (c1 > c0 && c1 == q.x) {
                c1 = q.y;
                continue;
            }
            if (c1 > c0 && !lost) {
                if (w > kMaxRuns && w % kMaxRuns == 0) wc = x.pool.chunk_next[wc];
                *slot(x.pool, w, wc) = make_int2(c0, c1);
                ++w;
            }
            c0 = q.x;
            c1 = q.y;
        }
        if (c1 > c0 && !lost) {
            if (w > kMaxRuns && w % kMaxRuns == 0) wc = x.pool.chunk_next[wc];
            *slot(x.pool, w, wc) = make_int2(c0, c1);
            ++w;
        }
        if (lost) x.pool.lost[atomicAdd(x.pool.n_lost, 1)] = (int32_t)ray;
        else nr = w;
    }
};

__device__ __forceinline__ CountVis make_count_vis(int64_t ray, const RunPool &pool) {
    CountVis v;
    v.n = 0;
    v.nr = 0;
    v.kept = 0;
    v.ray = ray;
    v.first = -1;
    v.chunk = -1;
    pool.ray_next[ray] = -1;
    return v;
}

// Uniform context of the traversal fill.
struct FillCtx {
    Lattice lat;
    int64_t capacity;
    int32_t *ray_ids;
    float *t0, *t1;
    int32_t *vox;         // written when kVox
    int R;
};

// Per-lane state of the traversal fill.
template <bool kVox>
struct FillVis {
    int64_t idx;
    int32_t ray;
    int lev;
    Axis A0, A1, A2;      // level geometry, for voxel ids only

    __device__ __forceinline__ void begin_level(int l, const Axis &a0, const Axis &a1, const Axis &a2) {
        lev = l;
        if (kVox) {
            A0 = a0;
            A1 = a1;
            A2 = a2;
        }
    }
    __device__ __forceinline__ static int vcoord(const Axis &A, float t) {
        return A.zero ? A.zero_voxel() : A.voxel(A.locate(t, false));
    }
    __device__ __forceinline__ void run(const FillCtx &x, float lo, float hi) {
        int n0 = x.lat.first_above(lo);
        int n1 = x.lat.first_above(fminf(hi, x.lat.tmax));
        float tn = x.lat.t(n0);
        for (int n = n0; n < n1; ++n) {
            float tnext = x.lat.t(n + 1);
            if (idx < x.capacity) {
                x.ray_ids[idx] = ray;
                x.t0[idx] = tn;
                x.t1[idx] = tnext;
                if (kVox) {
                    int i = vcoord(A0, tn), j = vcoord(A1, tn), k = vcoord(A2, tn);
                    x.vox[idx] = ((lev * x.R + i) * x.R + j) * x.R + k;
                }
            }
            ++idx;
            tn = tnext;
        }
    }
};

// Dense bitfield with chessboard distances (a traversal the paper discusses
// but does not evaluate, Sec. 2.3 and Fig. 1): in an empty voxel at distance d >= 2 from
// every occupied voxel, the whole cube of voxels within d - 1 of it is empty,
// so the ray leaves that cube in one step.  The cube's exit planes are the
// current voxel's ray-order index plus d per axis; after the exit, the axes
// it did not leave through are re-located exactly at the exit parameter
// within the cube (the search the VDB walk uses on descent).  Occupied voxels
// and empty ones at distance 1 are single cells, stepped as by the dense
// march.
struct DistCursor {
    const uint32_t *bits;
    const uint8_t *dist;
    uint64_t level_base;   // index of the level's voxel (0,0,0)
    int R;
    Axis A0, A1, A2;
    int u0, u1, u2;        // ray-order voxel per moving axis
    int v0, v1, v2;        // voxel index per axis
    int k0, k1, k2;        // ray-order exit plane of the current cell per moving axis
    float e0, e1, e2;      // their crossing parameters (+inf for zero axes)
    int kx;                // exit plane of the axis exit() chose
    int h;                 // the current cell reaches h voxels past the current voxel (0: a single voxel)
    bool occ;

    __device__ __forceinline__ void classify() {
        const uint64_t idx = level_base + ((uint64_t)((uint32_t)v0 * (uint32_t)R + (uint32_t)v1) * (uint32_t)R + (uint32_t)v2);
        const int d = dist[idx];
        occ = d == 0;
        h = d >= 2 ? d - 1 : 0;
    }
    // every axis computed, a zero axis's parameter replaced by +inf (cheaper
    // than a per-axis branch)
    __device__ __forceinline__ void exits_all() {
        const float inf = __builtin_huge_valf();
        k0 = min(u0 + h + 1, R);
        k1 = min(u1 + h + 1, R);
        k2 = min(u2 + h + 1, R);
        e0 = A0.zero ? inf : A0.Tk(k0);
        e1 = A1.zero ? inf : A1.Tk(k1);
        e2 = A2.zero ? inf : A2.Tk(k2);
    }
    __device__ __forceinline__ void enter() {
        classify();
        exits_all();
    }
    __device__ __forceinline__ bool occupied() const { return occ; }
    __device__ __forceinline__ float exit(int &axis) {
        float hi = e0;
        int k = k0;
        axis = 0;
        if (e1 < hi) { hi = e1; k = k1; axis = 1; }
        if (e2 < hi) { hi = e2; k = k2; axis = 2; }
        kx = k;
        return hi;
    }
    __device__ __forceinline__ bool step(int axis, float t) {
        const int ka = kx;
        if (ka >= R) return false;
        const int h_old = h;
        if (axis == 0) { u0 = ka; v0 = A0.voxel(ka); }
        if (axis == 1) { u1 = ka; v1 = A1.voxel(ka); }
        if (axis == 2) { u2 = ka; v2 = A2.voxel(ka); }
        if (h_old > 0) {
            // out of an empty cube: the other axes' voxels at t, inside the cube
            if (axis != 0 && !A0.zero) { u0 = A0.advance_to(u0, t, k0 - 1); v0 = A0.voxel(u0); }
            if (axis != 1 && !A1.zero) { u1 = A1.advance_to(u1, t, k1 - 1); v1 = A1.voxel(u1); }
            if (axis != 2 && !A2.zero) { u2 = A2.advance_to(u2, t, k2 - 1); v2 = A2.voxel(u2); }
        }
        classify();
        if (h_old == 0 && h == 0) {
            // one voxel to the next: only the stepping axis's exit moves
            if (axis == 0) { k0 = ka + 1; e0 = A0.Tk(k0); }
            if (axis == 1) { k1 = ka + 1; e1 = A1.Tk(k1); }
            if (axis == 2) { k2 = ka + 1; e2 = A2.Tk(k2); }
        } else {
            exits_all();
        }
        return true;
    }
};

// ------------------------------------------------------------------ ray

struct Ray {
    float o0, o1, o2, d0, d1, d2, r0, r1, r2;
};

// Traversals: 0 dense bitfield, 1 VDB tree with hierarchical steps, 2 dense
// bitfield with chessboard distances (GridView::kind 0, 1, 2), 3 the VDB
// tree walked one voxel per step and 4 the VDB tree with hierarchical steps
// that also pass uniform sub-blocks inside leaves (both on kind-1 grids).
template <int kGrid>
struct CursorOf {
    using type = DenseCursor;
};
template <>
struct CursorOf<1> {
    using type = VdbWalk<true>;
};
template <>
struct CursorOf<2> {
    using type = DistCursor;
};
template <>
struct CursorOf<3> {
    using type = VdbWalk<false>;
};
template <>
struct CursorOf<4> {
    using type = VdbWalk<true, true>;
};

// Traversals that read the VDB tree.
constexpr bool reads_tree(int kGrid) { return kGrid == 1 || kGrid == 3 || kGrid == 4; }

// Puts the cursor of level `lev` on the voxel owning t_min when t_min lies
// after the segment start a, else on the voxel owning the parameters just
// after a.  False when that voxel is outside the grid.
template <int kGrid, class Vis>
__device__ __forceinline__ bool cursor_begin(typename CursorOf<kGrid>::type &c, const GridView &g, const Tree &tree,
                                             int lev, const Ray &ray, float a, const Lattice &lat, Vis &vis) {
    const int R = g.R;
    Axis A0 = load_axis(g.geom, lev, 0, R, ray.o0, ray.d0, ray.r0);
    Axis A1 = load_axis(g.geom, lev, 1, R, ray.o1, ray.d1, ray.r1);
    Axis A2 = load_axis(g.geom, lev, 2, R, ray.o2, ray.d2, ray.r2);
    vis.begin_level(lev, A0, A1, A2);
    const bool after = lat.tmin > a;
    const float ts = after ? lat.tmin : a;
    int u0 = A0.zero ? 0 : A0.locate(ts, !after);
    int u1 = A1.zero ? 0 : A1.locate(ts, !after);
    int u2 = A2.zero ? 0 : A2.locate(ts, !after);
    int v0 = A0.zero ? A0.zero_voxel() : A0.voxel(u0);
    int v1 = A1.zero ? A1.zero_voxel() : A1.voxel(u1);
    int v2 = A2.zero ? A2.zero_voxel() : A2.voxel(u2);
    if ((unsigned)v0 >= (unsigned)R || (unsigned)v1 >= (unsigned)R || (unsigned)v2 >= (unsigned)R) return false;
    c.R = R;
    c.A0 = A0; c.A1 = A1; c.A2 = A2;
    c.u0 = u0; c.u1 = u1; c.u2 = u2;
    c.v0 = v0; c.v1 = v1; c.v2 = v2;
    if constexpr (kGrid == 0) {
        const float inf = __builtin_huge_valf();
        c.bits = g.bits;
        c.level_base = (uint64_t)lev * R * R * R;
        c.tn0 = A0.zero ? inf : A0.Tk(u0 + 1);
        c.tn1 = A1.zero ? inf : A1.Tk(u1 + 1);
        c.tn2 = A2.zero ? inf : A2.Tk(u2 + 1);
    } else if constexpr (kGrid == 2) {
        c.bits = g.bits;
        c.dist = g.dist;
        c.level_base = (uint64_t)lev * R * R * R;
        c.k0 = c.k1 = c.k2 = 0;
        c.enter();
    } else {
        c.t = tree;
        c.lev = lev;
        c.sh = 3 + tree.ilog2;
        c.k0 = c.k1 = c.k2 = 0;
        c.lblk = -1;
        c.lbase = 0;
        c.lu4 = 0;
        c.enter();
    }
    return true;
}

template <int kGrid, bool kSkip, class Vis, class Ctx>
__device__ __forceinline__ void march_segment(const GridView &g, const Tree &tree, int lev, const Ray &ray, float a,
                                              float b, const Lattice &lat, Vis &vis, const Ctx &ctx) {
    typename CursorOf<kGrid>::type c;
    if (!cursor_begin<kGrid>(c, g, tree, lev, ray, a, lat, vis)) return;
    drive<kSkip>(c, a, b, lat.tmax, vis, ctx);
}

// Level `lev` holds exactly the parameters (E, X]; false if the ray misses it.
__device__ __forceinline__ bool span_of(const GridView &g, int lev, const Ray &ray, float &E, float &X) {
    Axis A0 = load_axis(g.geom, lev, 0, g.R, ray.o0, ray.d0, ray.r0);
    Axis A1 = load_axis(g.geom, lev, 1, g.R, ray.o1, ray.d1, ray.r1);
    Axis A2 = load_axis(g.geom, lev, 2, g.R, ray.o2, ray.d2, ray.r2);
    return level_span(A0, A1, A2, E, X);
}

// A single-level ray before its walk: the reciprocal direction and the
// grid's span (E, X]; hit is false for a ray with no samples to find (it
// misses the grid, the span lies outside [t_min, t_max], t_min > t_max, or
// the origin or direction is not finite).
struct L1Span {
    Ray ray;
    float E, X;
    bool hit;
};

__device__ __forceinline__ L1Span l1_span(const GridView &g, const float o[3], const float d[3], const Lattice &lat) {
    L1Span s{};
    bool ok = lat.tmin <= lat.tmax;
#pragma unroll
    for (int a = 0; a < 3; ++a) ok = ok && __builtin_isfinite(o[a]) && __builtin_isfinite(d[a]);
    s.ray = Ray{o[0], o[1], o[2], d[0], d[1], d[2], __fdiv_rn(1.0f, d[0]), __fdiv_rn(1.0f, d[1]), __fdiv_rn(1.0f, d[2])};
    s.hit = ok && span_of(g, 0, s.ray, s.E, s.X) && s.E < lat.tmax && s.X >= lat.tmin;
    return s;
}

// Issue priority of a wave from the dense-step estimate of its longest ray:
// sum over axes of |d_a| * len / h_a, with len its span's length inside
// [t_min, t_max], against the grid's resolution R (a ray through the grid
// crosses between R and 3R planes).  The waves of long rays walk longest --
// on a camera looking at an object, the image's centre tiles run for the
// whole launch while most waves end early -- so letting them issue first
// when several waves of a SIMD are ready shortens the launch, and the short
// waves fill the gaps.  The level is made wave-uniform (readfirstlane), so
// the wave takes one scalar branch.  All 64 lanes must call it together.
__device__ __forceinline__ void set_wave_priority(float nv, int R) {
    if (!(nv >= 0.0f)) nv = 0.0f;
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1) nv = fmaxf(nv, __shfl_xor(nv, k));
    const float r = (float)R;
    const int lvl = __builtin_amdgcn_readfirstlane(nv > 1.65f * r ? 3 : nv > 1.15f * r ? 2 : nv > 0.6f * r ? 1 : 0);
    if (lvl == 3) __builtin_amdgcn_s_setprio(3);
    else if (lvl == 2) __builtin_amdgcn_s_setprio(2);
    else if (lvl == 1) __builtin_amdgcn_s_setprio(1);
}

// All samples of one ray, in increasing t.  The cascade boxes are nested
// (checked when the grid is built), so level l holds exactly (E_l, X_l] and
// these intervals nest.  With f the finest level the ray meets and
// m = L-1-f, segment k = 0..2m runs in t order: for k < m level L-1-k on
// (E_{L-1-k}, E_{L-2-k}]; for k = m level f on (E_f, X_f]; for k > m level
// f+(k-m) on (X_{f+k-m-1}, X_{f+k-m}].  Each segment is marched by its level.
// kL1: the grid has a single level (no cascades), so the level geometry is
// uniform across the wave.
template <int kGrid, bool kSkip, bool kL1 = false, class Vis, class Ctx>
__device__ __forceinline__ void trace_ray(const GridView &g, const Tree &tree, const float o[3], const float d[3],
                                          const Lattice &lat, Vis &vis, const Ctx &ctx) {
    if (kL1) {
        const L1Span s = l1_span(g, o, d, lat);
        if (s.hit) march_segment<kGrid, kSkip>(g, tree, 0, s.ray, s.E, s.X, lat, vis, ctx);
        return;
    }
    if (!(lat.tmin <= lat.tmax)) return;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (!__builtin_isfinite(o[a]) || !__builtin_isfinite(d[a])) return;
    Ray ray{o[0], o[1], o[2], d[0], d[1], d[2], __fdiv_rn(1.0f, d[0]), __fdiv_rn(1.0f, d[1]), __fdiv_rn(1.0f, d[2])};
    const int L = g.L;
    int f = -1;
    for (int lev = 0; lev < L && f < 0; ++lev) {
        float E, X;
        if (span_of(g, lev, ray, E, X)) f = lev;
    }
    if (f < 0) return;
    const int m = L - 1 - f;
    for (int k = 0; k <= 2 * m; ++k) {
        // the two levels whose spans bound segment k
        int lev, inner;
        if (k < m) {
            lev = L - 1 - k;
            inner = lev - 1;
        } else if (k == m) {
            lev = f;
            inner = f;
        } else {
            lev = f + (k - m);
            inner = lev - 1;
        }
        float E_l = 0.f, X_l = 0.f, E_i = 0.f, X_i = 0.f;
        for (int q = 0; q < 2; ++q) {
            float E, X;
            span_of(g, q == 0 ? lev : inner, ray, E, X);
            if (q == 0) {
                E_l = E;
                X_l = X;
            } else {
                E_i = E;
                X_i = X;
            }
        }
        float a = k <= m ? E_l : X_i;
        float b = k < m ? E_i : X_l;
        if (a >= lat.tmax) break;   // this and every later segment lie past t_max
        if (a < b && b >= lat.tmin) march_segment<kGrid, kSkip>(g, tree, lev, ray, a, b, lat, vis, ctx);
    }
}

// ------------------------------------------------------------------ expansion fill

// Expansion fill: the output range [offsets[r0], offsets[r0 + 256]) of 256
// consecutive rays (a chunk) is cut into windows of 4-output groups, and a
// block writes its share of them with consecutive lanes on consecutive groups
// (full-wave 16-byte stores).  The rays' kept runs are staged
// in LDS in output order with block-relative first outputs; a ray whose runs
// were lost contributes one placeholder run over its outputs, which the
// traversal fill writes instead, so the runs tile the outputs without gaps.
// The owner of every group comes from a map built per window of groups:
// each run marks the group holding its first output with its index (LDS
// max), and a block-wide max-scan then names, for every group, the last run
// starting at or before its last output.  A lane reads its group's owner and
// looks back over at most three earlier runs; there is no per-output search.
// The run starting last before a window marks the window's first group, so
// each window's map stands alone.  Marks carry the window's number in their
// high bits, so the map is cleared once per chunk: entries left by earlier
// windows are smaller than the current window's first mark.
// The windows of a chunk (2048 groups each, counted from the chunk's first
// group) are dealt round-robin to kExpandParts blocks, so a chunk dense with
// samples does not run its windows one after another in one block while the
// rest of the chip has finished.
// Block-relative offsets fit in 32 bits: a ray has at most 2^24 lattice
// points, so 256 rays stay below 2^32 outputs.
constexpr int kExpandRuns = 1024;     // runs staged per pass
constexpr int kExpandGroups = 2048;   // 4-output groups per owner window
constexpr int kExpandParts = 4;       // blocks sharing one chunk's windows
// Waves per SIMD asked of the expansion kernels: six blocks of 256 lanes per CU
// (LDS allows six).  At the register budget this leaves (80 VGPRs) the
// expansion keeps its loops free of spills; only the rarely taken lost-ray
// traversal spills (the -O1 build; at -O2 the growing-step path spilled as
// well).  An expansion block
// spends much of its life waiting on loads and barriers while the other
// blocks' stores fill HBM, so residency is what keeps the writes flowing.
constexpr int kExpandWaves = 6;
constexpr int kGroupsPerLane = kExpandGroups / kBlock;
constexpr int kOwnerBits = 11;        // owner entries: window number << 11 | (1 + run), run < 1024
// The owner map is padded with one word after every kGroupsPerLane entries:
// the max-scan has lane t read entries kGroupsPerLane*t .. +kGroupsPerLane-1,
// which then sit at words 9t .. 9t+7; with 9 odd, the 32 lanes an LDS access
// serves at a time meet 32 different banks (unpadded, stride 8 put four lanes
// on every bank).
constexpr int kOwnSlots = kExpandGroups + kExpandGroups / kGroupsPerLane;
__device__ __forceinline__ int own_slot(int g) { return g + g / kGroupsPerLane; }

struct OneLattice {       // every ray on one lattice
    static constexpr bool kMulti = false;
    Lattice lat;
    __device__ __forceinline__ int scene_of(int64_t) const { return 0; }
    __device__ __forceinline__ Lattice get(int) const { return lat; }
};

struct SceneLattices {    // ray r on the lattice of its scene
    static constexpr bool kMulti = true;
    const Lattice *lats;   // [n], n <= kBlock
    const int64_t *first;  // first global ray of each scene, [n + 1]
    int n;
    __device__ __forceinline__ int scene_of(int64_t r) const {
        int s = 0;
        while (s + 1 < n && first[s + 1] <= r) ++s;
        return s;
    }
    __device__ __forceinline__ Lattice get(int s) const { return lats[s]; }
};

struct RunReader {
    const int2 *slots;    // [kMaxRuns][stride]
    int64_t stride;
    const int32_t *ray_next;
    const int2 *chunks;
    const int32_t *chunk_next;
};

__device__ __forceinline__ int64_t block_incl_scan256(int64_t x, int64_t *lds, int64_t &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int64_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    int64_t base = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        int64_t v = lds[w];
        if (w < wid) base += v;
        total += v;
    }
    __syncthreads();
    return base + x;   // inclusive
}

// The scan done inside the expansion (one-call sampling): every block derives
// its 256-ray chunk's offsets from the count pass's per-ray counts and its
// sums per 4096-ray scan tile and per 256-ray chunk, and the first part of
// every chunk writes them to the offsets array (the last chunk also the total
// and the overflow flag).  counts == nullptr: the offsets array is read.
constexpr int kChunksPerTile = kScanTile / kBlock;
struct ChunkScan {
    const int32_t *counts;       // [n_rays]
    const int64_t *tile_sums;    // [ceil(n_rays / kScanTile)]
    const int64_t *chunk_sums;   // [ceil(n_rays / kBlock)]
    int32_t *overflow;           // nullable: set to (total > capacity)
};

// First output of ray i from the sums (for the rare rays the count pass could
// not keep runs for; a plain sequential sum).
__device__ inline int64_t offset_of_ray(int64_t i, const ChunkScan &cs) {
    const int64_t c = i / kBlock, T = i / kScanTile;
    int64_t s = 0;
    for (int64_t k = 0; k < T; ++k) s += cs.tile_sums[k];
    for (int64_t j = T * kChunksPerTile; j < c; ++j) s += cs.chunk_sums[j];
    for (int64_t r = c * kBlock; r < i; ++r) s += cs.counts[r];
    return s;
}

// Inclusive block scan of x (returned, with its total) and the block sum of
// y, sharing one exchange through LDS (lds holds 2 * kBlock / 64 entries).
__device__ __forceinline__ int64_t block_scan_and_sum256(int64_t x, int64_t y, int64_t *lds, int64_t &x_total,
                                                        int64_t &y_total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t a = __shfl_up(x, off, 64);
        if (lane >= off) x += a;
        y += __shfl_xor(y, off, 64);
    }
    if (lane == 63) {
        lds[wid] = x;
        lds[kBlock / 64 + wid] = y;
    }
    __syncthreads();
    int64_t below = 0;
    x_total = 0;
    y_total = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        const int64_t v = lds[w];
        if (w < wid) below += v;
        x_total += v;
        y_total += lds[kBlock / 64 + w];
    }
    __syncthreads();
    return below + x;
}

// LDS of one expansion block, declared once per kernel so that the two
// instantiations of expand_chunk share it.
struct ExpandLds {
    uint32_t start[kExpandRuns + 1];   // [cn] bounds the last run of the pass
    uint32_t bn[kExpandRuns];          // n0 - start (mod 2^32): output j has lattice index bn + j
    int32_t ray[kExpandRuns];          // -1: placeholder of a lost ray
    int16_t scene[kExpandRuns];
    uint32_t own[kOwnSlots];           // 1 + owner run of each group of the window, at own_slot(group)
    uint32_t wmax[kBlock / 64];
    int64_t wave[2 * (kBlock / 64)];
};

// kCone: some ray is on a growing-step lattice, whose points come from a table
// in global memory.  Otherwise the write loop issues no load: a load there
// would make every group wait for the stores of the one before (one counter
// covers both on this architecture).
template <bool kCone, bool kScan, class Lats>
__device__ __forceinline__ void expand_chunk(ExpandLds &sh, const float2 *s_lat, int64_t r0, int part,
                                             int64_t *__restrict__ offsets, const ChunkScan &cs, int64_t n_rays,
                                             const int32_t *__restrict__ nruns, const RunReader &rd,
                                             const Lats &lats, int64_t capacity, int32_t *__restrict__ ray_ids,
                                             float *__restrict__ t0, float *__restrict__ t1, bool vec4) {
    uint32_t *const s_start = sh.start, *const s_bn = sh.bn, *const s_own = sh.own, *const s_wmax = sh.wmax;
    int32_t *const s_ray = sh.ray;
    int16_t *const s_scene = sh.scene;
    int64_t *const s_wave = sh.wave;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t r = r0 + threadIdx.x;
    const bool in = r < n_rays;
    const int64_t rc = in ? r : n_rays - 1;   // lanes past the last ray load a valid one's
    int64_t base, bend, off, off_next;
    int nr_rc;
    int2 slot0, slot1;
    if constexpr (kScan) {
        // every load here depends on r alone and is issued in one round: the
        // sums before the chunk (whole tiles, then the earlier chunks of its
        // tile) and the ray's count; the run count and run slots follow once
        // the scan shows whether the ray's outputs meet this part's windows
        const int64_t c = r0 / kBlock, T = r0 / kScanTile;
        if (part > 0) {
            // the chunk's outputs span at most (count + 6) / 4 groups, wherever
            // they start: a part beyond them has no window (and part 0, which
            // writes the chunk's offsets, always goes on)
            if ((cs.chunk_sums[c] + 6) / 4 <= (int64_t)part * kExpandGroups) return;
        }
        int64_t before = 0;
        for (int64_t k = threadIdx.x; k < T; k += kBlock) before += cs.tile_sums[k];
        const int64_t j = T * kChunksPerTile + threadIdx.x;
        if (j < c) before += cs.chunk_sums[j];
        const int64_t cnt = in ? (int64_t)cs.counts[r] : 0;
        int64_t total;
        const int64_t incl = block_scan_and_sum256(cnt, before, s_wave, total, base);
        off = base + incl - cnt;
        off_next = base + incl;
        bend = base + total;
        if (part == 0) {
            if (in) offsets[r] = off;
            if (r0 + kBlock >= n_rays && threadIdx.x == 0) {
                offsets[n_rays] = bend;
                if (cs.overflow) *cs.overflow = bend > capacity ? 1 : 0;
            }
        }
    } else {
        // the chunk's bounds first (uniform loads): a part with no window of
        // the chunk returns before it reads anything per ray
        base = offsets[r0];
        bend = offsets[min(r0 + kBlock, n_rays)];
    }
    const int64_t lim = min(bend, capacity);
    if (lim <= base) return;   // block-uniform: nothing to write
    const int64_t G0 = base >> 2;   // the chunk's first group; windows count from it
    if ((((lim - 1) >> 2) - G0) / kExpandGroups < part) return;   // block-uniform: no window of this part
    // Every other global load of the staging depends on r alone, so all of
    // them are issued here together: one memory round trip (the ray's offsets
    // and run count, and its first two run slots, read whether or not the ray
    // has them; the slot arrays have a column for every ray).
    if constexpr (!kScan) {
        off = offsets[rc];
        off_next = offsets[rc + 1];
        nr_rc = nruns[rc];
        slot0 = rd.slots[rc];
        slot1 = rd.slots[rd.stride + rc];
    }
    bool mine = in;
    if constexpr (kScan) {
        // With the offsets computed here, a part stages only the rays whose
        // outputs meet one of its windows (w = part, part + kExpandParts, ...),
        // and only those rays' run counts and first run slots are read: the
        // windows are tiled by such rays, and the other parts write the rest.
        // This cuts the expansion's reads by more than half.  The three-call
        // form, whose offsets come from memory, measured slower with it and
        // keeps every ray.
        mine = in && off_next > off;
        if (mine) {
            const int64_t wa = ((off >> 2) - G0) / kExpandGroups, wb = (((off_next - 1) >> 2) - G0) / kExpandGroups;
            mine = wa + ((part - (int)(wa % kExpandParts)) + kExpandParts) % kExpandParts <= wb;
        }
        nr_rc = 0;
        slot0 = slot1 = make_int2(0, 0);
        if (mine) {
            nr_rc = nruns[rc];
            slot0 = rd.slots[rc];
            slot1 = rd.slots[rd.stride + rc];
        }
    }
    const int nr_raw = mine ? nr_rc : 0;
    const uint32_t end_rel = (uint32_t)(bend - base);
    const uint32_t lim_rel = (uint32_t)(min(bend, capacity) - base);
    int nr = nr_raw, scene = 0;
    const bool lost = nr_raw == kRunsLost;
    const uint32_t start = in ? (uint32_t)(off - base) : 0u;
    const uint32_t lost_len = lost ? (uint32_t)(off_next - off) : 0u;
    if (lost) nr = lost_len > 0 ? 1 : 0;
    if (in) scene = lats.scene_of(r);
    for (int i = threadIdx.x; i < kOwnSlots; i += kBlock) s_own[i] = 0;
    int64_t total;
    const int rb = (int)(block_incl_scan256((int64_t)nr, s_wave, total) - nr);
    uint32_t epoch = 0;   // window number within the block
    for (int c0 = 0; c0 < (int)total; c0 += kExpandRuns) {
        const int cn = min((int)total - c0, kExpandRuns);
        // stage runs c0 .. c0+cn-1; slot cn takes the next pass's first start.
        uint32_t st = start;
        int32_t chunk = -1;
        const int2 *sp = rd.slots + r;
        const int2 r0v = lost ? make_int2(0, (int)lost_len) : slot0, r1v = slot1;
        for (int k = 0; k < nr; ++k) {
            int2 rn = k == 0 ? r0v : r1v;
            if (!lost && k >= 2) {
                if (k < kMaxRuns) {
                    rn = sp[(int64_t)k * rd.stride];
                } else {
                    if (k % kMaxRuns == 0) chunk = k == kMaxRuns ? rd.ray_next[r] : rd.chunk_next[chunk];
                    rn = rd.chunks[(int64_t)chunk * kMaxRuns + k % kMaxRuns];
                }
            }
            const int idx = rb + k - c0;
            if (idx >= 0 && idx <= cn) s_start[idx] = st;
            if (idx >= 0 && idx < cn) {
                s_bn[idx] = (uint32_t)rn.x - st;
                s_ray[idx] = lost ? -1 : (int32_t)r;
                s_scene[idx] = (int16_t)scene;
            }
            st += (uint32_t)(rn.y - rn.x);
        }
        if (threadIdx.x == 0 && c0 + cn == (int)total) s_start[cn] = end_rel;
        __syncthreads();
        const uint32_t lo = s_start[0];
        const uint32_t hi = min(s_start[cn], lim_rel);
        if (hi > lo) {
            // absolute groups of 4 outputs covering [base + lo, base + hi)
            const int64_t g_first = (base + lo) >> 2, g_last = (base + hi - 1) >> 2;
            // this part's windows that meet the pass: w = part, part + kExpandParts, ...
            int64_t w = (g_first - G0) / kExpandGroups;
            w += ((part - (int)(w % kExpandParts)) + kExpandParts) % kExpandParts;
            for (; G0 + w * kExpandGroups <= g_last; w += kExpandParts) {
                const int64_t gw = max(g_first, G0 + w * kExpandGroups);
                const int nwin = (int)(min(g_last, G0 + (w + 1) * kExpandGroups - 1) - gw + 1);
                const uint32_t tag = ++epoch << kOwnerBits;
                for (int a = threadIdx.x; a < cn; a += kBlock) {
                    const int64_t g = ((base + s_start[a]) >> 2) - gw;
                    if (g >= nwin) continue;
                    // a run starting before the window marks group 0 if it is the last such run
                    // (run 0 starts at or before gw, so group 0 always holds a mark of this window)
                    if (g >= 0 || a + 1 == cn || ((base + s_start[a + 1]) >> 2) >= gw)
                        atomicMax(&s_own[own_slot(g > 0 ? (int)g : 0)], tag | (uint32_t)(a + 1));
                }
                __syncthreads();
                // block-wide inclusive max-scan of s_own
                uint32_t v[kGroupsPerLane];
                uint32_t m = 0;
#pragma unroll
                for (int e = 0; e < kGroupsPerLane; ++e) {
                    m = max(m, s_own[(kGroupsPerLane + 1) * threadIdx.x + e]);
                    v[e] = m;
                }
                uint32_t incl = m;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const uint32_t y = __shfl_up(incl, off, 64);
                    if (lane >= off) incl = max(incl, y);
                }
                if (lane == 63) s_wmax[wid] = incl;
                __syncthreads();
                uint32_t pre = 0;
                for (int q = 0; q < wid; ++q) pre = max(pre, s_wmax[q]);
                const uint32_t below = __shfl_up(incl, 1, 64);
                if (lane > 0) pre = max(pre, below);
#pragma unroll
                for (int e = 0; e < kGroupsPerLane; ++e) s_own[(kGroupsPerLane + 1) * threadIdx.x + e] = max(pre, v[e]);
                __syncthreads();
                // each lane writes groups k = tid, tid + 256, ... of the window
                for (int k = threadIdx.x; k < nwin; k += kBlock) {
                    const int a = (int)(s_own[own_slot(k)] & ((1u << kOwnerBits) - 1)) - 1;   // owns the group's last output
                    const int64_t j4 = 4 * (gw + k) - base;       // block-relative, may lie below lo
                    // runs a-1, a-2, a-3 may own the group's earlier outputs
                    const uint32_t sa = s_start[a];
                    const uint32_t sb = a >= 1 ? s_start[a - 1] : 0u;
                    const uint32_t sc = a >= 2 ? s_start[a - 2] : 0u;
                    int32_t id[4];
                    float x0[4], x1[4];
                    bool ok[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int64_t j = j4 + q;
                        ok[q] = j >= (int64_t)lo && j < (int64_t)hi;
                        const uint32_t ju = (uint32_t)j;
                        const int aq = a - (int)(sa > ju) - (int)(a >= 1 && sb > ju) - (int)(a >= 2 && sc > ju);
                        const int b = ok[q] ? aq : a;
                        id[q] = s_ray[b];
                        ok[q] = ok[q] && id[q] >= 0;
                        const int n = (int)(s_bn[b] + ju);
                        if constexpr (kCone) {
                            const Lattice L = lats.get(s_scene[b]);
                            x0[q] = ok[q] ? L.t(n) : 0.0f;
                            x1[q] = ok[q] ? L.t(n + 1) : 0.0f;
                        } else {   // Lattice::t of a constant step, from LDS or the arguments
                            float2 c;
                            if constexpr (Lats::kMulti) c = s_lat[s_scene[b]];
                            else c = make_float2(lats.lat.tmin, lats.lat.dt);
                            x0[q] = ok[q] ? __fadd_rn(c.x, __fmul_rn((float)n, c.y)) : 0.0f;
                            x1[q] = ok[q] ? __fadd_rn(c.x, __fmul_rn((float)(n + 1), c.y)) : 0.0f;
                        }
                    }
                    const int64_t at = base + j4;
                    if (vec4 && ok[0] && ok[1] && ok[2] && ok[3]) {
                        *reinterpret_cast<int4 *>(ray_ids + at) = make_int4(id[0], id[1], id[2], id[3]);
                        *reinterpret_cast<float4 *>(t0 + at) = make_float4(x0[0], x0[1], x0[2], x0[3]);
                        *reinterpret_cast<float4 *>(t1 + at) = make_float4(x1[0], x1[1], x1[2], x1[3]);
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (ok[q]) {
                                ray_ids[at + q] = id[q];
                                t0[at + q] = x0[q];
                                t1[at + q] = x1[q];
                            }
                    }
                }
                __syncthreads();
            }
        }
        __syncthreads();
    }
}

// Work items are (256-ray chunk, part) pairs, kExpandParts per chunk, part
// by part: item i is part i / chunks of chunk i % chunks.  Blocks go to the
// XCDs round-robin, so this order gives every XCD an even share of part 0
// (which every chunk with samples has) instead of sending all of it to the
// XCDs whose index is a multiple of kExpandParts.  The grid strides over the
// items, so a launch may use fewer blocks than items (every item ends on a
// barrier or returns before its first one, so its LDS is free for the next).
__host__ __device__ inline int64_t expand_items(int64_t n_rays) {
    return (n_rays + kBlock - 1) / kBlock * kExpandParts;
}

template <bool kScan = false, class Lats>
__device__ __forceinline__ void expand_block(int64_t *__restrict__ offsets, const ChunkScan &cs, int64_t n_rays,
                                             const int32_t *__restrict__ nruns, const RunReader &rd,
                                             const Lats &lats, int64_t capacity, int32_t *__restrict__ ray_ids,
                                             float *__restrict__ t0, float *__restrict__ t1, bool vec4) {
    __shared__ ExpandLds sh;
    __shared__ float2 s_lat[Lats::kMulti ? kBlock : 1];   // (tmin, dt) of every scene
    bool cone;
    if constexpr (Lats::kMulti) {
        bool c = false;
        if ((int)threadIdx.x < lats.n) {
            const Lattice L = lats.get(threadIdx.x);
            s_lat[threadIdx.x] = make_float2(L.tmin, L.dt);
            c = L.cone;
        }
        cone = __syncthreads_or(c) != 0;
    } else {
        cone = lats.lat.cone;
    }
    const int64_t chunks = (n_rays + kBlock - 1) / kBlock;
    if (cone) {
        for (int64_t it = blockIdx.x; it < chunks * kExpandParts; it += gridDim.x)
            expand_chunk<true, kScan>(sh, s_lat, it % chunks * kBlock, (int)(it / chunks), offsets, cs, n_rays, nruns,
                                      rd, lats, capacity, ray_ids, t0, t1, vec4);
    } else {
        for (int64_t it = blockIdx.x; it < chunks * kExpandParts; it += gridDim.x)
            expand_chunk<false, kScan>(sh, s_lat, it % chunks * kBlock, (int)(it / chunks), offsets, cs, n_rays,
                                       nruns, rd, lats, capacity, ray_ids, t0, t1, vec4);
    }
}

// ------------------------------------------------------------------ ray order

// Threads per image-tiled launch: 8x8-pixel tiles of 64 lanes (one wave).
__host__ __device__ inline int64_t tiled_threads(int64_t n, int width) {
    if (width <= 0) return n;
    const int64_t rows = (n + width - 1) / width;
    return ((width + 7) / 8) * ((rows + 7) / 8) * (int64_t)64;
}

// Ray walked by thread t: t itself, or with an image of `width` pixels per
// row, lane l of wave w takes pixel (8*(w % tiles_x) + l % 8, 8*(w / tiles_x)
// + l / 8) of the row-major image; -1 for a lane past the image.
__device__ __forceinline__ int64_t ray_of_thread(int64_t t, int64_t n, int width) {
    if (width <= 0) return t < n ? t : -1;
    const int64_t w = t >> 6;
    const int l = (int)(t & 63);
    const int64_t tiles_x = (width + 7) >> 3;
    const int64_t px = (w % tiles_x) * 8 + (l & 7);
    const int64_t py = (w / tiles_x) * 8 + (l >> 3);
    if (px >= width) return -1;
    const int64_t r = py * width + px;
    return r < n ? r : -1;
}

// ------------------------------------------------------------------ ray loads

__device__ __forceinline__ void load_ray(const float *origins, const float *dirs, int64_t i, float o[3], float d[3]) {
    o[0] = origins[3 * i + 0];
    o[1] = origins[3 * i + 1];
    o[2] = origins[3 * i + 2];
    d[0] = dirs[3 * i + 0];
    d[1] = dirs[3 * i + 1];
    d[2] = dirs[3 * i + 2];
}

}  // namespace ogv
