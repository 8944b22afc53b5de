// Grid builders: the dense bitfield (the paper's occupancy grid, 1 bit per
// voxel) and the VDB tree (Sec. 3: root table -> internal nodes -> 8^3
// leaves, uniform blocks pruned into tiles), both built on the GPU from the
// dense uint8 occupancy, plus decoding back to dense for round-trip checks.
//
// VDB build, all on the device:
//   1. classify: one wave per 8^3 block slot packs the block into its
//      512-bit mask (lane = (x, y) row of 8 z-voxels) and marks it empty,
//      full or mixed;
//   2. root: per root cell, all slots empty -> empty root tile, all full ->
//      full root tile, else an internal node;
//   3. exclusive scans number the nodes and the leaves (mixed blocks under
//      node roots, in root-then-slot order);
//   4. write the root table, node masks (child, value, per-word leaf rank),
//      the nodes' per-slot child tables and leaf masks.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>

#include "internal.hpp"
#include "scan.hpp"

namespace ogv {

thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

static float host_plane(const float *box, int R, int a, int m) {
    float h = (box[3 + a] - box[a]) / (float)R;
    float mh = (float)m * h;
    return box[a] + mh;
}

bool boxes_valid(int L, int R, const float *boxes, std::string *why) {
    for (int l = 0; l < L; ++l) {
        const float *b = boxes + 6 * l;
        for (int a = 0; a < 3; ++a) {
            if (!std::isfinite(b[a]) || !std::isfinite(b[3 + a]) || !(b[a] < b[3 + a])) {
                *why = "level " + std::to_string(l) + ": box must be finite with min < max";
                return false;
            }
            float h = (b[3 + a] - b[a]) / (float)R;
            if (!(h > 0.0f) || !std::isfinite(h)) {
                *why = "level " + std::to_string(l) + ": voxel size underflows";
                return false;
            }
            if (l > 0) {
                const float *f = boxes + 6 * (l - 1);
                if (!(host_plane(b, R, a, 0) <= host_plane(f, R, a, 0)) ||
                    !(host_plane(b, R, a, R) >= host_plane(f, R, a, R))) {
                    *why = "level " + std::to_string(l) + " does not contain level " + std::to_string(l - 1);
                    return false;
                }
            }
        }
    }
    return true;
}

namespace {

// ------------------------------------------------------------------ dense

// one voxel per lane: a wave's 64 consecutive voxels form two words
__global__ void __launch_bounds__(256) dense_pack_kernel(const uint8_t *__restrict__ occ, uint64_t n_vox,
                                                        uint32_t *__restrict__ bits) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t m = __ballot(i < n_vox && occ[i] != 0);
    const int lane = threadIdx.x & 63;
    if ((lane == 0 || lane == 32) && i < n_vox) bits[i >> 5] = lane == 0 ? (uint32_t)m : (uint32_t)(m >> 32);
}

__global__ void dense_unpack_kernel(const uint32_t *__restrict__ bits, uint64_t n_vox, uint8_t *__restrict__ out) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_vox) return;
    out[i] = (bits[i >> 5] >> (i & 31)) & 1u;
}

// A dense or distance grid's allocation: boxes at 0 (<= 192 bytes), plane
// geometry at 512 (<= 384 bytes), a density refresh's two change counters at
// kDenseChanged, the bitfield from 1024.
constexpr size_t kDenseChanged = 960;

// ------------------------------------------------------------------ density cache

// One refresh from a density cache (Sec. 2.1: the grid caches the field's
// predicted densities, and samples are taken in the voxels whose cached
// density exceeds a threshold).  With a new density d the cached value c
// becomes max(decay*c, d) -- one binary32 product, then the larger value
// (taken as d when d > decay*c, else decay*c) -- and is written back; the
// voxel is occupied when the (updated) cached value exceeds the threshold.
struct DensityUpdate {
    float *cache;            // [L][R][R][R], updated in place when density is set
    const float *density;    // nullable: threshold the cache as it stands
    float decay, threshold;
};

__device__ __forceinline__ bool density_bit(const DensityUpdate &u, uint64_t i) {
    float c = u.cache[i];
    if (u.density) {
        const float dc = __fmul_rn(u.decay, c), d = u.density[i];
        c = d > dc ? d : dc;
        u.cache[i] = c;
    }
    return c > u.threshold;
}

// changed[0] += voxels whose occupancy changed (a wave's sum, one atomic)
__device__ __forceinline__ void add_changed(int32_t n, int32_t *changed) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off, 64);
    if ((threadIdx.x & 63) == 0 && n != 0) atomicAdd(changed, n);
}

// dense bitfield from the density cache: one voxel per lane, a wave's 64
// voxels form two consecutive words
__global__ void __launch_bounds__(256) density_pack_kernel(DensityUpdate u, uint64_t n_vox,
                                                          uint32_t *__restrict__ bits, int32_t *__restrict__ changed) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool on = i < n_vox && density_bit(u, i);
    const uint64_t m = __ballot(on);
    const int lane = threadIdx.x & 63;
    int32_t diff = 0;
    if ((lane == 0 || lane == 32) && i < n_vox) {
        const uint32_t word = lane == 0 ? (uint32_t)m : (uint32_t)(m >> 32);
        diff = __popc(word ^ bits[i >> 5]);
        bits[i >> 5] = word;
    }
    add_changed(diff, changed);
}

// uint8 occupancy from the density cache (for the distance passes)
__global__ void __launch_bounds__(256) density_bytes_kernel(DensityUpdate u, uint64_t n_vox,
                                                           const uint32_t *__restrict__ bits, uint8_t *__restrict__ occ,
                                                           int32_t *__restrict__ changed) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t diff = 0;
    if (i < n_vox) {
        const bool on = density_bit(u, i);
        occ[i] = on ? 1 : 0;
        diff = on != (((bits[i >> 5] >> (i & 31)) & 1u) != 0);
    }
    add_changed(diff, changed);
}

__global__ void zero_changed_kernel(int32_t *changed) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        changed[0] = 0;
        changed[1] = 0;
    }
}

// ------------------------------------------------------------------ distances

// Chebyshev (chessboard) distance from every voxel of a level to the nearest
// occupied voxel of that level, capped at kDistCap, by three separable passes:
// along x the distance to the nearest occupied voxel of the row; along y and
// then z, d(v) = min over |e| <= cap of max(|e|, d(v + e along the axis)).
// Capping each pass keeps the result exactly min(cap, distance).  Voxels
// outside the grid count as empty.  One thread per voxel; the search walks
// outwards and stops once |e| reaches the best value found.
template <int kAxis>
__global__ void __launch_bounds__(256) dist_pass_kernel(const uint8_t *__restrict__ in, int L, int R,
                                                       uint8_t *__restrict__ out) {
    const uint64_t n = (uint64_t)L * R * R * R;
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int z = (int)(i % R), y = (int)((i / R) % R), x = (int)((i / ((uint64_t)R * R)) % R);
    const int c = kAxis == 0 ? x : (kAxis == 1 ? y : z);
    const int64_t stride = kAxis == 0 ? (int64_t)R * R : (kAxis == 1 ? R : 1);
    auto val = [&](int e) -> int {   // this pass's input at offset e along the axis (in the grid)
        const uint8_t v = in[(int64_t)i + e * stride];
        return kAxis == 0 ? (v != 0 ? 0 : kDistCap) : (int)v;
    };
    int best = val(0);
    for (int e = 1; e < best && e <= kDistCap; ++e) {
        if (c + e < R) best = min(best, max(e, val(e)));
        if (c - e >= 0) best = min(best, max(e, val(-e)));
    }
    out[i] = (uint8_t)min(best, kDistCap);
}

void enqueue_dist(const uint8_t *occ, int L, int R, uint8_t *dist, uint8_t *tmp, hipStream_t s) {
    const uint64_t n = (uint64_t)L * R * R * R;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    dist_pass_kernel<0><<<blocks, 256, 0, s>>>(occ, L, R, dist);
    dist_pass_kernel<1><<<blocks, 256, 0, s>>>(dist, L, R, tmp);
    dist_pass_kernel<2><<<blocks, 256, 0, s>>>(tmp, L, R, dist);
}

// ------------------------------------------------------------------ vdb

struct BuildDims {
    int L, R, ilog2, S, D, NR;
    int64_t n_root;   // L * NR^3
    int64_t n_slot;   // S^3
    int64_t n_block;  // n_root * n_slot
    int W;            // words per node mask
};

// block slot e -> voxel base of its 8^3 block
__device__ __forceinline__ void block_base(const BuildDims &b, int64_t e, int &lev, int &x0, int &y0, int &z0) {
    int64_t root = e / b.n_slot;
    int slot = (int)(e % b.n_slot);
    lev = (int)(root / ((int64_t)b.NR * b.NR * b.NR));
    int rl = (int)(root % ((int64_t)b.NR * b.NR * b.NR));
    int rx = rl / (b.NR * b.NR), ry = (rl / b.NR) % b.NR, rz = rl % b.NR;
    int sx = slot / (b.S * b.S), sy = (slot / b.S) % b.S, sz = slot % b.S;
    x0 = rx * b.D + sx * 8;
    y0 = ry * b.D + sy * 8;
    z0 = rz * b.D + sz * 8;
}

// Occupancy as bytes of 8 voxels along z, row by row: byte (row, zb) holds
// voxels z = 8zb .. 8zb+7 of row ((l*R + x)*R + y), bit z & 7, for
// Rb = ceil(R/8) bytes per row.  One thread per byte, so consecutive threads
// read consecutive 8-voxel runs (16- or 32-byte loads when the rows allow).
struct OccSource {        // uint8 occupancy, nonzero = occupied
    const uint8_t *occ;
    __device__ __forceinline__ uint8_t byte(uint64_t base, int cnt, bool vec) const {
        uint8_t v[8];
        if (vec && cnt == 8) {
            const uint2 w = *reinterpret_cast<const uint2 *>(occ + base);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v[j] = (uint8_t)(w.x >> (8 * j));
                v[4 + j] = (uint8_t)(w.y >> (8 * j));
            }
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = j < cnt ? occ[base + j] : 0;
        }
        uint8_t b = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) b |= (uint8_t)((v[j] != 0) << j);
        return b;
    }
};

struct DensitySource {    // density cache, updated and thresholded (DensityUpdate)
    DensityUpdate u;
    __device__ __forceinline__ uint8_t byte(uint64_t base, int cnt, bool vec) const {
        float c[8], d[8];
        if (vec && cnt == 8) {
            const float4 c0 = *reinterpret_cast<const float4 *>(u.cache + base);
            const float4 c1 = *reinterpret_cast<const float4 *>(u.cache + base + 4);
            c[0] = c0.x; c[1] = c0.y; c[2] = c0.z; c[3] = c0.w;
            c[4] = c1.x; c[5] = c1.y; c[6] = c1.z; c[7] = c1.w;
            if (u.density) {
                const float4 d0 = *reinterpret_cast<const float4 *>(u.density + base);
                const float4 d1 = *reinterpret_cast<const float4 *>(u.density + base + 4);
                d[0] = d0.x; d[1] = d0.y; d[2] = d0.z; d[3] = d0.w;
                d[4] = d1.x; d[5] = d1.y; d[6] = d1.z; d[7] = d1.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                c[j] = j < cnt ? u.cache[base + j] : 0.0f;
                d[j] = u.density && j < cnt ? u.density[base + j] : 0.0f;
            }
        }
        if (u.density) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float dc = __fmul_rn(u.decay, c[j]);
                c[j] = d[j] > dc ? d[j] : dc;
            }
            if (vec && cnt == 8) {
                *reinterpret_cast<float4 *>(u.cache + base) = make_float4(c[0], c[1], c[2], c[3]);
                *reinterpret_cast<float4 *>(u.cache + base + 4) = make_float4(c[4], c[5], c[6], c[7]);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    if (j < cnt) u.cache[base + j] = c[j];
            }
        }
        uint8_t b = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) b |= (uint8_t)((j < cnt && c[j] > u.threshold) << j);
        return b;
    }
};

template <class Src>
__global__ void __launch_bounds__(256) row_bits_kernel(Src src, int L, int R, bool vec, uint8_t *__restrict__ rows) {
    const int Rb = (R + 7) >> 3;
    const uint64_t n = (uint64_t)L * R * R * Rb;
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint64_t row = t / Rb;
    const int z0 = (int)(t % Rb) * 8;
    rows[t] = src.byte(row * R + z0, min(8, R - z0), vec);
}

// One wave per 8^3 block slot (4 per workgroup): the block's leaf words from
// the row bytes (word x, bit y*8 + z), its kind (0 empty, 1 full, 2 mixed).
// With changed (a refresh), the words are compared with the previous ones
// (masks): the block is marked dirty when they differ, changed[0] gains the
// voxels that flipped, and changed[1] is set when the block's kind changed,
// which is what forces the tree to be renumbered.
__global__ void __launch_bounds__(256) block_classify_kernel(BuildDims b, const uint8_t *__restrict__ rowbits,
                                                            int32_t *__restrict__ kind, int32_t *__restrict__ mixed,
                                                            uint64_t *__restrict__ masks, int32_t *__restrict__ dirty,
                                                            int32_t *__restrict__ changed) {
    __shared__ uint8_t rows[4][64];
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int64_t e = (int64_t)blockIdx.x * 4 + wid;
    bool live = e < b.n_block;
    uint8_t byte = 0;
    if (live) {
        int lev, x0, y0, z0;
        block_base(b, e, lev, x0, y0, z0);
        const int x = x0 + (lane >> 3), y = y0 + (lane & 7);
        const int Rb = (b.R + 7) >> 3;
        if (x < b.R && y < b.R && z0 < b.R) byte = rowbits[(((uint64_t)lev * b.R + x) * b.R + y) * Rb + (z0 >> 3)];
    }
    rows[wid][lane] = byte;
    __syncthreads();
    if (!live) return;
    // word x of the leaf = bytes (x, y=0..7): bit y*8 + z
    uint64_t word = 0;
    int32_t diff = 0;
    if (lane < 8) {
        for (int y = 0; y < 8; ++y) word |= (uint64_t)rows[wid][lane * 8 + y] << (8 * y);
        if (changed) diff = __popcll(word ^ masks[e * 8 + lane]);
        masks[e * 8 + lane] = word;
    }
    const bool any_on = __ballot(lane < 8 && word != 0) != 0;
    const bool all_on = __ballot(lane < 8 && word == ~0ull) == 0xffull;
    const int k = all_on ? 1 : (any_on ? 2 : 0);
    if (changed) {
        const bool dirt = __ballot(diff != 0) != 0;
        add_changed(diff, changed);
        if (lane == 0) {
            if (k != kind[e]) changed[1] = 1;
            dirty[e] = dirt;
        }
    }
    if (lane == 0) {
        kind[e] = k;
        mixed[e] = k == 2;
    }
}

// gate (nullable) on the kernels below: nothing is done when *gate is 0 (a
// refresh that changed no block's kind keeps the tree's numbering).
__global__ void __launch_bounds__(256) root_kernel(BuildDims b, const int32_t *__restrict__ kind,
                                                  int32_t *__restrict__ root_kind, int32_t *__restrict__ is_node,
                                                  const int32_t *gate) {
    __shared__ int n_empty, n_full;
    if (gate && *gate == 0) return;
    if (threadIdx.x == 0) {
        n_empty = 0;
        n_full = 0;
    }
    __syncthreads();
    int64_t r = blockIdx.x;
    int ce = 0, cf = 0;
    for (int64_t s = threadIdx.x; s < b.n_slot; s += blockDim.x) {
        int k = kind[r * b.n_slot + s];
        ce += k == 0;
        cf += k == 1;
    }
    atomicAdd(&n_empty, ce);
    atomicAdd(&n_full, cf);
    __syncthreads();
    if (threadIdx.x == 0) {
        int rk = n_empty == b.n_slot ? 0 : (n_full == b.n_slot ? 1 : 2);
        root_kind[r] = rk;
        is_node[r] = rk == 2;
    }
}

__global__ void root_write_kernel(BuildDims b, const int32_t *__restrict__ root_kind,
                                  const int64_t *__restrict__ node_idx, int32_t *__restrict__ root,
                                  VdbCounts *counts, const int32_t *gate) {
    if (gate && *gate == 0) return;
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= b.n_root) return;
    int rk = root_kind[r];
    root[r] = rk == 2 ? (int32_t)node_idx[r] : (rk == 1 ? -2 : -1);
    if (rk == 0) atomicAdd((unsigned long long *)&counts->n_root_empty, 1ull);
    if (rk == 1) atomicAdd((unsigned long long *)&counts->n_root_full, 1ull);
    if (r == 0) {
        counts->n_nodes = node_idx[b.n_root];
    }
}

// one wave per (root cell, mask word); only node roots write
__global__ void __launch_bounds__(256) node_write_kernel(BuildDims b, const int32_t *__restrict__ root_kind,
                                                        const int64_t *__restrict__ node_idx,
                                                        const int32_t *__restrict__ kind,
                                                        const int64_t *__restrict__ leaf_idx,
                                                        uint64_t *__restrict__ child, uint64_t *__restrict__ value,
                                                        uint32_t *__restrict__ rank, int32_t *__restrict__ slot,
                                                        VdbCounts *counts, const int32_t *gate) {
    if (gate && *gate == 0) return;
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int64_t job = (int64_t)blockIdx.x * 4 + wid;
    if (job >= b.n_root * b.W) return;
    int64_t r = job / b.W;
    int w = (int)(job % b.W);
    if (root_kind[r] != 2) return;
    int64_t node = node_idx[r];
    int64_t s = (int64_t)w * 64 + lane;
    int k = s < b.n_slot ? kind[r * b.n_slot + s] : -1;
    if (s < b.n_slot)
        slot[node * b.n_slot + s] = k == 2 ? (int32_t)leaf_idx[r * b.n_slot + s] : (k == 1 ? -2 : -1);
    uint64_t cm = __ballot(k == 2);
    uint64_t vm = __ballot(k == 1);
    uint64_t em = __ballot(k == 0);
    if (lane == 0) {
        child[node * b.W + w] = cm;
        value[node * b.W + w] = vm;
        rank[node * b.W + w] = (uint32_t)leaf_idx[r * b.n_slot + (int64_t)w * 64];
        atomicAdd((unsigned long long *)&counts->n_tiles_full, (unsigned long long)__popcll(vm));
        atomicAdd((unsigned long long *)&counts->n_tiles_empty, (unsigned long long)__popcll(em));
    }
}

// Uniform 4^3 sub-blocks of a leaf given its eight words (word x, bit
// y*8 + z): bit ((x>>2)*2 + (y>>2))*2 + (z>>2) is set when the 64 voxels of
// that sub-block are all occupied or all empty.
__device__ uint64_t leaf_uniform_quarters(const uint64_t *w) {
    uint64_t u4 = 0;
    for (int xq = 0; xq < 2; ++xq) {
        uint64_t a = ~0ull, o = 0;
        for (int x = 4 * xq; x < 4 * xq + 4; ++x) {
            a &= w[x];
            o |= w[x];
        }
        for (int yq = 0; yq < 2; ++yq)
            for (int zq = 0; zq < 2; ++zq) {
                const uint64_t m = 0x0F0F0F0Full << (32 * yq + 4 * zq);   // y in 4yq..4yq+3, z in 4zq..4zq+3
                if ((a & m) == m || (o & m) == 0) u4 |= 1ull << ((xq * 2 + yq) * 2 + zq);
            }
    }
    return u4;
}

// gate (nullable): when *gate is 0 only the leaves of dirty blocks (dirty[e]
// != 0) are rewritten -- the numbering is unchanged -- else every leaf.
__global__ void leaf_write_kernel(BuildDims b, const int32_t *__restrict__ mixed, const int64_t *__restrict__ leaf_idx,
                                  const uint64_t *__restrict__ masks, uint64_t *__restrict__ leaves,
                                  uint64_t *__restrict__ sub, VdbCounts *counts, const int32_t *gate,
                                  const int32_t *__restrict__ dirty) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t e = t >> 3;
    int j = (int)(t & 7);
    if (e >= b.n_block) return;
    const bool all = !gate || *gate != 0;
    if (!all && !dirty[e]) return;
    if (all && e == 0 && j == 0) counts->n_leaves = leaf_idx[b.n_block];
    if (!mixed[e]) return;
    leaves[leaf_idx[e] * 8 + j] = masks[e * 8 + j];
    if (j == 0) sub[leaf_idx[e]] = leaf_uniform_quarters(masks + e * 8);
}

// decode a VDB tree into dense bytes, one thread per voxel
__global__ void vdb_unpack_kernel(GridView g, uint8_t *__restrict__ out) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t R = (uint64_t)g.R;
    if (i >= (uint64_t)g.L * R * R * R) return;
    int z = (int)(i % R), y = (int)((i / R) % R), x = (int)((i / (R * R)) % R), lev = (int)(i / (R * R * R));
    const int sh = 3 + g.ilog2;
    int ri = ((lev * g.NR + (x >> sh)) * g.NR + (y >> sh)) * g.NR + (z >> sh);
    int node = g.root[ri];
    uint8_t v;
    if (node < 0) {
        v = node == -2;
    } else {
        const int m = g.S - 1;
        int s = (((x >> 3) & m) * g.S + ((y >> 3) & m)) * g.S + ((z >> 3) & m);
        int w = node * g.W + (s >> 6);
        uint64_t bit = 1ull << (s & 63);
        if (g.child[w] & bit) {
            uint32_t li = g.rank[w] + (uint32_t)__popcll(g.child[w] & (bit - 1));
            v = (g.leaves[(uint64_t)li * 8 + (x & 7)] >> (((y & 7) << 3) | (z & 7))) & 1ull;
        } else {
            v = (g.value[w] & bit) != 0;
        }
    }
    out[i] = v;
}

// Per-level plane geometry for the samplers, computed once at build time:
// voxel size h = fl((A-B)/R) (correctly rounded) and an approximate 1/h used
// only for index estimates.
__global__ void geom_kernel(const float *__restrict__ boxes, int L, int R, float *__restrict__ geom) {
    int t = threadIdx.x;
    if (t >= 3 * L) return;
    int lev = t / 3, a = t % 3;
    const float *b = boxes + 6 * lev;
    float *G = geom + 12 * lev;
    G[a] = b[a];
    G[3 + a] = __fdiv_rn(__fsub_rn(b[3 + a], b[a]), (float)R);
    G[6 + a] = (float)R / (b[3 + a] - b[a]);
    G[9 + a] = 0.0f;
}

__global__ void zero_counts_kernel(VdbCounts *c, const int32_t *gate) {
    if (gate && *gate == 0) return;
    if (threadIdx.x == 0) *c = VdbCounts{0, 0, 0, 0, 0, 0};
}

ogv_status check_common(int32_t L, int32_t R, const float *boxes, const uint8_t *occ, ogv_grid **out) {
    if (!out) OGV_FAIL(OGV_ERR_INVALID, "out is null");
    *out = nullptr;
    if (L < 1 || L > kMaxLevels) OGV_FAIL(OGV_ERR_INVALID, "n_levels must be in 1..8");
    if (R < 1 || R > OGV_MAX_RES) OGV_FAIL(OGV_ERR_INVALID, "res must be in 1..1024");
    if (!boxes || !occ) OGV_FAIL(OGV_ERR_INVALID, "null boxes or occupancy");
    std::string why;
    if (!boxes_valid(L, R, boxes, &why)) OGV_FAIL(OGV_ERR_INVALID, why);
    return OGV_OK;
}

// Scratch of a VDB build, kept with the grid so that a refresh can run the
// same kernels again without allocating.
struct VdbBuildState {
    BuildDims b;
    void *scratch = nullptr;
    int32_t *kind, *mixed, *root_kind, *is_node;
    uint64_t *masks;
    int64_t *leaf_idx, *node_idx, *tiles;
    uint8_t *rowbits;   // occupancy as row bytes (row_bits_kernel), L*R*R*ceil(R/8)
    int32_t *dirty;     // per block: its bits changed in the last density refresh
    int32_t *changed;   // [2] of the last density refresh when the caller passes none
};

// Classifies every 8^3 block of occ and writes the tree into the grid's
// storage (sized for the worst case at build time): the kernels of a build,
// all asynchronous on s.
// The tree from the block kinds and masks left by a classification: root
// kinds, node and leaf numbering, and the node and leaf records.  gate
// (nullable) as on the kernels: when it reads 0 only dirty leaves are
// rewritten.
hipError_t enqueue_tree(ogv_grid *g, const VdbBuildState &st, const int32_t *gate, hipStream_t s) {
    const BuildDims &b = st.b;
    GridView &v = g->view;
    root_kernel<<<(unsigned)b.n_root, 256, 0, s>>>(b, st.kind, st.root_kind, st.is_node, gate);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_excl_scan(st.is_node, b.n_root, st.node_idx, st.tiles, 0, nullptr, s, gate);
    if (e == hipSuccess) {
        root_write_kernel<<<(unsigned)((b.n_root + 255) / 256), 256, 0, s>>>(b, st.root_kind, st.node_idx,
                                                                            (int32_t *)v.root, g->counts_dev, gate);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = launch_excl_scan(st.mixed, b.n_block, st.leaf_idx, st.tiles, 0, nullptr, s, gate);
    if (e == hipSuccess) {
        node_write_kernel<<<(unsigned)((b.n_root * b.W + 3) / 4), 256, 0, s>>>(
            b, st.root_kind, st.node_idx, st.kind, st.leaf_idx, (uint64_t *)v.child, (uint64_t *)v.value,
            (uint32_t *)v.rank, (int32_t *)v.slot, g->counts_dev, gate);
        leaf_write_kernel<<<(unsigned)((b.n_block * 8 + 255) / 256), 256, 0, s>>>(
            b, st.mixed, st.leaf_idx, st.masks, (uint64_t *)v.leaves, (uint64_t *)v.sub, g->counts_dev, gate,
            st.dirty);
        e = hipGetLastError();
    }
    return e;
}

unsigned row_bits_blocks(const BuildDims &b) {
    return (unsigned)(((uint64_t)b.L * b.R * b.R * ((b.R + 7) / 8) + 255) / 256);
}

hipError_t enqueue_vdb(ogv_grid *g, const VdbBuildState &st, const uint8_t *occ, hipStream_t s) {
    const BuildDims &b = st.b;
    zero_counts_kernel<<<1, 64, 0, s>>>(g->counts_dev, nullptr);
    const bool vec = b.R % 8 == 0 && (uintptr_t)occ % 8 == 0;   // 8-byte loads stay aligned
    row_bits_kernel<<<row_bits_blocks(b), 256, 0, s>>>(OccSource{occ}, b.L, b.R, vec, st.rowbits);
    block_classify_kernel<<<(unsigned)((b.n_block + 3) / 4), 256, 0, s>>>(b, st.rowbits, st.kind, st.mixed, st.masks,
                                                                         st.dirty, nullptr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = enqueue_tree(g, st, nullptr, s);
    return e;
}

// Refresh from the density cache: classification with the threshold fused in,
// then the tree rebuilt -- renumbered when a block's kind changed, else only
// the leaves whose bits changed rewritten (every launch reads changed[1]).
hipError_t enqueue_vdb_density(ogv_grid *g, const VdbBuildState &st, const DensityUpdate &u, int32_t *changed,
                               hipStream_t s) {
    const BuildDims &b = st.b;
    zero_changed_kernel<<<1, 64, 0, s>>>(changed);
    const bool vec = b.R % 4 == 0 && ((uintptr_t)u.cache | (uintptr_t)u.density) % 16 == 0;   // 16-byte accesses aligned
    row_bits_kernel<<<row_bits_blocks(b), 256, 0, s>>>(DensitySource{u}, b.L, b.R, vec, st.rowbits);
    block_classify_kernel<<<(unsigned)((b.n_block + 3) / 4), 256, 0, s>>>(b, st.rowbits, st.kind, st.mixed, st.masks,
                                                                         st.dirty, changed);
    zero_counts_kernel<<<1, 64, 0, s>>>(g->counts_dev, changed + 1);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = enqueue_tree(g, st, changed + 1, s);
    return e;
}

void free_state(ogv_grid *g) {
    if (!g->state) return;
    VdbBuildState *st = (VdbBuildState *)g->state;
    (void)hipFree(st->scratch);
    delete st;
    g->state = nullptr;
}

}  // namespace
}  // namespace ogv

using namespace ogv;

extern "C" const char *ogv_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *ogv_version(void) { return "ogvdb 0.1 (gfx950)"; }

extern "C" ogv_status ogv_dense_build(int32_t L, int32_t R, const float *boxes, const uint8_t *occ, ogv_grid **out,
                                      void *stream) {
    ogv_status st = check_common(L, R, boxes, occ, out);
    if (st != OGV_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    uint64_t n_vox = (uint64_t)L * R * R * R;
    uint64_t n_words = (n_vox + 31) / 32;
    size_t off_boxes = 0, off_geom = 512, off_bits = 1024;
    size_t total = off_bits + n_words * 4;
    ogv_grid *g = new ogv_grid();
    if (hipMalloc(&g->mem, total) != hipSuccess) {
        delete g;
        OGV_FAIL(OGV_ERR_OOM, "device allocation of " + std::to_string(total) + " bytes failed");
    }
    g->mem_bytes = total;
    g->used_bytes = n_words * 4;
    std::memcpy(g->boxes_host, boxes, sizeof(float) * 6 * L);
    g->build_stream = s;
    GridView &v = g->view;
    std::memset(&v, 0, sizeof(v));
    v.kind = 0;
    v.L = L;
    v.R = R;
    v.boxes = (const float *)((char *)g->mem + off_boxes);
    v.geom = (const float *)((char *)g->mem + off_geom);
    v.bits = (const uint32_t *)((char *)g->mem + off_bits);
    hipError_t e = hipMemcpyAsync((void *)v.boxes, g->boxes_host, sizeof(float) * 6 * L, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        geom_kernel<<<1, 64, 0, s>>>(v.boxes, L, R, (float *)v.geom);
        dense_pack_kernel<<<(unsigned)((n_vox + 255) / 256), 256, 0, s>>>(occ, n_vox, (uint32_t *)v.bits);
        e = hipGetLastError();
    }
    // the host copy of the boxes must outlive the async copy
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(g->mem);
        delete g;
        OGV_FAIL(OGV_ERR_HIP, std::string("dense build failed: ") + hipGetErrorString(e));
    }
    g->counts_ready = true;
    *out = g;
    return OGV_OK;
}

extern "C" ogv_status ogv_dist_build(int32_t L, int32_t R, const float *boxes, const uint8_t *occ, ogv_grid **out,
                                     void *stream) {
    ogv_status st = check_common(L, R, boxes, occ, out);
    if (st != OGV_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const uint64_t n_vox = (uint64_t)L * R * R * R, n_words = (n_vox + 31) / 32;
    const size_t off_boxes = 0, off_geom = 512, off_bits = 1024;
    const size_t off_dist = align_up(off_bits + n_words * 4, 256);
    const size_t off_tmp = align_up(off_dist + n_vox, 256);
    const size_t total = off_tmp + n_vox;
    ogv_grid *g = new ogv_grid();
    if (hipMalloc(&g->mem, total) != hipSuccess) {
        delete g;
        OGV_FAIL(OGV_ERR_OOM, "device allocation of " + std::to_string(total) + " bytes failed");
    }
    g->mem_bytes = total;
    g->used_bytes = n_words * 4 + n_vox;
    std::memcpy(g->boxes_host, boxes, sizeof(float) * 6 * L);
    g->build_stream = s;
    GridView &v = g->view;
    std::memset(&v, 0, sizeof(v));
    v.kind = 2;
    v.L = L;
    v.R = R;
    char *m = (char *)g->mem;
    v.boxes = (const float *)(m + off_boxes);
    v.geom = (const float *)(m + off_geom);
    v.bits = (const uint32_t *)(m + off_bits);
    v.dist = (const uint8_t *)(m + off_dist);
    g->state = m + off_tmp;   // the distance passes' scratch, kept for refreshes
    hipError_t e = hipMemcpyAsync((void *)v.boxes, g->boxes_host, sizeof(float) * 6 * L, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        geom_kernel<<<1, 64, 0, s>>>(v.boxes, L, R, (float *)v.geom);
        dense_pack_kernel<<<(unsigned)((n_vox + 255) / 256), 256, 0, s>>>(occ, n_vox, (uint32_t *)v.bits);
        enqueue_dist(occ, L, R, (uint8_t *)v.dist, (uint8_t *)g->state, s);
        e = hipGetLastError();
    }
    // the host copy of the boxes must outlive the async copy
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(g->mem);
        delete g;
        OGV_FAIL(OGV_ERR_HIP, std::string("distance-grid build failed: ") + hipGetErrorString(e));
    }
    g->counts_ready = true;
    *out = g;
    return OGV_OK;
}

extern "C" ogv_status ogv_grid_distances(const ogv_grid *grid, uint8_t *out, void *stream) {
    if (!grid || !out) OGV_FAIL(OGV_ERR_INVALID, "null argument");
    const GridView &v = grid->view;
    if (v.kind != 2) OGV_FAIL(OGV_ERR_INVALID, "only a distance grid holds distances");
    const size_t n = (size_t)v.L * v.R * v.R * v.R;
    OGV_CHECK_HIP(hipMemcpyAsync(out, v.dist, n, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return OGV_OK;
}

extern "C" ogv_status ogv_vdb_build(int32_t L, int32_t R, const float *boxes, const uint8_t *occ, int32_t ilog2,
                                    ogv_grid **out, void *stream) {
    ogv_status st = check_common(L, R, boxes, occ, out);
    if (st != OGV_OK) return st;
    if (ilog2 < 1 || ilog2 > 5) OGV_FAIL(OGV_ERR_INVALID, "internal_log2 must be in 1..5");
    hipStream_t s = (hipStream_t)stream;
    BuildDims b;
    b.L = L;
    b.R = R;
    b.ilog2 = ilog2;
    b.S = 1 << ilog2;
    b.D = 8 * b.S;
    b.NR = (R + b.D - 1) / b.D;
    b.n_root = (int64_t)L * b.NR * b.NR * b.NR;
    b.n_slot = (int64_t)b.S * b.S * b.S;
    b.n_block = b.n_root * b.n_slot;
    b.W = (int)((b.n_slot + 63) / 64);

    // final storage, sized for the worst case (every root a node, every
    // block a leaf); the occupied part is reported by ogv_grid_info_get
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    size_t o_boxes = take(sizeof(float) * 6 * L);
    size_t o_geom = take(sizeof(float) * 12 * L);
    size_t o_counts = take(sizeof(VdbCounts));
    size_t o_root = take(sizeof(int32_t) * b.n_root);
    size_t o_child = take(sizeof(uint64_t) * b.n_root * b.W);
    size_t o_value = take(sizeof(uint64_t) * b.n_root * b.W);
    size_t o_rank = take(sizeof(uint32_t) * b.n_root * b.W);
    size_t o_slot = take(sizeof(int32_t) * b.n_root * b.n_slot);
    size_t o_leaves = take(sizeof(uint64_t) * 8 * b.n_block);
    size_t o_sub = take(sizeof(uint64_t) * b.n_block);
    size_t total = off;
    // build scratch
    off = 0;
    size_t t_kind = take(sizeof(int32_t) * b.n_block);
    size_t t_mixed = take(sizeof(int32_t) * b.n_block);
    size_t t_masks = take(sizeof(uint64_t) * 8 * b.n_block);
    size_t t_leafidx = take(sizeof(int64_t) * (b.n_block + 1));
    size_t t_rootkind = take(sizeof(int32_t) * b.n_root);
    size_t t_isnode = take(sizeof(int32_t) * b.n_root);
    size_t t_nodeidx = take(sizeof(int64_t) * (b.n_root + 1));
    size_t t_tiles = take(sizeof(int64_t) * (scan_tiles(b.n_block) + 1));
    size_t t_dirty = take(sizeof(int32_t) * b.n_block);
    size_t t_rowbits = take((size_t)L * R * R * ((R + 7) / 8));
    size_t t_changed = take(sizeof(int32_t) * 2);
    size_t scratch_total = off;

    ogv_grid *g = new ogv_grid();
    void *scratch = nullptr;
    if (hipMalloc(&g->mem, total) != hipSuccess) {
        delete g;
        OGV_FAIL(OGV_ERR_OOM, "device allocation of " + std::to_string(total) + " bytes failed");
    }
    if (hipMalloc(&scratch, scratch_total) != hipSuccess) {
        (void)hipFree(g->mem);
        delete g;
        OGV_FAIL(OGV_ERR_OOM, "device allocation of " + std::to_string(scratch_total) + " bytes failed");
    }
    VdbBuildState *bs = new VdbBuildState();
    bs->b = b;
    bs->scratch = scratch;
    g->state = bs;
    g->mem_bytes = total;
    std::memcpy(g->boxes_host, boxes, sizeof(float) * 6 * L);
    g->build_stream = s;
    char *m = (char *)g->mem, *t = (char *)scratch;
    GridView &v = g->view;
    std::memset(&v, 0, sizeof(v));
    v.kind = 1;
    v.L = L;
    v.R = R;
    v.ilog2 = ilog2;
    v.S = b.S;
    v.NR = b.NR;
    v.W = b.W;
    v.boxes = (const float *)(m + o_boxes);
    v.geom = (const float *)(m + o_geom);
    v.root = (const int32_t *)(m + o_root);
    v.child = (const uint64_t *)(m + o_child);
    v.value = (const uint64_t *)(m + o_value);
    v.rank = (const uint32_t *)(m + o_rank);
    v.slot = (const int32_t *)(m + o_slot);
    v.leaves = (const uint64_t *)(m + o_leaves);
    v.sub = (const uint64_t *)(m + o_sub);
    g->counts_dev = (VdbCounts *)(m + o_counts);

    bs->kind = (int32_t *)(t + t_kind);
    bs->mixed = (int32_t *)(t + t_mixed);
    bs->masks = (uint64_t *)(t + t_masks);
    bs->leaf_idx = (int64_t *)(t + t_leafidx);
    bs->node_idx = (int64_t *)(t + t_nodeidx);
    bs->root_kind = (int32_t *)(t + t_rootkind);
    bs->is_node = (int32_t *)(t + t_isnode);
    bs->tiles = (int64_t *)(t + t_tiles);
    bs->dirty = (int32_t *)(t + t_dirty);
    bs->rowbits = (uint8_t *)(t + t_rowbits);
    bs->changed = (int32_t *)(t + t_changed);

    hipError_t e = hipMemcpyAsync((void *)v.boxes, g->boxes_host, sizeof(float) * 6 * L, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        geom_kernel<<<1, 64, 0, s>>>(v.boxes, L, R, (float *)v.geom);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = enqueue_vdb(g, *bs, occ, s);
    // the host copy of the boxes must outlive the async copy; the build
    // scratch stays with the grid for refreshes
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_state(g);
        (void)hipFree(g->mem);
        delete g;
        OGV_FAIL(OGV_ERR_HIP, std::string("VDB build failed: ") + hipGetErrorString(e));
    }
    *out = g;
    return OGV_OK;
}

extern "C" ogv_status ogv_grid_info_get(const ogv_grid *grid, ogv_grid_info *info) {
    if (!grid || !info) OGV_FAIL(OGV_ERR_INVALID, "null argument");
    ogv_grid *g = const_cast<ogv_grid *>(grid);
    const GridView &v = g->view;
    std::memset(info, 0, sizeof(*info));
    info->kind = v.kind;
    info->n_levels = v.L;
    info->res = v.R;
    info->internal_log2 = v.ilog2;
    if (v.kind != 1) {
        info->bytes = (int64_t)g->used_bytes;
        return OGV_OK;
    }
    if (!g->counts_ready) {
        OGV_CHECK_HIP(hipStreamSynchronize(g->build_stream));
        OGV_CHECK_HIP(hipMemcpy(&g->counts_host, g->counts_dev, sizeof(VdbCounts), hipMemcpyDeviceToHost));
        g->counts_ready = true;
        const int64_t n_root = (int64_t)v.L * v.NR * v.NR * v.NR;
        g->used_bytes = (size_t)(n_root * 4 + g->counts_host.n_nodes * (int64_t)v.W * (8 + 8 + 4) +
                                 g->counts_host.n_nodes * (int64_t)v.S * v.S * v.S * 4 + g->counts_host.n_leaves * (64 + 8));
    }
    const VdbCounts &c = g->counts_host;
    info->bytes = (int64_t)g->used_bytes;
    info->n_nodes = c.n_nodes;
    info->n_leaves = c.n_leaves;
    info->n_tiles_full = c.n_tiles_full;
    info->n_tiles_empty = c.n_tiles_empty;
    info->n_root_tiles_full = c.n_root_full;
    info->n_root_tiles_empty = c.n_root_empty;
    return OGV_OK;
}

extern "C" ogv_status ogv_grid_to_dense(const ogv_grid *grid, uint8_t *out, void *stream) {
    if (!grid || !out) OGV_FAIL(OGV_ERR_INVALID, "null argument");
    const GridView &v = grid->view;
    uint64_t n_vox = (uint64_t)v.L * v.R * v.R * v.R;
    hipStream_t s = (hipStream_t)stream;
    unsigned blocks = (unsigned)((n_vox + 255) / 256);
    if (v.kind != 1) dense_unpack_kernel<<<blocks, 256, 0, s>>>(v.bits, n_vox, out);
    else vdb_unpack_kernel<<<blocks, 256, 0, s>>>(v, out);
    OGV_CHECK_LAUNCH();
    return OGV_OK;
}

extern "C" void ogv_grid_destroy(ogv_grid *grid) {
    if (!grid) return;
    if (grid->view.kind == 1) free_state(grid);   // a kind-2 grid's state points into its own allocation
    (void)hipFree(grid->mem);
    delete grid;
}

extern "C" ogv_status ogv_grid_refresh(ogv_grid *grid, const uint8_t *occ, void *stream) {
    if (!grid || !occ) OGV_FAIL(OGV_ERR_INVALID, "null argument");
    hipStream_t s = (hipStream_t)stream;
    GridView &v = grid->view;
    if (v.kind == 0 || v.kind == 2) {
        const uint64_t n_vox = (uint64_t)v.L * v.R * v.R * v.R;
        dense_pack_kernel<<<(unsigned)((n_vox + 255) / 256), 256, 0, s>>>(occ, n_vox, (uint32_t *)v.bits);
        if (v.kind == 2) enqueue_dist(occ, v.L, v.R, (uint8_t *)v.dist, (uint8_t *)grid->state, s);
        OGV_CHECK_LAUNCH();
        grid->build_stream = s;
        return OGV_OK;
    }
    if (!grid->state) OGV_FAIL(OGV_ERR_INVALID, "grid has no build state");
    const hipError_t e = enqueue_vdb(grid, *(const VdbBuildState *)grid->state, occ, s);
    if (e != hipSuccess) OGV_FAIL(OGV_ERR_HIP, std::string("VDB refresh failed: ") + hipGetErrorString(e));
    grid->counts_ready = false;   // ogv_grid_info_get waits for this stream and re-reads them
    grid->build_stream = s;
    return OGV_OK;
}

extern "C" ogv_status ogv_grid_refresh_density(ogv_grid *grid, float *cache, const float *density, float decay,
                                               float threshold, int32_t *changed, void *stream) {
    if (!grid || !cache) OGV_FAIL(OGV_ERR_INVALID, "null argument");
    if (density && !(decay >= 0.0f && decay <= 1.0f)) OGV_FAIL(OGV_ERR_INVALID, "decay must be in [0, 1]");
    if (std::isnan(threshold)) OGV_FAIL(OGV_ERR_INVALID, "threshold is NaN");
    hipStream_t s = (hipStream_t)stream;
    GridView &v = grid->view;
    const uint64_t n_vox = (uint64_t)v.L * v.R * v.R * v.R;
    const DensityUpdate u{cache, density, decay, threshold};
    const unsigned blocks = (unsigned)((n_vox + 255) / 256);
    if (v.kind == 0 || v.kind == 2) {
        int32_t *ch = changed ? changed : (int32_t *)((char *)grid->mem + kDenseChanged);
        zero_changed_kernel<<<1, 64, 0, s>>>(ch);
        if (v.kind == 0) {
            density_pack_kernel<<<blocks, 256, 0, s>>>(u, n_vox, (uint32_t *)v.bits, ch);
        } else {
            // thresholded bytes into the pass buffer, then the bitfield and the distances from them
            uint8_t *tmp = (uint8_t *)grid->state;
            density_bytes_kernel<<<blocks, 256, 0, s>>>(u, n_vox, v.bits, tmp, ch);
            dense_pack_kernel<<<(unsigned)((n_vox + 255) / 256), 256, 0, s>>>(tmp, n_vox, (uint32_t *)v.bits);
            enqueue_dist(tmp, v.L, v.R, (uint8_t *)v.dist, tmp, s);
        }
        OGV_CHECK_LAUNCH();
        grid->build_stream = s;
        return OGV_OK;
    }
    if (!grid->state) OGV_FAIL(OGV_ERR_INVALID, "grid has no build state");
    const VdbBuildState &st = *(const VdbBuildState *)grid->state;
    const hipError_t e = enqueue_vdb_density(grid, st, u, changed ? changed : st.changed, s);
    if (e != hipSuccess) OGV_FAIL(OGV_ERR_HIP, std::string("VDB density refresh failed: ") + hipGetErrorString(e));
    grid->counts_ready = false;
    grid->build_stream = s;
    return OGV_OK;
}
