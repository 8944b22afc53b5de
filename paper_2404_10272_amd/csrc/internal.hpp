// Internal declarations of the ogvdb library: error plumbing, the grid
// handle and the device-side view of a grid that kernels receive.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>

#include "../../include/ogvdb.h"

namespace ogv {

// ---------------------------------------------------------------- errors

void set_error(const std::string &msg);

#define OGV_FAIL(code, msg)                                                 \
    do {                                                                     \
        ::ogv::set_error(std::string(__func__) + ": " + (msg));            \
        return (code);                                                       \
    } while (0)

#define OGV_CHECK_HIP(expr)                                                                       \
    do {                                                                                          \
        hipError_t _e = (expr);                                                                   \
        if (_e != hipSuccess)                                                                     \
            OGV_FAIL(OGV_ERR_HIP, std::string(#expr) + " failed: " + hipGetErrorString(_e));     \
    } while (0)

#define OGV_CHECK_LAUNCH() OGV_CHECK_HIP(hipGetLastError())

// ---------------------------------------------------------------- grid

constexpr int kMaxLevels = OGV_MAX_LEVELS;

// VDB tree layout (device memory, one allocation):
//   root   int32  [L][NR^3]   >= 0 internal node index, -1 empty tile, -2 full tile
//   child  uint64 [nodes][W]  bit s: slot s holds a leaf
//   value  uint64 [nodes][W]  bit s: slot s is a full tile (when not a leaf)
//   rank   uint32 [nodes][W]  leaf index of the first leaf in word w
//   slot   int32  [nodes][S^3] per slot: leaf index (>= 0), -1 empty tile,
//                              -2 full tile (the node's child table, which
//                              the walk reads; the masks serve decoding)
//   leaves uint64 [leaves][8] word x (voxel x&7), bit (y&7)*8 + (z&7)
//   sub    uint64 [leaves]    uniform 4^3 sub-blocks of each leaf: bit
//                              ((x>>2)*2 + (y>>2))*2 + (z>>2) (x, y, z in
//                              0..7) set when all 64 voxels of that
//                              sub-block share one value
// with S = 2^ilog2 slots per axis per node, slot s = (sx*S + sy)*S + sz,
// W = ceil(S^3 / 64) words per mask.  A root cell covers D = 8*S voxels.
struct GridView {
    int32_t kind;      // 0 dense bitfield, 1 VDB tree, 2 dense bitfield + chessboard distances
    int32_t L, R;
    int32_t ilog2, S, NR, W;
    const float *boxes;        // [L][6] device copy of the boxes
    const float *geom;         // [L][12]: B[3], h[3] = fl((A-B)/R), approximate 1/h [3], unused[3]
    const uint32_t *bits;      // dense: bit ((l*R+x)*R+y)*R+z
    const int32_t *root;
    const uint64_t *child;
    const uint64_t *value;
    const uint32_t *rank;
    const int32_t *slot;
    const uint64_t *leaves;
    const uint64_t *sub;
    const uint8_t *dist;       // kind 2: per voxel min(kDistCap, Chebyshev distance to the nearest occupied voxel)
};

// Cap of the chessboard distances a kind-2 grid stores: an empty voxel at
// distance d >= 2 (d <= kDistCap) has every voxel within d - 1 of it empty.
constexpr int kDistCap = 16;

struct VdbCounts {             // device-side counters filled by the build
    int64_t n_nodes, n_leaves;
    int64_t n_tiles_full, n_tiles_empty;
    int64_t n_root_full, n_root_empty;
};

}  // namespace ogv

struct ogv_grid {
    ogv::GridView view;
    void *mem = nullptr;            // single device allocation
    size_t mem_bytes = 0;
    size_t used_bytes = 0;          // bytes the representation occupies
    ogv::VdbCounts *counts_dev = nullptr;
    ogv::VdbCounts counts_host{};
    bool counts_ready = false;
    hipStream_t build_stream = nullptr;   // stream of the last build or refresh
    float boxes_host[ogv::kMaxLevels][6];
    void *state = nullptr;                // VDB: build scratch and layout, kept for refreshes
};

namespace ogv {

// Host-side validation of level boxes: finite, min < max, and every level's
// outer planes nested inside the next coarser level's (binary32 planes).
bool boxes_valid(int L, int R, const float *boxes, std::string *why);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Length of the growing-step lattice table for [near, far] (0 for a constant
// step, -1 if longer than the library handles).
int32_t cone_table_capacity(float near_t, float far_t, const ogv_step *step);

// Host-side checks of one sampling call's arguments (status + message).
ogv_status validate_sampling(const ogv_grid *grid, int32_t variant, const float *o, const float *d, int64_t n_rays,
                             float near_t, float far_t, const ogv_step *step, const char *fn);

}  // namespace ogv
