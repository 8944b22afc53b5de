// The counting pass's Alg. 2 (skip) walks over a VDB tree: hierarchical,
// voxel and sub-leaf steps, single- and multi-level, tree in LDS or not.
// They live in a source of their own so the build can compile them at -O2
// while the rest of the sampler is built at -O1; sample.hip launches them.
#pragma clang fp contract(off)

#include "count.hpp"

namespace ogv {

#define OGV_COUNT_SKIP(V, L, L1)                                                                        \
    template __global__ void count_kernel<V, true, L, L1>(GridView, const float *, const float *, int64_t, \
                                                          Lattice, int32_t *, int32_t *, RunPool, int,  \
                                                          int64_t *, int64_t *);
OGV_COUNT_SKIP_ALL
#undef OGV_COUNT_SKIP

}  // namespace ogv
