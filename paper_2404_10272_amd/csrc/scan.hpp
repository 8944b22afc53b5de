// Device-wide exclusive scan of int32 values into int64 offsets (reduce per
// tile, then apply with each tile's base; a separate scan of the tile sums
// only for very long inputs), used for per-ray sample offsets and for leaf
// and node numbering when a VDB tree is built.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ogv {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ int64_t wave_incl_scan(int64_t x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int64_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// Exclusive scan within a block of kScanThreads; returns the block total.
__device__ __forceinline__ int64_t block_excl_scan(int64_t x, int64_t *lds, int64_t &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t incl = wave_incl_scan(x);
    if (lane == 63) lds[wid] = incl;
    __syncthreads();
    int64_t wbase = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) {
        int64_t s = lds[w];
        if (w < wid) wbase += s;
        total += s;
    }
    __syncthreads();
    return wbase + incl - x;
}

// gate (nullable, every kernel here): the kernel does nothing when *gate is 0.
__global__ void __launch_bounds__(kScanThreads) scan_reduce_kernel(const int32_t *__restrict__ counts, int64_t n,
                                                                  int64_t *__restrict__ tile_sums,
                                                                  const int32_t *gate = nullptr) {
    __shared__ int64_t lds[kScanThreads / 64];
    if (gate && *gate == 0) return;
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + (int64_t)j * kScanThreads + threadIdx.x;
        if (i < n) s += counts[i];
    }
    int64_t total;
    block_excl_scan(s, lds, total);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// One block: exclusive scan of the tile sums in place; writes the grand
// total to *total and, when overflow is given, whether it exceeds capacity.
__global__ void __launch_bounds__(kScanThreads) scan_tiles_kernel(int64_t *__restrict__ tile_sums, int64_t n_tiles,
                                                                 int64_t *__restrict__ total_out, int64_t capacity,
                                                                 int32_t *__restrict__ overflow,
                                                                 const int32_t *gate = nullptr) {
    __shared__ int64_t lds[kScanThreads / 64];
    if (gate && *gate == 0) return;
    int64_t carry = 0;
    for (int64_t base = 0; base < n_tiles; base += kScanThreads) {
        int64_t i = base + threadIdx.x;
        int64_t x = i < n_tiles ? tile_sums[i] : 0;
        int64_t total;
        int64_t ex = block_excl_scan(x, lds, total);
        if (i < n_tiles) tile_sums[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) {
        *total_out = carry;
        if (overflow) *overflow = carry > capacity ? 1 : 0;
    }
}

__global__ void __launch_bounds__(kScanThreads) scan_apply_kernel(const int32_t *__restrict__ counts, int64_t n,
                                                                 const int64_t *__restrict__ tile_base,
                                                                 int64_t *__restrict__ offsets,
                                                                 const int32_t *gate = nullptr) {
    __shared__ int64_t lds[kScanThreads / 64];
    if (gate && *gate == 0) return;
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t c[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + j;
        c[j] = i < n ? counts[i] : 0;
        s += c[j];
    }
    int64_t total;
    int64_t ex = block_excl_scan(s, lds, total) + tile_base[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + j;
        if (i < n) offsets[i] = ex;
        ex += c[j];
    }
}

// Apply with the tile's base summed in place from the raw tile sums (no
// separate scan of the tile sums); the last tile also writes the total and
// the overflow flag.  For up to kScanDirectTiles tiles.
constexpr int64_t kScanDirectTiles = 4096;

__global__ void __launch_bounds__(kScanThreads) scan_apply_direct_kernel(const int32_t *__restrict__ counts, int64_t n,
                                                                        const int64_t *__restrict__ tile_sums,
                                                                        int64_t *__restrict__ offsets,
                                                                        int64_t capacity,
                                                                        int32_t *__restrict__ overflow,
                                                                        const int32_t *gate = nullptr) {
    __shared__ int64_t lds[kScanThreads / 64];
    if (gate && *gate == 0) return;
    int64_t before = 0;
    for (int64_t k = threadIdx.x; k < (int64_t)blockIdx.x; k += kScanThreads) before += tile_sums[k];
    int64_t tile_base;
    block_excl_scan(before, lds, tile_base);   // block total = sum of the earlier tiles
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t c[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + j;
        c[j] = i < n ? counts[i] : 0;
        s += c[j];
    }
    int64_t total;
    int64_t ex = block_excl_scan(s, lds, total) + tile_base;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + j;
        if (i < n) offsets[i] = ex;
        ex += c[j];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        offsets[n] = tile_base + total;
        if (overflow) *overflow = tile_base + total > capacity ? 1 : 0;
    }
}

// out[0..n-1] = exclusive scan of in, out[n] = total; tiles needs
// scan_tiles(n) + 1 int64 of scratch.  overflow (nullable) <- total > capacity.
inline int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

// gate (nullable): device flag; when it reads 0 the launched kernels do
// nothing (out is left as it was).
inline hipError_t launch_excl_scan(const int32_t *in, int64_t n, int64_t *out, int64_t *tiles, int64_t capacity,
                                   int32_t *overflow, hipStream_t s, const int32_t *gate = nullptr) {
    int64_t nt = scan_tiles(n);
    if (nt > 0 && nt <= kScanDirectTiles) {
        scan_reduce_kernel<<<(unsigned)nt, kScanThreads, 0, s>>>(in, n, tiles, gate);
        scan_apply_direct_kernel<<<(unsigned)nt, kScanThreads, 0, s>>>(in, n, tiles, out, capacity, overflow, gate);
        return hipGetLastError();
    }
    if (nt > 0) scan_reduce_kernel<<<(unsigned)nt, kScanThreads, 0, s>>>(in, n, tiles, gate);
    scan_tiles_kernel<<<1, kScanThreads, 0, s>>>(tiles, nt, out + n, capacity, overflow, gate);
    if (nt > 0) scan_apply_kernel<<<(unsigned)nt, kScanThreads, 0, s>>>(in, n, tiles, out, gate);
    return hipGetLastError();
}

// As launch_excl_scan, for a producer that has already left each tile's sum
// of `in` in tiles[0 .. scan_tiles(n)-1]: up to kScanDirectTiles tiles one
// apply launch reads them (and leaves them intact, so the scan can be
// repeated); longer inputs take the full three launches.
inline hipError_t launch_excl_scan_from_sums(const int32_t *in, int64_t n, int64_t *out, int64_t *tiles,
                                             int64_t capacity, int32_t *overflow, hipStream_t s) {
    int64_t nt = scan_tiles(n);
    if (nt > 0 && nt <= kScanDirectTiles) {
        scan_apply_direct_kernel<<<(unsigned)nt, kScanThreads, 0, s>>>(in, n, tiles, out, capacity, overflow);
        return hipGetLastError();
    }
    return launch_excl_scan(in, n, out, tiles, capacity, overflow, s);
}

}  // namespace
}  // namespace ogv
