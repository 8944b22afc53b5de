// Volume-rendering composite over packed samples and its backward pass.
//
// The paper only says a ray's sample colours and densities are accumulated
// into the pixel colour (Sec. 1); the emission-absorption quadrature is
// used: per ray, tau_i = sigma_i (t1_i - t0_i), alpha_i = 1 - exp(-tau_i),
// T_i = exp(-sum_{j<i} tau_j), w_i = T_i alpha_i, C = sum w_i c_i,
// A = sum w_i.  The backward pass gives
//   dL/dc_i     = w_i g_C
//   dL/dsigma_i = dt_i (g_C . (T_{i+1} c_i - sum_{k>i} w_k c_k) + g_A T_n),
// with the suffix sum accumulated in a reverse pass (not as C minus a
// prefix) and T rebuilt from the exponent sum, whose absolute error stays
// at the level of one rounding of the ray's total optical depth.  One 16-lane
// row (a DPP row) handles one ray, 16 consecutive samples per chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "internal.hpp"

namespace ogv {
namespace {

constexpr int kBlock = 256;
constexpr int kRow = 16;                    // lanes per ray: one DPP row
constexpr int kRaysPerBlock = kBlock / kRow;

// Row-local data movement on the VALU (DPP): lane j of a 16-lane row reads
// lane j - n (row_shr) or j + n (row_shl) of the same row; lanes whose
// source falls outside the row read 0.
template <int kCtrl>
__device__ __forceinline__ float dpp(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kCtrl, 0xF, 0xF, true));
}
// inclusive prefix sum over the row (lane 15 ends with the row total)
__device__ __forceinline__ float row_prefix(float x) {
    x += dpp<0x111>(x);
    x += dpp<0x112>(x);
    x += dpp<0x114>(x);
    x += dpp<0x118>(x);
    return x;
}
// inclusive suffix sum over the row (lane 0 ends with the row total)
__device__ __forceinline__ float row_suffix(float x) {
    x += dpp<0x101>(x);
    x += dpp<0x102>(x);
    x += dpp<0x104>(x);
    x += dpp<0x108>(x);
    return x;
}
// value of lane `src` (0..15) of this lane's row
__device__ __forceinline__ float row_lane(float x, int src) {
    return __shfl(x, ((int)threadIdx.x & 63 & ~(kRow - 1)) | src, 64);
}

// Samples of one row are loaded kGroup chunks of 16 at a time, all loads of a
// group issued before any of its arithmetic, so that one memory latency
// covers kGroup * 16 samples instead of 16.  The backward keeps the ray's last
// group in registers between its two passes, so a larger group there means
// more rays read their inputs once.
constexpr int kGroup = 4;
constexpr int kSpan = kGroup * kRow;
constexpr int kGroupBwd = 8;
constexpr int kSpanBwd = kGroupBwd * kRow;

// One 16-lane row per ray, 16 consecutive samples per chunk (coalesced
// loads); the optical depth before each sample is a row prefix sum plus the
// carry of the earlier chunks.  Rows past the last ray do nothing, but stay
// in their wave so that every DPP source lane is active.
__global__ void __launch_bounds__(kBlock) composite_fwd_kernel(const int64_t *__restrict__ offsets, int64_t n_rays,
                                                              const float *__restrict__ t0,
                                                              const float *__restrict__ t1,
                                                              const float *__restrict__ sigma,
                                                              const float *__restrict__ rgb, float *__restrict__ out_rgb,
                                                              float *__restrict__ out_opacity) {
    const int l = threadIdx.x & (kRow - 1);
    const int64_t r = (int64_t)blockIdx.x * kRaysPerBlock + (threadIdx.x / kRow);
    const bool live = r < n_rays;
    const int64_t a = live ? offsets[r] : 0, b = live ? offsets[r + 1] : 0;
    float cr = 0.f, cg = 0.f, cb = 0.f, acc = 0.f, carry = 0.f;
    for (int64_t g0 = a; g0 < b; g0 += kSpan) {   // row-uniform
        float tau[kGroup], xr[kGroup], xg[kGroup], xb[kGroup];
#pragma unroll
        for (int c = 0; c < kGroup; ++c) {
            const int64_t i = g0 + c * kRow + l;
            tau[c] = xr[c] = xg[c] = xb[c] = 0.f;
            if (i < b) {
                tau[c] = sigma[i] * (t1[i] - t0[i]);
                xr[c] = rgb[3 * i + 0];
                xg[c] = rgb[3 * i + 1];
                xb[c] = rgb[3 * i + 2];
            }
        }
#pragma unroll
        for (int c = 0; c < kGroup; ++c) {
            if (g0 + c * kRow >= b) break;   // row-uniform
            const float incl = row_prefix(tau[c]);
            const float T = expf(-(carry + incl - tau[c]));
            const float w = g0 + c * kRow + l < b ? T * (-expm1f(-tau[c])) : 0.f;
            cr += w * xr[c];
            cg += w * xg[c];
            cb += w * xb[c];
            acc += w;
            carry += row_lane(incl, kRow - 1);
        }
    }
    cr = row_prefix(cr);
    cg = row_prefix(cg);
    cb = row_prefix(cb);
    acc = row_prefix(acc);
    if (live && l == kRow - 1) {
        out_rgb[3 * r + 0] = cr;
        out_rgb[3 * r + 1] = cg;
        out_rgb[3 * r + 2] = cb;
        if (out_opacity) out_opacity[r] = acc;
    }
}

// One 16-lane row per ray.  Pass 1: the ray's total optical depth; its last
// group of chunks stays in registers.  Pass 2, groups and chunks from the
// back: T_i and T_{i+1} from the total minus the depth at and after i (row
// suffix sum plus the carry of later chunks), and sum_{k>i} w_k c_k by a row
// suffix sum plus the carry -- never as C minus a prefix.
__global__ void __launch_bounds__(kBlock) composite_bwd_kernel(
    const int64_t *__restrict__ offsets, int64_t n_rays, int64_t n_samples, const float *__restrict__ t0,
    const float *__restrict__ t1,
    const float *__restrict__ sigma, const float *__restrict__ rgb, const float *__restrict__ g_rgb,
    const float *__restrict__ g_opacity, float *__restrict__ d_sigma, float *__restrict__ d_rgb) {
    const int l = threadIdx.x & (kRow - 1);
    const int64_t r = (int64_t)blockIdx.x * kRaysPerBlock + (threadIdx.x / kRow);
    const bool live = r < n_rays;
    const int64_t a = live ? offsets[r] : 0, b = live ? offsets[r + 1] : 0;
    const int64_t last = b > a ? a + ((b - a - 1) / kSpanBwd) * kSpanBwd : a;   // first sample of the last group
    float dt[kGroupBwd], tau[kGroupBwd], xr[kGroupBwd], xg[kGroupBwd], xb[kGroupBwd];
    auto load_group = [&](int64_t g0) {
#pragma unroll
        for (int c = 0; c < kGroupBwd; ++c) {
            const int64_t i = g0 + c * kRow + l;
            dt[c] = tau[c] = xr[c] = xg[c] = xb[c] = 0.f;
            if (i < b) {
                dt[c] = t1[i] - t0[i];
                tau[c] = sigma[i] * dt[c];
                xr[c] = rgb[3 * i + 0];
                xg[c] = rgb[3 * i + 1];
                xb[c] = rgb[3 * i + 2];
            }
        }
    };

    float part = 0.f;
    for (int64_t g0 = a; g0 < last; g0 += kSpanBwd) {   // whole groups before the last
        float q[kGroupBwd];
#pragma unroll
        for (int c = 0; c < kGroupBwd; ++c) {
            const int64_t i = g0 + c * kRow + l;
            q[c] = sigma[i] * (t1[i] - t0[i]);
        }
#pragma unroll
        for (int c = 0; c < kGroupBwd; ++c) part += q[c];
    }
    load_group(last);
#pragma unroll
    for (int c = 0; c < kGroupBwd; ++c) part += tau[c];
    const float total = row_lane(row_prefix(part), kRow - 1);

    const float gr = live ? g_rgb[3 * r + 0] : 0.f, gg = live ? g_rgb[3 * r + 1] : 0.f;
    const float gb = live ? g_rgb[3 * r + 2] : 0.f;
    const float ga = live && g_opacity ? g_opacity[r] : 0.f;
    const float T_end = expf(-total);
    float after_tau = 0.f;                      // depth of the later chunks
    float ar = 0.f, ag = 0.f, ab = 0.f;         // sum of w c over the later chunks
    for (int64_t g0 = last; g0 >= a; g0 -= kSpanBwd) {   // row-uniform
        if (g0 != last) load_group(g0);
#pragma unroll
        for (int c = kGroupBwd - 1; c >= 0; --c) {
            if (g0 + c * kRow >= b) continue;   // row-uniform
            const int64_t i = g0 + c * kRow + l;
            const bool ok = i < b;
            const float sfx_row = row_suffix(tau[c]);
            const float sfx = sfx_row + after_tau;   // depth at and after i
            const float T_here = expf(-(total - sfx));
            const float T_next = expf(-(total - (sfx - tau[c])));
            const float w = ok ? T_here * (-expm1f(-tau[c])) : 0.f;
            const float wr = w * xr[c], wg = w * xg[c], wb = w * xb[c];
            const float qr = row_suffix(wr), qg = row_suffix(wg), qb = row_suffix(wb);
            const float sr = qr - wr + ar;   // sum over k > i
            const float sg = qg - wg + ag;
            const float sb = qb - wb + ab;
            if (ok) {
                const float dC = gr * (T_next * xr[c] - sr) + gg * (T_next * xg[c] - sg) + gb * (T_next * xb[c] - sb);
                d_sigma[i] = dt[c] * (dC + ga * T_end);
                d_rgb[3 * i + 0] = w * gr;
                d_rgb[3 * i + 1] = w * gg;
                d_rgb[3 * i + 2] = w * gb;
            }
            after_tau += row_lane(sfx_row, 0);
            ar += row_lane(qr, 0);
            ag += row_lane(qg, 0);
            ab += row_lane(qb, 0);
        }
        if (g0 == a) break;
    }
    // samples no ray owns (before offsets[0], from offsets[n_rays] on) get zero gradient
    const int64_t lo = offsets[0], hi = offsets[n_rays];
    const int64_t before = lo < n_samples ? lo : n_samples, after = hi < n_samples ? n_samples - hi : 0;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < before + after; k += (int64_t)gridDim.x * kBlock) {
        const int64_t i = k < before ? k : hi + (k - before);
        d_sigma[i] = 0.f;
        d_rgb[3 * i + 0] = 0.f;
        d_rgb[3 * i + 1] = 0.f;
        d_rgb[3 * i + 2] = 0.f;
    }
}

// ------------------------------------------------------------------ blob field

// Blob parameters as the kernel takes them (a by-value argument, so they sit
// in scalar registers): nk = -log2(e) / (2 radius^2), so that
// g = exp2(|x - c|^2 nk) is one hardware exp2.
struct BlobArgs {
    int n;
    float cx[OGV_MAX_BLOBS], cy[OGV_MAX_BLOBS], cz[OGV_MAX_BLOBS], nk[OGV_MAX_BLOBS];
    float a[OGV_MAX_BLOBS], r[OGV_MAX_BLOBS], g[OGV_MAX_BLOBS], b[OGV_MAX_BLOBS];
};

// One 16-lane row per ray, the composite forward's structure, with sigma and
// colour computed in registers from the field at each sample's midpoint
// instead of being read.
__global__ void __launch_bounds__(kBlock) render_blobs_kernel(const int64_t *__restrict__ offsets, int64_t n_rays,
                                                             const float *__restrict__ origins,
                                                             const float *__restrict__ dirs,
                                                             const float *__restrict__ t0,
                                                             const float *__restrict__ t1, BlobArgs f,
                                                             float *__restrict__ out_rgb,
                                                             float *__restrict__ out_opacity) {
    const int l = threadIdx.x & (kRow - 1);
    const int64_t r = (int64_t)blockIdx.x * kRaysPerBlock + (threadIdx.x / kRow);
    const bool live = r < n_rays;
    const int64_t a = live ? offsets[r] : 0, b = live ? offsets[r + 1] : 0;
    float o[3] = {0.f, 0.f, 0.f}, d[3] = {0.f, 0.f, 0.f};
    if (live && b > a) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            o[q] = origins[3 * r + q];
            d[q] = dirs[3 * r + q];
        }
    }
    float cr = 0.f, cg = 0.f, cb = 0.f, acc = 0.f, carry = 0.f;
    for (int64_t g0 = a; g0 < b; g0 += kSpan) {   // row-uniform
        float mid[kGroup], dt[kGroup];
#pragma unroll
        for (int c = 0; c < kGroup; ++c) {
            const int64_t i = g0 + c * kRow + l;
            mid[c] = dt[c] = 0.f;
            if (i < b) {
                const float u = t0[i], v = t1[i];
                mid[c] = 0.5f * (u + v);
                dt[c] = v - u;
            }
        }
#pragma unroll
        for (int c = 0; c < kGroup; ++c) {
            if (g0 + c * kRow >= b) break;   // row-uniform
            const bool ok = g0 + c * kRow + l < b;
            const float x = fmaf(d[0], mid[c], o[0]), y = fmaf(d[1], mid[c], o[1]), z = fmaf(d[2], mid[c], o[2]);
            float sig = 0.f, nr = 0.f, ng = 0.f, nb = 0.f;
            for (int k = 0; k < f.n; ++k) {
                const float ex = x - f.cx[k], ey = y - f.cy[k], ez = z - f.cz[k];
                const float d2 = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
                const float w = f.a[k] * __builtin_amdgcn_exp2f(d2 * f.nk[k]);
                sig += w;
                nr = fmaf(w, f.r[k], nr);
                ng = fmaf(w, f.g[k], ng);
                nb = fmaf(w, f.b[k], nb);
            }
            const float inv = sig > 0.f ? 1.0f / sig : 0.f;
            const float tau = ok ? sig * dt[c] : 0.f;
            const float incl = row_prefix(tau);
            const float T = expf(-(carry + incl - tau));
            const float w = ok ? T * (-expm1f(-tau)) : 0.f;
            const float wi = w * inv;
            cr = fmaf(wi, nr, cr);
            cg = fmaf(wi, ng, cg);
            cb = fmaf(wi, nb, cb);
            acc += w;
            carry += row_lane(incl, kRow - 1);
        }
    }
    cr = row_prefix(cr);
    cg = row_prefix(cg);
    cb = row_prefix(cb);
    acc = row_prefix(acc);
    if (live && l == kRow - 1) {
        out_rgb[3 * r + 0] = cr;
        out_rgb[3 * r + 1] = cg;
        out_rgb[3 * r + 2] = cb;
        if (out_opacity) out_opacity[r] = acc;
    }
}

}  // namespace
}  // namespace ogv

using namespace ogv;

extern "C" ogv_status ogv_composite_fwd(const int64_t *offsets, int64_t n_rays, const float *t0, const float *t1,
                                        const float *sigma, const float *rgb, float *out_rgb, float *out_opacity,
                                        void *stream) {
    if (n_rays < 0) OGV_FAIL(OGV_ERR_INVALID, "n_rays < 0");
    if (n_rays == 0) return OGV_OK;
    if (!offsets || !out_rgb || !t0 || !t1 || !sigma || !rgb) OGV_FAIL(OGV_ERR_INVALID, "null argument");
    hipStream_t s = (hipStream_t)stream;
    const unsigned blocks = (unsigned)((n_rays + kRaysPerBlock - 1) / kRaysPerBlock);
    composite_fwd_kernel<<<blocks, kBlock, 0, s>>>(offsets, n_rays, t0, t1, sigma, rgb, out_rgb, out_opacity);
    OGV_CHECK_LAUNCH();
    return OGV_OK;
}

extern "C" ogv_status ogv_composite_bwd(const int64_t *offsets, int64_t n_rays, int64_t n_samples, const float *t0,
                                        const float *t1,
                                        const float *sigma, const float *rgb, const float *g_rgb,
                                        const float *g_opacity, float *d_sigma, float *d_rgb, void *stream) {
    if (n_rays < 0) OGV_FAIL(OGV_ERR_INVALID, "n_rays < 0");
    if (n_samples < 0) OGV_FAIL(OGV_ERR_INVALID, "n_samples < 0");
    if (n_rays == 0 && n_samples == 0) return OGV_OK;
    if (!offsets || !t0 || !t1 || !sigma || !rgb || !g_rgb || !d_sigma || !d_rgb)
        OGV_FAIL(OGV_ERR_INVALID, "null argument");
    hipStream_t s = (hipStream_t)stream;
    // at least one block, so that an empty ray range still zeroes the samples
    const unsigned blocks = (unsigned)std::max<int64_t>((n_rays + kRaysPerBlock - 1) / kRaysPerBlock, 1);
    composite_bwd_kernel<<<blocks, kBlock, 0, s>>>(offsets, n_rays, n_samples, t0, t1, sigma, rgb, g_rgb, g_opacity,
                                                   d_sigma, d_rgb);
    OGV_CHECK_LAUNCH();
    return OGV_OK;
}

extern "C" ogv_status ogv_render_blobs(const int64_t *offsets, int64_t n_rays, const float *origins, const float *dirs,
                                       const float *t0, const float *t1, const ogv_blob_field *field, float *out_rgb,
                                       float *out_opacity, void *stream) {
    if (n_rays < 0) OGV_FAIL(OGV_ERR_INVALID, "n_rays < 0");
    if (!field) OGV_FAIL(OGV_ERR_INVALID, "null field");
    if (field->n < 1 || field->n > OGV_MAX_BLOBS) OGV_FAIL(OGV_ERR_INVALID, "blob count outside 1..16");
    BlobArgs f{};
    f.n = field->n;
    for (int k = 0; k < field->n; ++k) {
        const float rad = field->radius[k], den = field->density[k];
        if (!(rad > 0.f) || !(den >= 0.f) || !std::isfinite(rad) || !std::isfinite(den))
            OGV_FAIL(OGV_ERR_INVALID, "blob radius must be > 0 and density >= 0, both finite");
        f.cx[k] = field->centre[k][0];
        f.cy[k] = field->centre[k][1];
        f.cz[k] = field->centre[k][2];
        f.nk[k] = (float)(-1.4426950408889634 / (2.0 * (double)rad * (double)rad));   // -log2(e) / (2 r^2)
        f.a[k] = den;
        f.r[k] = field->colour[k][0];
        f.g[k] = field->colour[k][1];
        f.b[k] = field->colour[k][2];
    }
    if (n_rays == 0) return OGV_OK;
    if (!offsets || !origins || !dirs || !t0 || !t1 || !out_rgb) OGV_FAIL(OGV_ERR_INVALID, "null argument");
    hipStream_t s = (hipStream_t)stream;
    const unsigned blocks = (unsigned)((n_rays + kRaysPerBlock - 1) / kRaysPerBlock);
    render_blobs_kernel<<<blocks, kBlock, 0, s>>>(offsets, n_rays, origins, dirs, t0, t1, f, out_rgb, out_opacity);
    OGV_CHECK_LAUNCH();
    return OGV_OK;
}
