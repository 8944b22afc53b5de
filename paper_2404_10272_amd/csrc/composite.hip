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
// at the level of one rounding of the ray's total optical depth.  One wave
// handles one ray, 64 consecutive samples at a time.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace ogv {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;

__device__ __forceinline__ float wave_incl_scan(float x, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        float y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// inclusive scan from the high lanes down: lane i gets sum over lanes >= i
__device__ __forceinline__ float wave_rev_incl_scan(float x, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        float y = __shfl_down(x, off, 64);
        if (lane + off < 64) x += y;
    }
    return x;
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// One wave per ray: 64 consecutive samples per step (coalesced loads), the
// optical depth before each sample by a wave prefix scan plus the running
// carry of the earlier chunks.
__global__ void __launch_bounds__(kBlock) composite_fwd_kernel(const int64_t *__restrict__ offsets, int64_t n_rays,
                                                              const float *__restrict__ t0,
                                                              const float *__restrict__ t1,
                                                              const float *__restrict__ sigma,
                                                              const float *__restrict__ rgb, float *__restrict__ out_rgb,
                                                              float *__restrict__ out_opacity) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (r >= n_rays) return;
    const int64_t a = offsets[r], b = offsets[r + 1];
    float cr = 0.f, cg = 0.f, cb = 0.f, acc = 0.f, carry = 0.f;
    for (int64_t base = a; base < b; base += 64) {
        const int64_t i = base + lane;
        const bool ok = i < b;
        const float tau = ok ? sigma[i] * (t1[i] - t0[i]) : 0.f;
        const float incl = wave_incl_scan(tau, lane);
        const float T = expf(-(carry + incl - tau));
        const float w = ok ? T * (-expm1f(-tau)) : 0.f;
        if (ok) {
            cr += w * rgb[3 * i + 0];
            cg += w * rgb[3 * i + 1];
            cb += w * rgb[3 * i + 2];
        }
        acc += w;
        carry += __shfl(incl, 63, 64);
    }
    cr = wave_sum(cr);
    cg = wave_sum(cg);
    cb = wave_sum(cb);
    acc = wave_sum(acc);
    if (lane == 0) {
        out_rgb[3 * r + 0] = cr;
        out_rgb[3 * r + 1] = cg;
        out_rgb[3 * r + 2] = cb;
        if (out_opacity) out_opacity[r] = acc;
    }
}

// One wave per ray.  Pass 1: the ray's total optical depth.  Pass 2, chunks
// from the back: T_i and T_{i+1} from the total minus the depth at and after
// i (reverse scan plus the carry of later chunks), and sum_{k>i} w_k c_k by a
// reverse scan plus the carry -- never as C minus a prefix.
__global__ void __launch_bounds__(kBlock) composite_bwd_kernel(
    const int64_t *__restrict__ offsets, int64_t n_rays, const float *__restrict__ t0, const float *__restrict__ t1,
    const float *__restrict__ sigma, const float *__restrict__ rgb, const float *__restrict__ g_rgb,
    const float *__restrict__ g_opacity, float *__restrict__ d_sigma, float *__restrict__ d_rgb) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (r >= n_rays) return;
    const int64_t a = offsets[r], b = offsets[r + 1];
    if (a == b) return;
    float part = 0.f;
    for (int64_t i = a + lane; i < b; i += 64) part += sigma[i] * (t1[i] - t0[i]);
    const float total = wave_sum(part);
    const float gr = g_rgb[3 * r + 0], gg = g_rgb[3 * r + 1], gb = g_rgb[3 * r + 2];
    const float ga = g_opacity ? g_opacity[r] : 0.f;
    const float T_end = expf(-total);
    float after_tau = 0.f;                      // depth of the later chunks
    float ar = 0.f, ag = 0.f, ab = 0.f;         // sum of w c over the later chunks
    for (int64_t base = a + ((b - a - 1) / 64) * 64; base >= a; base -= 64) {
        const int64_t i = base + lane;
        const bool ok = i < b;
        const float dt = ok ? t1[i] - t0[i] : 0.f;
        const float tau = ok ? sigma[i] * dt : 0.f;
        const float sfx = wave_rev_incl_scan(tau, lane) + after_tau;   // depth at and after i
        const float T_here = expf(-(total - sfx));
        const float T_next = expf(-(total - (sfx - tau)));
        const float w = ok ? T_here * (-expm1f(-tau)) : 0.f;
        float cr = 0.f, cg = 0.f, cb = 0.f;
        if (ok) {
            cr = rgb[3 * i + 0];
            cg = rgb[3 * i + 1];
            cb = rgb[3 * i + 2];
        }
        const float wr = w * cr, wg = w * cg, wb = w * cb;
        const float sr = wave_rev_incl_scan(wr, lane) - wr + ar;   // sum over k > i
        const float sg = wave_rev_incl_scan(wg, lane) - wg + ag;
        const float sb = wave_rev_incl_scan(wb, lane) - wb + ab;
        if (ok) {
            const float dC = gr * (T_next * cr - sr) + gg * (T_next * cg - sg) + gb * (T_next * cb - sb);
            d_sigma[i] = dt * (dC + ga * T_end);
            d_rgb[3 * i + 0] = w * gr;
            d_rgb[3 * i + 1] = w * gg;
            d_rgb[3 * i + 2] = w * gb;
        }
        after_tau += wave_sum(tau);
        ar += wave_sum(wr);
        ag += wave_sum(wg);
        ab += wave_sum(wb);
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
    const unsigned blocks = (unsigned)((n_rays + kWavesPerBlock - 1) / kWavesPerBlock);
    composite_fwd_kernel<<<blocks, kBlock, 0, s>>>(offsets, n_rays, t0, t1, sigma, rgb, out_rgb, out_opacity);
    OGV_CHECK_LAUNCH();
    return OGV_OK;
}

extern "C" ogv_status ogv_composite_bwd(const int64_t *offsets, int64_t n_rays, const float *t0, const float *t1,
                                        const float *sigma, const float *rgb, const float *g_rgb,
                                        const float *g_opacity, float *d_sigma, float *d_rgb, void *stream) {
    if (n_rays < 0) OGV_FAIL(OGV_ERR_INVALID, "n_rays < 0");
    if (n_rays == 0) return OGV_OK;
    if (!offsets || !t0 || !t1 || !sigma || !rgb || !g_rgb || !d_sigma || !d_rgb)
        OGV_FAIL(OGV_ERR_INVALID, "null argument");
    hipStream_t s = (hipStream_t)stream;
    const unsigned blocks = (unsigned)((n_rays + kWavesPerBlock - 1) / kWavesPerBlock);
    composite_bwd_kernel<<<blocks, kBlock, 0, s>>>(offsets, n_rays, t0, t1, sigma, rgb, g_rgb, g_opacity, d_sigma,
                                                   d_rgb);
    OGV_CHECK_LAUNCH();
    return OGV_OK;
}
