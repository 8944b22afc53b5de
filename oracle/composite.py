"""FP64 volume-rendering composite over packed samples, and its gradient.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper only says that the colours and densities of a ray's samples are
accumulated into the pixel colour (Sec. 1); the standard emission-absorption
quadrature is used, per ray over its samples i = 0..n-1 in order:

    dt_i    = t1_i - t0_i
    tau_i   = sigma_i * dt_i
    alpha_i = 1 - exp(-tau_i)
    T_i     = exp(-sum_{j<i} tau_j)            (transmittance before sample i)
    w_i     = T_i * alpha_i
    C       = sum_i w_i * c_i                  (pixel RGB)
    A       = sum_i w_i = 1 - T_n              (opacity)

Gradient, with g_C = dL/dC and g_A = dL/dA:

    dL/dc_i     = w_i * g_C
    dL/dsigma_i = dt_i * ( g_C . (T_{i+1} c_i - sum_{k>i} w_k c_k) + g_A * T_n )

The suffix sum is taken as a reverse running sum (not C minus a prefix).
No early termination and no clipping at t_max.
"""
import numpy as np


def _rays(offsets):
    offsets = np.asarray(offsets, dtype=np.int64)
    return offsets.shape[0] - 1, offsets


def composite_forward(offsets, t0, t1, sigma, rgb):
    """Returns (C[N,3], A[N], T_final[N]) in float64."""
    n_rays, offsets = _rays(offsets)
    t0 = np.asarray(t0, np.float64)
    t1 = np.asarray(t1, np.float64)
    sigma = np.asarray(sigma, np.float64)
    rgb = np.asarray(rgb, np.float64).reshape(-1, 3)
    C = np.zeros((n_rays, 3))
    A = np.zeros(n_rays)
    Tf = np.ones(n_rays)
    for r in range(n_rays):
        a, b = offsets[r], offsets[r + 1]
        T = 1.0
        for i in range(a, b):
            tau = sigma[i] * (t1[i] - t0[i])
            alpha = -np.expm1(-tau)
            w = T * alpha
            C[r] += w * rgb[i]
            A[r] += w
            T = T * np.exp(-tau)
        Tf[r] = T
    return C, A, Tf


def composite_backward(offsets, t0, t1, sigma, rgb, g_C, g_A):
    """Returns (dL/dsigma[S], dL/drgb[S,3]) in float64."""
    n_rays, offsets = _rays(offsets)
    t0 = np.asarray(t0, np.float64)
    t1 = np.asarray(t1, np.float64)
    sigma = np.asarray(sigma, np.float64)
    rgb = np.asarray(rgb, np.float64).reshape(-1, 3)
    g_C = np.asarray(g_C, np.float64).reshape(-1, 3)
    g_A = np.asarray(g_A, np.float64).reshape(-1)
    d_sigma = np.zeros(sigma.shape[0])
    d_rgb = np.zeros((sigma.shape[0], 3))
    for r in range(n_rays):
        a, b = offsets[r], offsets[r + 1]
        if a == b:
            continue
        n = b - a
        dt = t1[a:b] - t0[a:b]
        tau = sigma[a:b] * dt
        T_before = np.empty(n)
        T_after = np.empty(n)
        T = 1.0
        for i in range(n):
            T_before[i] = T
            T = T * np.exp(-tau[i])
            T_after[i] = T
        T_final = T
        w = T_before * (-np.expm1(-tau))
        suffix = np.zeros(3)  # sum_{k>i} w_k c_k, built from the back
        for i in range(n - 1, -1, -1):
            c = rgb[a + i]
            dC_dtau = T_after[i] * c - suffix
            d_sigma[a + i] = dt[i] * (np.dot(g_C[r], dC_dtau) + g_A[r] * T_final)
            d_rgb[a + i] = w[i] * g_C[r]
            suffix = suffix + w[i] * c
    return d_sigma, d_rgb


def composite_loss_grad(C, target):
    """L = mean over rays and channels of (C - target)^2; returns (L, dL/dC)."""
    C = np.asarray(C, np.float64)
    target = np.asarray(target, np.float64)
    diff = C - target
    return float(np.mean(diff * diff)), 2.0 * diff / diff.size


# ---------------------------------------------------------------------------
# The same quantities for every ray at once, in array form, so that a whole
# image of packed samples can be checked: per-ray sums become segment sums
# over the ray each sample belongs to.  T before sample i is exp of minus the
# sum of the ray's earlier tau (the loop form multiplies the factors; the two
# agree to FP64 rounding), and the suffix sum over later samples is the ray's
# total less the inclusive prefix.  offsets[0] must be 0.

def _ray_of_sample(offsets):
    offsets = np.asarray(offsets, dtype=np.int64)
    counts = np.diff(offsets)
    return offsets, counts, np.repeat(np.arange(counts.size), counts)


def _earlier_sum(x, offsets, ray):
    """For each sample, the sum of x over the earlier samples of its ray."""
    cs = np.cumsum(x, axis=0)
    before = np.concatenate([np.zeros((1,) + x.shape[1:]), cs])[offsets[:-1]]
    return cs - x - before[ray]


def composite_forward_all(offsets, t0, t1, sigma, rgb):
    """composite_forward over every ray in array form: (C[N,3], A[N], T_final[N])."""
    offsets, counts, ray = _ray_of_sample(offsets)
    n_rays = counts.size
    tau = np.asarray(sigma, np.float64) * (np.asarray(t1, np.float64) - np.asarray(t0, np.float64))
    rgb = np.asarray(rgb, np.float64).reshape(-1, 3)
    w = np.exp(-_earlier_sum(tau, offsets, ray)) * (-np.expm1(-tau))
    C = np.stack([np.bincount(ray, weights=w * rgb[:, k], minlength=n_rays) for k in range(3)], axis=1)
    A = np.bincount(ray, weights=w, minlength=n_rays)
    Tf = np.exp(-np.bincount(ray, weights=tau, minlength=n_rays))
    return C, A, Tf


def composite_backward_all(offsets, t0, t1, sigma, rgb, g_C, g_A):
    """composite_backward over every ray in array form: (dL/dsigma[S], dL/drgb[S,3])."""
    offsets, counts, ray = _ray_of_sample(offsets)
    n_rays = counts.size
    dt = np.asarray(t1, np.float64) - np.asarray(t0, np.float64)
    tau = np.asarray(sigma, np.float64) * dt
    rgb = np.asarray(rgb, np.float64).reshape(-1, 3)
    g_C = np.asarray(g_C, np.float64).reshape(-1, 3)
    g_A = np.asarray(g_A, np.float64).reshape(-1)
    earlier = _earlier_sum(tau, offsets, ray)
    T_after = np.exp(-(earlier + tau))
    T_final = np.exp(-np.bincount(ray, weights=tau, minlength=n_rays))
    w = np.exp(-earlier) * (-np.expm1(-tau))
    wc = w[:, None] * rgb
    total = np.stack([np.bincount(ray, weights=wc[:, k], minlength=n_rays) for k in range(3)], axis=1)
    later = total[ray] - (_earlier_sum(wc, offsets, ray) + wc)   # sum_{k>i} w_k c_k
    dC_dtau = T_after[:, None] * rgb - later
    d_sigma = dt * (np.einsum("ij,ij->i", g_C[ray], dC_dtau) + g_A[ray] * T_final[ray])
    d_rgb = w[:, None] * g_C[ray]
    return d_sigma, d_rgb
