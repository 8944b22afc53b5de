"""FP64 rendering of packed samples through a Gaussian-blob radiance field.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The sampler's points are fed to a radiance field and the results composited
into the pixel (Sec. 1). The paper's field is a trained network, which is not
available here, so a synthetic field of K Gaussian blobs stands in for it:

    g_k(x)    = exp(-|x - c_k|^2 / (2 r_k^2))
    sigma(x)  = sum_k a_k g_k(x)
    colour(x) = sum_k a_k g_k(x) col_k / sigma(x)        (0 where sigma(x) = 0)

Each sample is taken at its interval midpoint, x_i = o + d (t0_i + t1_i) / 2,
and the ray is composited with composite_forward (emission-absorption).
render_blobs_all does the same for every ray at once (the field evaluated in
chunks of samples, the composite in array form), for checks over a whole
image.
"""
import numpy as np

from .composite import composite_forward, composite_forward_all


def blob_field(points, centres, radii, densities, colours):
    """(sigma[P], colour[P,3]) of the blob field at points [P,3], in float64."""
    x = np.asarray(points, np.float64).reshape(-1, 3)
    c = np.asarray(centres, np.float64).reshape(-1, 3)
    r = np.asarray(radii, np.float64)
    a = np.asarray(densities, np.float64)
    col = np.asarray(colours, np.float64).reshape(-1, 3)
    d2 = ((x[:, None, :] - c[None, :, :]) ** 2).sum(axis=2)          # [P, K]
    w = a[None, :] * np.exp(-d2 / (2.0 * r[None, :] ** 2))           # [P, K]
    sigma = w.sum(axis=1)
    num = w @ col
    colour = np.where(sigma[:, None] > 0, num / np.where(sigma > 0, sigma, 1.0)[:, None], 0.0)
    return sigma, colour


def render_blobs(offsets, origins, dirs, t0, t1, centres, radii, densities, colours, rays=None):
    """Pixel (C[R,3], A[R]) of the listed rays (all if None), float64."""
    offsets = np.asarray(offsets, np.int64)
    o = np.asarray(origins, np.float64).reshape(-1, 3)
    d = np.asarray(dirs, np.float64).reshape(-1, 3)
    t0 = np.asarray(t0, np.float64)
    t1 = np.asarray(t1, np.float64)
    rays = np.arange(offsets.shape[0] - 1) if rays is None else np.asarray(rays, np.int64)
    C = np.zeros((rays.shape[0], 3))
    A = np.zeros(rays.shape[0])
    for j, r in enumerate(rays):
        a, b = offsets[r], offsets[r + 1]
        if b <= a:
            continue
        mid = 0.5 * (t0[a:b] + t1[a:b])
        pts = o[r][None, :] + d[r][None, :] * mid[:, None]
        sigma, colour = blob_field(pts, centres, radii, densities, colours)
        Cr, Ar, _ = composite_forward([0, b - a], t0[a:b], t1[a:b], sigma, colour)
        C[j], A[j] = Cr[0], Ar[0]
    return C, A


def render_blobs_all(offsets, origins, dirs, t0, t1, centres, radii, densities, colours, chunk=1 << 21):
    """Pixel (C[N,3], A[N]) of every ray, float64: render_blobs in array form.
    offsets[0] must be 0; samples past offsets[-1] are ignored."""
    offsets = np.asarray(offsets, np.int64)
    counts = np.diff(offsets)
    ray = np.repeat(np.arange(counts.size), counts)
    S = ray.shape[0]
    o = np.asarray(origins, np.float64).reshape(-1, 3)
    d = np.asarray(dirs, np.float64).reshape(-1, 3)
    t0 = np.asarray(t0, np.float64)[:S]
    t1 = np.asarray(t1, np.float64)[:S]
    sigma = np.empty(S)
    colour = np.empty((S, 3))
    for a in range(0, S, chunk):
        b = min(S, a + chunk)
        mid = 0.5 * (t0[a:b] + t1[a:b])
        pts = o[ray[a:b]] + d[ray[a:b]] * mid[:, None]
        sigma[a:b], colour[a:b] = blob_field(pts, centres, radii, densities, colours)
    C, A, _ = composite_forward_all(offsets, t0, t1, sigma, colour)
    return C, A
