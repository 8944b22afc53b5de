"""Fused composite forward/backward on the GPU against the FP64 oracle (every
ray of the object workload's packed samples, and the loop form on sampled
rays) and FP64 central finite differences (sampled rays).

Tolerance (per ray, separately for d_sigma and d_rgb and for the forward
outputs): ||g - g_ref||_inf <= 1e-4 * max(||g_ref||_inf, tiny).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2404_10272_amd import api, scenes

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def packed():
    w = scenes.workload("object")
    g = api.build_vdb(torch.from_numpy(w.occ).cuda(), w.boxes, w.ilog2)
    out = api.sample_rays(g, torch.from_numpy(w.origins).cuda(), torch.from_numpy(w.dirs).cuda(), w.near, w.far,
                          api.make_step(w.step), "skip")
    S = out["t0"].numel()
    sigma, rgb, target = scenes.composite_inputs(S, w.n_rays)
    return out, sigma, rgb, target


def test_forward_backward_against_oracle(packed):
    out, sigma, rgb, target = packed
    offsets = out["offsets"]
    rng = np.random.default_rng(4001)
    off_h = offsets.cpu().numpy()
    counts = np.diff(off_h)
    rays = rng.choice(np.nonzero(counts > 0)[0], size=256, replace=False)
    rays.sort()
    t0 = out["t0"].cpu().numpy()
    t1 = out["t1"].cpu().numpy()

    sig_d = torch.from_numpy(sigma).cuda().requires_grad_(True)
    rgb_d = torch.from_numpy(rgb).cuda().requires_grad_(True)
    C, A = api.composite(sig_d, rgb_d, offsets, out["t0"], out["t1"])
    tgt = torch.from_numpy(target).cuda()
    loss = ((C - tgt) ** 2).mean()
    loss.backward()
    C_h, A_h = C.detach().cpu().numpy(), A.detach().cpu().numpy()
    gs, gr = sig_d.grad.cpu().numpy(), rgb_d.grad.cpu().numpy()
    N = off_h.shape[0] - 1
    for r in rays:
        a, b = off_h[r], off_h[r + 1]
        sub_off = np.array([0, b - a])
        Cr, Ar, _ = oracle.composite_forward(sub_off, t0[a:b], t1[a:b], sigma[a:b], rgb[a:b])
        assert np.abs(C_h[r] - Cr[0]).max() <= TOL * max(np.abs(Cr[0]).max(), 1e-30), r
        assert abs(A_h[r] - Ar[0]) <= TOL * max(abs(Ar[0]), 1e-30), r
        # the loss is a mean over all N rays and 3 channels
        gC = 2.0 * (Cr - target[r].astype(np.float64)) / (3.0 * N)
        ds, drgb = oracle.composite_backward(sub_off, t0[a:b], t1[a:b], sigma[a:b], rgb[a:b], gC, [0.0])
        assert np.abs(gs[a:b] - ds).max() <= TOL * max(np.abs(ds).max(), 1e-30), r
        assert np.abs(gr[a:b] - drgb).max() <= TOL * max(np.abs(drgb).max(), 1e-30), r


def _ray_max(x, off_h, counts):
    """Per nonempty ray, the largest |x| over its samples (x: [S] or [S, 3])."""
    x = np.abs(np.asarray(x, np.float64)).reshape(x.shape[0], -1).max(axis=1)
    return np.maximum.reduceat(x, off_h[:-1][counts > 0])


def test_all_rays_against_oracle(packed):
    """Every ray of the workload (640,000 rays, 25.8 M samples): the forward
    outputs, and the backward pass for a random upstream gradient of both
    outputs, against the oracle's array form, to the same per-ray bound."""
    out, sigma, rgb, _ = packed
    off = out["offsets"]
    N = off.numel() - 1
    off_h = off.cpu().numpy()
    counts = np.diff(off_h)
    t0 = out["t0"].cpu().numpy()
    t1 = out["t1"].cpu().numpy()
    sig = torch.from_numpy(sigma).cuda()
    col = torch.from_numpy(rgb).cuda()
    rng = np.random.default_rng(4004)
    g_rgb = rng.normal(size=(N, 3)).astype(np.float32)
    g_a = rng.normal(size=N).astype(np.float32)
    C, A = api.composite_forward(off, out["t0"], out["t1"], sig, col)
    d_s, d_c = api.composite_backward(off, out["t0"], out["t1"], sig, col, torch.from_numpy(g_rgb).cuda(),
                                      torch.from_numpy(g_a).cuda())
    torch.cuda.synchronize()
    C_h, A_h = C.cpu().numpy().astype(np.float64), A.cpu().numpy().astype(np.float64)
    Cr, Ar, _ = oracle.composite_forward_all(off_h, t0, t1, sigma, rgb)
    bad = np.abs(C_h - Cr).max(axis=1) > TOL * np.maximum(np.abs(Cr).max(axis=1), 1e-30)
    assert not bad.any(), (int(bad.sum()), np.nonzero(bad)[0][:5])
    bad = np.abs(A_h - Ar) > TOL * np.maximum(np.abs(Ar), 1e-30)
    assert not bad.any(), (int(bad.sum()), np.nonzero(bad)[0][:5])
    ds, dc = oracle.composite_backward_all(off_h, t0, t1, sigma, rgb, g_rgb, g_a)
    for got, ref, what in ((d_s.cpu().numpy(), ds, "d_sigma"), (d_c.cpu().numpy(), dc, "d_rgb")):
        err = _ray_max(got.astype(np.float64) - ref, off_h, counts)
        scale = np.maximum(_ray_max(ref, off_h, counts), 1e-30)
        assert (err <= TOL * scale).all(), (what, int((err > TOL * scale).sum()), float((err / scale).max()))


def test_gradient_against_fp64_finite_differences(packed):
    """FP64 central differences of the oracle's forward pass against the GPU
    backward pass of the loss mean((C - target)^2) + 0.5 A of each ray, for
    sigma and rgb, on 256 sampled rays with samples."""
    out, sigma, rgb, target = packed
    off_h = out["offsets"].cpu().numpy()
    t0 = out["t0"].cpu().numpy()
    t1 = out["t1"].cpu().numpy()
    counts = np.diff(off_h)
    rng = np.random.default_rng(4002)
    rays = rng.choice(np.nonzero(counts > 0)[0], size=256, replace=False)
    for r in rays:
        a, b = off_h[r], off_h[r + 1]
        sub = torch.tensor([0, b - a], dtype=torch.int64, device="cuda")
        s_d = torch.from_numpy(sigma[a:b].copy()).cuda().requires_grad_(True)
        c_d = torch.from_numpy(rgb[a:b].copy()).cuda().requires_grad_(True)
        C, A = api.composite(s_d, c_d, sub, out["t0"][a:b].contiguous(), out["t1"][a:b].contiguous())
        tg = torch.from_numpy(target[r:r + 1]).cuda()
        loss = ((C - tg) ** 2).mean() + 0.5 * A.sum()
        loss.backward()
        gs = s_d.grad.cpu().numpy().astype(np.float64)
        gc = c_d.grad.cpu().numpy().astype(np.float64)

        def L(sv, cv):
            Cr, Ar, _ = oracle.composite_forward([0, b - a], t0[a:b], t1[a:b], sv, cv)
            return np.mean((Cr - target[r:r + 1]) ** 2) + 0.5 * Ar.sum()

        s64 = sigma[a:b].astype(np.float64)
        c64 = rgb[a:b].astype(np.float64)
        fd_s = np.zeros(b - a)
        fd_c = np.zeros((b - a, 3))
        for i in range(b - a):
            e = 1e-6 * max(1.0, abs(s64[i]))
            sp, sm = s64.copy(), s64.copy()
            sp[i] += e
            sm[i] -= e
            fd_s[i] = (L(sp, c64) - L(sm, c64)) / (2 * e)
            for ch in range(3):
                cp, cm = c64.copy(), c64.copy()
                cp[i, ch] += 1e-6
                cm[i, ch] -= 1e-6
                fd_c[i, ch] = (L(s64, cp) - L(s64, cm)) / 2e-6
        assert np.abs(gs - fd_s).max() <= TOL * max(np.abs(fd_s).max(), 1e-12), (r, np.abs(gs - fd_s).max())
        assert np.abs(gc - fd_c).max() <= TOL * max(np.abs(fd_c).max(), 1e-12), (r, np.abs(gc - fd_c).max())


def test_empty_rays_give_zero(packed):
    off = torch.tensor([0, 0, 0], dtype=torch.int64, device="cuda")
    e = torch.zeros(1, device="cuda")  # no ray reads it: every range is empty
    C, A = api.composite_forward(off, e, e, e, torch.zeros((1, 3), device="cuda"))
    torch.cuda.synchronize()
    assert C.abs().sum().item() == 0 and A.abs().sum().item() == 0


def test_backward_zeroes_samples_no_ray_owns(packed):
    """ogv_composite_bwd writes every entry of its outputs: the gradient of a
    middle range of rays over the full sample arrays is the full call's inside
    the range and exactly zero outside it, whatever the buffers held."""
    out, sigma, rgb, _ = packed
    off = out["offsets"]
    N = off.numel() - 1
    S = out["t0"].numel()
    sig = torch.from_numpy(sigma).cuda()
    col = torch.from_numpy(rgb).cuda()
    g_rgb = torch.from_numpy(np.random.default_rng(4003).random((N, 3), np.float32)).cuda()
    g_a = torch.ones(N, device="cuda")
    full_s, full_c = api.composite_backward(off, out["t0"], out["t1"], sig, col, g_rgb, g_a)
    r0, r1 = N // 3, 2 * N // 3
    sub = off[r0:r1 + 1].contiguous()
    d_s = torch.full((S,), float("nan"), device="cuda")
    d_c = torch.full((S, 3), float("nan"), device="cuda")
    g_sub, a_sub = g_rgb[r0:r1].contiguous(), g_a[r0:r1].contiguous()
    api._check(api.lib().ogv_composite_bwd(api._ptr(sub), r1 - r0, S, api._ptr(out["t0"]), api._ptr(out["t1"]),
                                           api._ptr(sig), api._ptr(col), api._ptr(g_sub), api._ptr(a_sub),
                                           api._ptr(d_s), api._ptr(d_c), api._stream()))
    torch.cuda.synchronize()
    a, b = int(off[r0].item()), int(off[r1].item())
    assert 0 < a < b < S
    for got, ref in ((d_s, full_s), (d_c, full_c)):
        got, ref = got.cpu().numpy(), ref.cpu().numpy()
        assert not np.isnan(got).any()
        np.testing.assert_array_equal(got[a:b], ref[a:b])
        assert (got[:a] == 0).all() and (got[b:] == 0).all()
