"""FP64 composite oracle against closed forms and central finite differences.

The paper only says the samples' colours and densities are accumulated into
the pixel (Sec. 1); the emission-absorption quadrature is the reading taken
(alpha = 1 - exp(-sigma*dt), T = exp(-sum of earlier sigma*dt)).
"""
import math

import numpy as np
import pytest

from oracle import (composite_forward, composite_backward, composite_loss_grad, composite_forward_all,
                    composite_backward_all)

# the loop form (ray by ray, sample by sample) and the array form (every ray at
# once, for checks over a whole image) face the same pins
FORMS = {"loop": (composite_forward, composite_backward), "array": (composite_forward_all, composite_backward_all)}


@pytest.mark.parametrize("form", FORMS)
def test_one_sample_closed_form(form):
    composite_forward, composite_backward = FORMS[form]
    # dt = 1, sigma = ln 2: alpha = w = A = 1/2, C = c/2, dA/dsigma = 1/2, dC/dsigma = c/2
    c = np.array([[0.2, 0.5, 0.9]])
    C, A, Tf = composite_forward([0, 1], [0.0], [1.0], [math.log(2.0)], c)
    np.testing.assert_allclose(A, [0.5], rtol=1e-15)
    np.testing.assert_allclose(C, 0.5 * c, rtol=1e-15)
    np.testing.assert_allclose(Tf, [0.5], rtol=1e-15)
    ds, _ = composite_backward([0, 1], [0.0], [1.0], [math.log(2.0)], c, np.zeros((1, 3)), [1.0])
    np.testing.assert_allclose(ds, [0.5], rtol=1e-15)
    for ch in range(3):
        g = np.zeros((1, 3))
        g[0, ch] = 1.0
        ds, drgb = composite_backward([0, 1], [0.0], [1.0], [math.log(2.0)], c, g, [0.0])
        np.testing.assert_allclose(ds, [0.5 * c[0, ch]], rtol=1e-14)
        np.testing.assert_allclose(drgb[0], 0.5 * g[0], rtol=1e-15)


@pytest.mark.parametrize("form", FORMS)
def test_two_samples_closed_form(form):
    composite_forward, composite_backward = FORMS[form]
    # w = (1/2, 1/4), A = 3/4; dA/dsigma_0 = dA/dsigma_1 = 1/4;
    # dC/dsigma_0 = c0/2 - c1/4, dC/dsigma_1 = c1/4
    c = np.array([[0.3, 0.6, 0.1], [0.8, 0.2, 0.4]])
    sig = [math.log(2.0)] * 2
    t0, t1 = [0.0, 1.0], [1.0, 2.0]
    C, A, _ = composite_forward([0, 2], t0, t1, sig, c)
    np.testing.assert_allclose(A, [0.75], rtol=1e-15)
    np.testing.assert_allclose(C[0], 0.5 * c[0] + 0.25 * c[1], rtol=1e-15)
    ds, _ = composite_backward([0, 2], t0, t1, sig, c, np.zeros((1, 3)), [1.0])
    np.testing.assert_allclose(ds, [0.25, 0.25], rtol=1e-14)
    for ch in range(3):
        g = np.zeros((1, 3))
        g[0, ch] = 1.0
        ds, _ = composite_backward([0, 2], t0, t1, sig, c, g, [0.0])
        np.testing.assert_allclose(ds, [0.5 * c[0, ch] - 0.25 * c[1, ch], 0.25 * c[1, ch]], rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("form", FORMS)
def test_weights_sum_to_opacity_and_empty_rays(form):
    composite_forward, composite_backward = FORMS[form]
    rng = np.random.default_rng(0)
    counts = np.array([0, 3, 0, 7, 1])
    off = np.concatenate([[0], np.cumsum(counts)])
    S = off[-1]
    t0 = np.sort(rng.random(S))
    t1 = t0 + rng.uniform(0.001, 0.1, S)
    sig = np.exp(rng.normal(size=S))
    rgb = np.ones((S, 3))
    C, A, Tf = composite_forward(off, t0, t1, sig, rgb)
    np.testing.assert_allclose(A, 1.0 - Tf, atol=1e-15)
    np.testing.assert_allclose(C[:, 0], A, atol=1e-15)  # white samples: C = A
    assert A[0] == 0 and A[2] == 0 and np.all(C[[0, 2]] == 0)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_gradient_matches_central_differences(seed, form):
    composite_forward, composite_backward = FORMS[form]
    rng = np.random.default_rng(seed)
    counts = rng.integers(0, 12, size=6)
    off = np.concatenate([[0], np.cumsum(counts)])
    S = int(off[-1])
    t0 = np.cumsum(rng.uniform(0.001, 0.02, S))
    t1 = t0 + rng.uniform(0.001, 0.02, S)
    sig = np.exp(rng.normal(size=S)) * 20
    rgb = rng.random((S, 3))
    target = rng.random((len(counts), 3))

    def loss(s, c):
        C, _, _ = composite_forward(off, t0, t1, s, c)
        return composite_loss_grad(C, target)[0]

    C, A, _ = composite_forward(off, t0, t1, sig, rgb)
    _, gC = composite_loss_grad(C, target)
    ds, drgb = composite_backward(off, t0, t1, sig, rgb, gC, np.zeros(len(counts)))
    eps = 1e-6
    for i in range(S):
        sp, sm = sig.copy(), sig.copy()
        sp[i] += eps
        sm[i] -= eps
        fd = (loss(sp, rgb) - loss(sm, rgb)) / (2 * eps)
        assert abs(fd - ds[i]) <= 1e-7 * max(1.0, abs(ds).max()), (i, fd, ds[i])
        for ch in range(3):
            cp, cm = rgb.copy(), rgb.copy()
            cp[i, ch] += eps
            cm[i, ch] -= eps
            fd = (loss(sig, cp) - loss(sig, cm)) / (2 * eps)
            assert abs(fd - drgb[i, ch]) <= 1e-7 * max(1.0, abs(drgb).max())


@pytest.mark.parametrize("form", FORMS)
def test_opacity_gradient_matches_central_differences(form):
    composite_forward, composite_backward = FORMS[form]
    rng = np.random.default_rng(9)
    off = np.array([0, 5])
    t0 = np.cumsum(rng.uniform(0.01, 0.05, 5))
    t1 = t0 + 0.03
    sig = np.exp(rng.normal(size=5)) * 10
    rgb = rng.random((5, 3))
    ds, _ = composite_backward(off, t0, t1, sig, rgb, np.zeros((1, 3)), [1.0])
    eps = 1e-6
    for i in range(5):
        sp, sm = sig.copy(), sig.copy()
        sp[i] += eps
        sm[i] -= eps
        fd = (composite_forward(off, t0, t1, sp, rgb)[1][0] - composite_forward(off, t0, t1, sm, rgb)[1][0]) / (2 * eps)
        assert abs(fd - ds[i]) < 1e-8


def test_forms_agree_on_an_image():
    # uneven rays (empty ones included) of dense and sparse media; the two forms
    # differ only in FP64 rounding order
    rng = np.random.default_rng(17)
    counts = rng.integers(0, 300, size=200)
    counts[rng.choice(200, 20, replace=False)] = 0
    off = np.concatenate([[0], np.cumsum(counts)])
    S = int(off[-1])
    t0 = rng.uniform(2.0, 6.0, S)
    t1 = t0 + 0.005
    sig = np.exp(rng.normal(size=S)) * rng.choice([0.1, 10.0, 200.0], S)
    rgb = rng.random((S, 3))
    gC = rng.normal(size=(200, 3))
    gA = rng.normal(size=200)
    a = composite_forward(off, t0, t1, sig, rgb)
    b = composite_forward_all(off, t0, t1, sig, rgb)
    for x, y in zip(a, b):
        np.testing.assert_allclose(y, x, rtol=1e-11, atol=1e-15)
    a = composite_backward(off, t0, t1, sig, rgb, gC, gA)
    b = composite_backward_all(off, t0, t1, sig, rgb, gC, gA)
    for x, y in zip(a, b):
        np.testing.assert_allclose(y, x, rtol=1e-9, atol=1e-12 * np.abs(x).max())
