"""Pins of the oracle's blob-field rendering against closed forms: the field
at a blob's centre and at one radius, the density-weighted colour, the
empty-field limit, the midpoint rule, and a constant field's opacity; the
rendering pins hold for the ray-by-ray form and the array form, which also
agree with each other on an uneven image."""
import math

import numpy as np
import pytest

from oracle import blob_field, render_blobs, render_blobs_all

FORMS = {"loop": render_blobs, "array": render_blobs_all}


def test_field_at_centre_and_one_radius():
    c, r, a, col = [[0.1, -0.2, 0.3]], [0.4], [7.0], [[0.2, 0.5, 0.9]]
    s, k = blob_field([[0.1, -0.2, 0.3], [0.5, -0.2, 0.3]], c, r, a, col)
    assert s[0] == 7.0
    assert abs(s[1] - 7.0 * math.exp(-0.5)) <= 1e-15 * 7.0
    np.testing.assert_allclose(k, [[0.2, 0.5, 0.9]] * 2, rtol=1e-15)


def test_colour_is_density_weighted():
    # two blobs, the point at distance 0 from the first and far from the second
    c = [[0, 0, 0], [1, 0, 0]]
    s, k = blob_field([[0.5, 0, 0]], c, [0.3, 0.3], [2.0, 6.0], [[1, 0, 0], [0, 0, 1]])
    g = math.exp(-0.25 / (2 * 0.09))
    assert abs(s[0] - 8.0 * g) <= 1e-14
    np.testing.assert_allclose(k[0], [0.25, 0.0, 0.75], rtol=1e-14)


def test_far_from_every_blob_is_empty_not_nan():
    s, k = blob_field([[1e3, 0, 0]], [[0, 0, 0]], [0.1], [5.0], [[1, 1, 1]])
    assert s[0] == 0.0 and np.all(k[0] == 0.0)


@pytest.mark.parametrize("form", FORMS)
def test_samples_are_taken_at_interval_midpoints(form):
    render_blobs = FORMS[form]
    # one sample [1, 3] on the x axis; the blob sits at x = 2 (the midpoint):
    # sigma = a there, so C = (1 - exp(-a dt)) col exactly
    a, dt = 0.3, 2.0
    C, A = render_blobs([0, 1], [[0, 0, 0]], [[1, 0, 0]], [1.0], [3.0], [[2, 0, 0]], [0.05], [a], [[0.4, 0.6, 0.8]])
    alpha = -math.expm1(-a * dt)
    assert abs(A[0] - alpha) <= 1e-15
    np.testing.assert_allclose(C[0], alpha * np.array([0.4, 0.6, 0.8]), rtol=1e-14)


@pytest.mark.parametrize("form", FORMS)
def test_constant_field_opacity(form):
    render_blobs = FORMS[form]
    # a blob far wider than the ray's span is constant (to 1e-12) along it:
    # A = 1 - exp(-a * sum dt), C = A col
    t = np.linspace(0.0, 1.0, 11)
    t0, t1 = t[:-1], t[1:]
    C, A = render_blobs([0, 10], [[0, 0, 0]], [[0, 0, 1]], t0, t1, [[0, 0, 0.5]], [1e6], [1.5], [[1, 0.5, 0.25]])
    want = -math.expm1(-1.5)
    assert abs(A[0] - want) <= 1e-10
    np.testing.assert_allclose(C[0], want * np.array([1, 0.5, 0.25]), rtol=1e-10)


@pytest.mark.parametrize("form", FORMS)
def test_empty_ray_is_zero(form):
    render_blobs = FORMS[form]
    C, A = render_blobs([0, 0], [[0, 0, 0]], [[1, 0, 0]], [], [], [[0, 0, 0]], [1.0], [1.0], [[1, 1, 1]])
    assert A[0] == 0.0 and np.all(C[0] == 0.0)


def test_forms_agree_on_an_image():
    rng = np.random.default_rng(23)
    n = 150
    counts = rng.integers(0, 60, size=n)
    counts[:10] = 0
    off = np.concatenate([[0], np.cumsum(counts)])
    S = int(off[-1])
    o = rng.uniform(-3, 3, (n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    t0 = np.concatenate([np.sort(rng.uniform(0.5, 6.0, c)) for c in counts])
    t1 = t0 + 0.01
    blobs = (rng.uniform(-1, 1, (5, 3)), rng.uniform(0.2, 0.8, 5), rng.uniform(1, 30, 5), rng.random((5, 3)))
    Ca, Aa = render_blobs(off, o, d, t0, t1, *blobs)
    Cb, Ab = render_blobs_all(off, o, d, t0, t1, *blobs, chunk=97)   # chunks that cut rays
    np.testing.assert_allclose(Cb, Ca, rtol=1e-11, atol=1e-15)
    np.testing.assert_allclose(Ab, Aa, rtol=1e-11, atol=1e-15)
    assert S > 97 and (Aa > 1e-3).any()
