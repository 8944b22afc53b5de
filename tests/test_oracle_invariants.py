"""Properties the sampling rule fixes, checked on the oracle with random tiny inputs.

* Brute force, dense DDA (Alg. 1 branch / Alg. 2 skip), VDB + hierarchical
  DDA (branch / skip) and the same with uniform sub-blocks inside leaves give
  the identical sample list: they differ only in how empty space is skipped
  (Sec. 2.3, Fig. 1, Sec. 3).
* Occupancy enters point by point: S(G1 | G2) = S(G1) | S(G2),
  S(G1 & G2) = S(G1) & S(G2), S(~G) = S(full) - S(G).
* Exact symmetries: permuting the axes of grid and ray permutes voxel ids and
  keeps every t; mirroring a symmetric box with o, d -> -o, -d mirrors voxel
  ids and keeps every t.
* Geometry in float64: every sample point o + t*d lies in the (closed) voxel
  it names, that voxel is occupied and belongs to the finest cascade holding
  the point; every lattice point clearly inside an occupied voxel of its
  finest cascade is a sample, and no lattice point clearly elsewhere is.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle

METHODS = ["brute", "dense_branch", "dense_skip", "hdda_branch", "hdda_skip", "subleaf_branch", "subleaf_skip"]


def random_scene(rng, R, L, p):
    boxes = []
    half = 1.0
    for _ in range(L):
        boxes.append([-half, -half, -half, half, half, half])
        half *= 2.0
    occ = (rng.random((L, R, R, R)) < p).astype(np.uint8)
    return occ, np.asarray(boxes, np.float32)


def random_ray(rng, R, L, kind):
    span = 2.0 ** (L - 1)
    o = rng.uniform(-3 * span, 3 * span, 3)
    target = rng.uniform(-span, span, 3)
    d = target - o
    h = 2.0 / R
    if kind == "axis":           # parallel to an axis, possibly on a plane
        a = rng.integers(3)
        d = np.zeros(3)
        d[a] = rng.choice([-1.0, 1.0])
        o = np.round(rng.uniform(-span, span, 3) / h * 2) * h / 2
        o[a] = -d[a] * 3 * span
    elif kind == "diag":         # through lattice corners: ties on 2-3 axes
        d = rng.choice([-1.0, 1.0], 3) * rng.choice([0.0, 1.0, 1.0], 3)
        if not d.any():
            d[0] = 1.0
        o = -d * 3 * span + np.round(rng.uniform(-span, span, 3) / h) * h * (d == 0)
    elif kind == "inside":       # origin inside the grid
        o = rng.uniform(-span, span, 3)
    d = d / max(np.linalg.norm(d), 1e-12)
    return o.astype(np.float32), d.astype(np.float32)


def sample_set(t0, t1, vox):
    return set(zip(t0.tolist(), t1.tolist(), vox.tolist()))


def run_all(scene, o, d, tmin, tmax, step, ilog2):
    return {m: oracle.ray_samples(scene, o, d, tmin, tmax, step, m, ilog2=ilog2) for m in METHODS}


steps = st.sampled_from([
    oracle.make_step("const", dt=0.0625),
    oracle.make_step("const", dt=0.037),
    oracle.make_step("cone", cone=1 / 16, dt_min=0.02),
])


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), R=st.sampled_from([4, 8, 12, 16]), L=st.sampled_from([1, 2]),
       p=st.sampled_from([0.0, 0.05, 0.3, 0.7, 1.0]), kind=st.sampled_from(["free", "axis", "diag", "inside"]),
       step=steps, ilog2=st.sampled_from([1, 2, 3]))
def test_all_methods_identical(seed, R, L, p, kind, step, ilog2):
    rng = np.random.default_rng(seed)
    occ, boxes = random_scene(rng, R, L, p)
    scene = oracle.Scene(occ, boxes)
    o, d = random_ray(rng, R, L, kind)
    tmin = float(rng.choice([0.0, rng.uniform(0, 4)]))
    tmax = float(tmin + rng.uniform(0, 12))
    res = run_all(scene, o, d, tmin, tmax, step, ilog2)
    ref = res["brute"]
    for m, got in res.items():
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b, err_msg=m)


@settings(max_examples=100, deadline=None)
@given(seed=st.integers(0, 2**31 - 1), R=st.sampled_from([8, 16]), L=st.sampled_from([1, 2]),
       kind=st.sampled_from(["free", "axis", "diag", "inside"]), step=steps)
def test_union_intersection_complement(seed, R, L, kind, step):
    rng = np.random.default_rng(seed)
    g1, boxes = random_scene(rng, R, L, 0.3)
    g2, _ = random_scene(rng, R, L, 0.3)
    o, d = random_ray(rng, R, L, kind)
    tmin, tmax = 0.0, 16.0

    def S(g, method):
        return sample_set(*oracle.ray_samples(oracle.Scene(g, boxes), o, d, tmin, tmax, step, method, ilog2=1))

    for method in ["dense_branch", "hdda_skip"]:
        s1, s2 = S(g1, method), S(g2, method)
        assert S(g1 | g2, method) == s1 | s2
        assert S(g1 & g2, method) == s1 & s2
        full = S(np.ones_like(g1), method)
        assert S(1 - g1, method) == full - s1


def _perm_vox(vox, perm, R, inv=False):
    lev = vox // (R ** 3)
    r = vox % (R ** 3)
    ijk = np.stack([r // (R * R), (r // R) % R, r % R], 1)
    p = ijk[:, perm]
    return ((lev * R + p[:, 0]) * R + p[:, 1]) * R + p[:, 2]


@settings(max_examples=100, deadline=None)
@given(seed=st.integers(0, 2**31 - 1), R=st.sampled_from([8, 16]), L=st.sampled_from([1, 2]),
       kind=st.sampled_from(["free", "axis", "diag", "inside"]), step=steps,
       perm=st.permutations([0, 1, 2]))
def test_axis_permutation(seed, R, L, kind, step, perm):
    rng = np.random.default_rng(seed)
    occ, boxes = random_scene(rng, R, L, 0.3)
    o, d = random_ray(rng, R, L, kind)
    perm = list(perm)
    # new axis a is old axis perm[a]
    occ_p = np.ascontiguousarray(occ.transpose([0] + [1 + q for q in perm]))
    boxes_p = boxes[:, perm + [3 + q for q in perm]]
    for method in ["brute", "hdda_skip"]:
        t0, t1, vox = oracle.ray_samples(oracle.Scene(occ, boxes), o, d, 0.0, 16.0, step, method, ilog2=1)
        u0, u1, uvox = oracle.ray_samples(oracle.Scene(occ_p, boxes_p), o[perm], d[perm], 0.0, 16.0, step,
                                          method, ilog2=1)
        np.testing.assert_array_equal(t0, u0)
        np.testing.assert_array_equal(t1, u1)
        np.testing.assert_array_equal(_perm_vox(vox, perm, R), uvox)


@settings(max_examples=100, deadline=None)
@given(seed=st.integers(0, 2**31 - 1), R=st.sampled_from([8, 16]), L=st.sampled_from([1, 2]),
       step=steps, axes=st.lists(st.booleans(), min_size=3, max_size=3))
def test_mirror_symmetry(seed, R, L, step, axes):
    # Boxes [-2^k, 2^k] with R a power of two have planes P(R-m) = -P(m)
    # exactly, so T'(m) = T(R-m) bit for bit after o_a, d_a -> -o_a, -d_a.
    rng = np.random.default_rng(seed)
    occ, boxes = random_scene(rng, R, L, 0.3)
    o, d = random_ray(rng, R, L, "free")
    flip = np.asarray(axes)
    o2 = np.where(flip, -o, o).astype(np.float32)
    d2 = np.where(flip, -d, d).astype(np.float32)
    occ2 = occ
    for a in range(3):
        if flip[a]:
            occ2 = np.flip(occ2, axis=1 + a)
    occ2 = np.ascontiguousarray(occ2)
    t0, t1, vox = oracle.ray_samples(oracle.Scene(occ, boxes), o, d, 0.0, 16.0, step, "hdda_skip", ilog2=1)
    u0, u1, uvox = oracle.ray_samples(oracle.Scene(occ2, boxes), o2, d2, 0.0, 16.0, step, "hdda_skip", ilog2=1)
    np.testing.assert_array_equal(t0, u0)
    np.testing.assert_array_equal(t1, u1)
    lev = vox // R ** 3
    r = vox % R ** 3
    ijk = np.stack([r // (R * R), (r // R) % R, r % R], 1)
    ijk = np.where(flip, R - 1 - ijk, ijk)
    np.testing.assert_array_equal(((lev * R + ijk[:, 0]) * R + ijk[:, 1]) * R + ijk[:, 2], uvox)


def _finest_level(p, boxes, margin):
    """Finest level whose box holds p with `margin` to spare, or None if the
    point is within `margin` of some box face (ambiguous) or outside all."""
    for lev, b in enumerate(boxes):
        lo, hi = b[:3].astype(np.float64), b[3:].astype(np.float64)
        dist = np.minimum(p - lo, hi - p)
        if np.all(dist > margin):
            return lev
        if np.all(dist > -margin):
            return None
    return -1


@settings(max_examples=150, deadline=None)
@given(seed=st.integers(0, 2**31 - 1), R=st.sampled_from([8, 16]), L=st.sampled_from([1, 2, 3]),
       p=st.sampled_from([0.1, 0.5]), step=steps, kind=st.sampled_from(["free", "inside"]))
def test_geometric_containment(seed, R, L, p, step, kind):
    rng = np.random.default_rng(seed)
    occ, boxes = random_scene(rng, R, L, p)
    scene = oracle.Scene(occ, boxes)
    o, d = random_ray(rng, R, L, kind)
    tmin, tmax = 0.0, 20.0
    t0, t1, vox = oracle.ray_samples(scene, o, d, tmin, tmax, step, "hdda_skip", ilog2=1)
    o64, d64 = o.astype(np.float64), d.astype(np.float64)
    emitted = {}
    for t, v in zip(t0.tolist(), vox.tolist()):
        lev = v // R ** 3
        r = v % R ** 3
        ijk = np.array([r // (R * R), (r // R) % R, r % R])
        h = (boxes[lev, 3:] - boxes[lev, :3]).astype(np.float64) / R
        lo = boxes[lev, :3] + ijk * h
        pt = o64 + t * d64
        tol = 1e-4 * h + 1e-6 * (1 + abs(t))
        assert np.all(pt >= lo - tol) and np.all(pt <= lo + h + tol), (t, v, pt, lo)
        assert occ[lev, ijk[0], ijk[1], ijk[2]]
        emitted[t] = v
    # every clearly-placed lattice point: emitted iff its voxel is occupied
    lat = oracle.lattice(step, tmin, 4000)
    lat = lat[lat <= tmax]
    for t in lat.tolist():
        pt = o64 + t * d64
        h_f = (boxes[0, 3:] - boxes[0, :3]).astype(np.float64) / R
        lev = _finest_level(pt, boxes, 1e-3 * h_f.min())
        if lev is None:
            continue
        if lev < 0:
            assert t not in emitted
            continue
        h = (boxes[lev, 3:] - boxes[lev, :3]).astype(np.float64) / R
        u = (pt - boxes[lev, :3]) / h
        ijk = np.floor(u).astype(int)
        if np.any(np.abs(u - np.round(u)) < 1e-3):
            continue  # within a hair of a face: the binary32 rule decides
        want = bool(occ[lev, ijk[0], ijk[1], ijk[2]])
        assert (t in emitted) == want, (t, lev, ijk)
        if want:
            assert emitted[t] == ((lev * R + ijk[0]) * R + ijk[1]) * R + ijk[2]


@pytest.mark.parametrize("bad", [
    ([np.nan, 0, 0], [1, 0, 0]), ([0, 0, 0], [np.inf, 0, 0]), ([np.inf, 0, 0], [1, 0, 0])])
def test_nonfinite_rays_have_no_samples(bad):
    occ = np.ones((1, 8, 8, 8), np.uint8)
    scene = oracle.Scene(occ, [[-1, -1, -1, 1, 1, 1]])
    for m in METHODS:
        t0, _, _ = oracle.ray_samples(scene, bad[0], bad[1], 0.0, 10.0, oracle.make_step("const", dt=0.1), m)
        assert t0.size == 0


def test_tmin_after_tmax_has_no_samples():
    occ = np.ones((1, 8, 8, 8), np.uint8)
    scene = oracle.Scene(occ, [[-1, -1, -1, 1, 1, 1]])
    for m in METHODS:
        t0, _, _ = oracle.ray_samples(scene, [-2, 0.1, 0.1], [1, 0, 0], 3.0, 2.0,
                                      oracle.make_step("const", dt=0.1), m)
        assert t0.size == 0


def test_denormal_and_negative_zero_directions():
    # -0.0 and a denormal whose reciprocal overflows are zero axes; a denormal
    # with a finite reciprocal is not.  All methods agree with brute force.
    occ = (np.random.default_rng(5).random((1, 8, 8, 8)) < 0.5).astype(np.uint8)
    scene = oracle.Scene(occ, [[-1, -1, -1, 1, 1, 1]])
    step = oracle.make_step("const", dt=0.03)
    for d in ([1.0, -0.0, 0.0], [1.0, 1e-45, -0.0], [0.7, 2e-38, 1e-39], [-0.5, -1e-40, 0.3]):
        res = run_all(scene, [-2.0, 0.13, -0.41], d, 0.0, 10.0, step, 1)
        for m in METHODS:
            for a, b in zip(res[m], res["brute"]):
                np.testing.assert_array_equal(a, b, err_msg=f"{m} {d}")
