"""The oracle's seven ways of sampling reproduce hand-derived answers exactly.

The answers in tests/golden/handmade_cases.json were derived by hand from the
ownership rule (a voxel owns (entry, exit], the "<=" tests of Alg. 1), the
fixed or growing step (Sec. 3) and finest-cascade priority (Sec. 3); each case
carries its derivation.
"""
import numpy as np
import pytest

import oracle
from tests import handmade

DATA = handmade.load()
METHODS = ["brute", "dense_branch", "dense_skip", "hdda_branch", "hdda_skip", "subleaf_branch", "subleaf_skip"]


@pytest.mark.parametrize("case", DATA["cases"], ids=lambda c: c["name"])
@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("ilog2", [1, 3])
def test_handmade_samples(case, method, ilog2):
    occ, boxes = handmade.grid_of(case)
    scene = oracle.Scene(occ, boxes)
    t0, t1, vox = oracle.ray_samples(scene, case["o"], case["d"], case["tmin"], case["tmax"],
                                     handmade.step_of(case), method, ilog2=ilog2)
    np.testing.assert_array_equal(t0, np.asarray(case["t0"], np.float32))
    np.testing.assert_array_equal(t1, np.asarray(case["t1"], np.float32))
    np.testing.assert_array_equal(vox, np.asarray(case["vox"], np.int32))


@pytest.mark.parametrize("case", [c for c in DATA["cases"] if "vdb" in c] + DATA["vdb_cases"],
                         ids=lambda c: c["name"])
def test_handmade_vdb_structure(case):
    occ, boxes = handmade.grid_of(case)
    scene = oracle.Scene(occ, boxes)
    want = case.get("stats") or {k: v for k, v in case["vdb"].items() if k != "ilog2"}
    ilog2 = case.get("ilog2", case.get("vdb", {}).get("ilog2"))
    assert scene.vdb_stats(ilog2) == want


def test_lattice_pins():
    # constant step: t_n = fl(t_min + fl(n * dt)); with dt = 0.25 every value is exact
    lat = oracle.lattice(oracle.make_step("const", dt=0.25), 1.0, 8)
    np.testing.assert_array_equal(lat, 1.0 + 0.25 * np.arange(8, dtype=np.float32))
    # growing step worked by hand in case I
    lat = oracle.lattice(oracle.make_step("cone", cone=0.5, dt_min=0.25), 0.0, 10)
    np.testing.assert_array_equal(lat, np.asarray(
        [0, .25, .5, .75, 1.125, 1.6875, 2.53125, 3.796875, 5.6953125, 8.54296875], np.float32))


def test_lattice_is_index_defined_not_accumulated():
    # The constant-step lattice is defined by index, t_n = t_min + n*dt, each
    # in binary32.  Repeated addition drifts: pin that the oracle does not
    # accumulate, using numpy binary32 arithmetic (two roundings, no FMA).
    dt = np.float32(5e-3)
    tmin = np.float32(2.0)
    n = 801
    lat = oracle.lattice(oracle.make_step("const", dt=float(dt)), float(tmin), n)
    idx = (tmin + np.arange(n, dtype=np.float32) * dt).astype(np.float32)
    np.testing.assert_array_equal(lat, idx)
    acc = np.empty(n, np.float32)
    t = tmin
    for i in range(n):
        acc[i] = t
        t = np.float32(t + dt)
    assert np.max(np.abs(acc.astype(np.float64) - idx)) > 1e-5  # the drift the index form avoids


def test_planes_are_binary32_formula():
    # P(m) = fl(B + fl(m*h)), h = fl((A-B)/R); T(m) = fl(fl(P(m) - o) * fl(1/d)),
    # evaluated here in numpy binary32 for a box whose planes are NOT exact.
    box = np.asarray([-1.3, 0, 0, 1.7, 1, 1], np.float32)
    R = 7
    o, d = np.float32(-2.1), np.float32(0.37)
    P, T = oracle.planes(box, R, 0, float(o), float(d))
    h = np.float32(np.float32(box[3] - box[0]) / np.float32(R))
    m = np.arange(R + 1, dtype=np.float32)
    P_ref = (box[0] + (m * h).astype(np.float32)).astype(np.float32)
    r = np.float32(np.float32(1.0) / d)
    T_ref = ((P_ref - o).astype(np.float32) * r).astype(np.float32)
    np.testing.assert_array_equal(P, P_ref)
    np.testing.assert_array_equal(T, T_ref)
