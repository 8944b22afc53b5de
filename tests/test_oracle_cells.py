"""Cell counts of the oracle's walks, pinned to closed forms.

A walk over cells of edge D voxels, from the grid entry to the grid exit of a
ray that crosses no two planes at once, visits one cell more than the number
of planes at multiples of D strictly inside the grid that it crosses.  That
gives the count of every walk on grids built so that the cells are known:

* dense voxel DDA: every voxel crossed, D = 1, whatever the grid holds;
* hierarchical DDA (Sec. 2.3) on an all-empty or all-full grid: one root tile
  per root cell, D = 8 * 2^ilog2;
* sub-leaf steps (Fig. 1: empty space passed by powers of two) on a grid that
  is a checkerboard of 4^3 blocks: every leaf is mixed, but every 4^3 block is
  uniform, so D = 4; on checkerboards of single voxels or of 2^3 blocks no 4^3
  block is uniform, nothing merges and the count is the dense one.

Plus the ordering every grid must show: a sub-leaf walk visits no more cells
than the hierarchical one, which visits no more than the dense one.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle

STEP = oracle.make_step("const", dt=0.05)
TMAX = 1.0e6   # the walk runs to the grid exit


def crossings_inside(o, d, R, D, lo=-1.0, hi=1.0):
    """Planes at multiples of D voxels strictly inside the box [lo, hi]^3 that
    the ray crosses between its entry and exit, in float64, and the smallest
    gap between any two of the crossings (entry and exit included)."""
    o = np.asarray(o, np.float64)
    d = np.asarray(d, np.float64)
    h = (hi - lo) / R
    t_in, t_out = -np.inf, np.inf
    for a in range(3):
        if d[a] == 0.0:
            continue
        ta, tb = (lo - o[a]) / d[a], (hi - o[a]) / d[a]
        t_in, t_out = max(t_in, min(ta, tb)), min(t_out, max(ta, tb))
    ts = []
    for a in range(3):
        if d[a] == 0.0:
            continue
        for m in range(D, R, D):
            t = (lo + m * h - o[a]) / d[a]
            if t_in < t < t_out:
                ts.append(t)
    allt = np.sort(np.asarray(ts + [t_in, t_out]))
    gap = np.min(np.diff(allt)) if len(allt) > 1 else np.inf
    return len(ts), t_in, t_out, gap


def generic_rays(seed, n, R):
    """Rays from outside the box towards a random point inside it, kept only
    when they enter the box and no two crossings come within 1e-3 voxel."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        o = rng.uniform(-1, 1, 3)
        a = rng.integers(3)
        o[a] = rng.choice([-3.0, 3.0])
        d = rng.uniform(-1, 1, 3) - o
        d /= np.linalg.norm(d)
        o32, d32 = o.astype(np.float32), d.astype(np.float32)
        k, t_in, t_out, gap = crossings_inside(o32, d32, R, 1)
        if t_in < t_out and t_in > 0 and gap > 2.0 / R * 1e-3:
            out.append((o32, d32))
    return out


def cells(scene, rays, method, ilog2):
    o = np.stack([r[0] for r in rays])
    d = np.stack([r[1] for r in rays])
    return oracle.cell_counts(scene, o, d, 0.0, TMAX, STEP, method, ilog2=ilog2)


def expected(rays, R, D):
    return np.asarray([1 + crossings_inside(o, d, R, D)[0] for o, d in rays])


def box1():
    return np.asarray([[-1, -1, -1, 1, 1, 1]], np.float32)


@pytest.mark.parametrize("fill", [0, 1])
def test_dense_walk_counts_every_voxel(fill):
    R = 16
    occ = np.full((1, R, R, R), fill, np.uint8)
    occ[0, 3:9, 5:12, 2:7] ^= 1
    scene = oracle.Scene(occ, box1())
    rays = generic_rays(1, 60, R)
    for m in ("dense_branch", "dense_skip"):
        np.testing.assert_array_equal(cells(scene, rays, m, 1), expected(rays, R, 1), err_msg=m)


@pytest.mark.parametrize("fill", [0, 1])
@pytest.mark.parametrize("R,ilog2", [(16, 1), (32, 1), (64, 2), (64, 3)])
def test_uniform_grid_walks_root_tiles(fill, R, ilog2):
    occ = np.full((1, R, R, R), fill, np.uint8)
    scene = oracle.Scene(occ, box1())
    rays = generic_rays(2, 40, R)
    D = 8 << ilog2
    # the skip loop passes empty tiles one by one too: each is a cell it visits
    for m in ("hdda_branch", "hdda_skip", "subleaf_branch", "subleaf_skip"):
        np.testing.assert_array_equal(cells(scene, rays, m, ilog2), expected(rays, R, D), err_msg=m)


def checkerboard(R, e):
    i = np.arange(R) // e
    return ((i[:, None, None] + i[None, :, None] + i[None, None, :]) % 2).astype(np.uint8)[None]


@pytest.mark.parametrize("e", [1, 2, 4])
def test_subleaf_walk_on_block_checkerboards(e):
    R = 32
    scene = oracle.Scene(checkerboard(R, e), box1())
    rays = generic_rays(3 + e, 60, R)
    dense = expected(rays, R, 1)
    # every 8^3 block is mixed, so the hierarchical walk steps voxel by voxel
    np.testing.assert_array_equal(cells(scene, rays, "hdda_branch", 1), dense)
    np.testing.assert_array_equal(cells(scene, rays, "subleaf_branch", 1), expected(rays, R, 4 if e == 4 else 1))


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), R=st.sampled_from([8, 16, 24]), p=st.sampled_from([0.02, 0.2, 0.6, 0.95]),
       blocky=st.booleans(), ilog2=st.sampled_from([1, 2]))
def test_cell_counts_are_ordered(seed, R, p, blocky, ilog2):
    rng = np.random.default_rng(seed)
    if blocky:   # uniform 4^3 blocks, so sub-leaf steps have something to merge
        occ = np.repeat(np.repeat(np.repeat(rng.random((R // 4,) * 3) < p, 4, 0), 4, 1), 4, 2)
    else:
        occ = rng.random((R, R, R)) < p
    scene = oracle.Scene(occ.astype(np.uint8)[None], box1())
    n = 32
    o = rng.uniform(-3, 3, (n, 3)).astype(np.float32)
    d = (rng.uniform(-0.8, 0.8, (n, 3)) - o).astype(np.float32)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    c = {m: oracle.cell_counts(scene, o, d, 0.0, TMAX, STEP, m, ilog2=ilog2)
         for m in ("dense_branch", "hdda_branch", "subleaf_branch")}
    assert np.all(c["subleaf_branch"] <= c["hdda_branch"])
    assert np.all(c["hdda_branch"] <= c["dense_branch"])


def test_brute_force_has_no_cells():
    scene = oracle.Scene(np.zeros((1, 8, 8, 8), np.uint8), box1())
    with pytest.raises(ValueError):
        oracle.cell_counts(scene, np.zeros((1, 3), np.float32), np.ones((1, 3), np.float32), 0.0, 1.0, STEP, "brute")
