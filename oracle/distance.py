"""Chessboard distances of an occupancy grid, the input of the distance-field
traversal (Sec. 2.3 and Fig. 1 describe it; the paper does not evaluate it).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Per level, every voxel's L-infinity (Chebyshev) distance in voxel indices to
the nearest occupied voxel of that level, 0 for an occupied voxel, capped at
`cap`; voxels outside the grid count as empty.
"""
import numpy as np
from scipy import ndimage


def chessboard_distance(occ, cap=16):
    """uint8 [L][R][R][R] of min(cap, distance) via scipy's chessboard chamfer transform."""
    occ = np.asarray(occ)
    out = np.empty(occ.shape, np.uint8)
    for lev in range(occ.shape[0]):
        if not occ[lev].any():
            out[lev] = cap
            continue
        d = ndimage.distance_transform_cdt(occ[lev] == 0, metric="chessboard")
        out[lev] = np.minimum(d, cap).astype(np.uint8)
    return out


def chessboard_distance_brute(occ, cap=16):
    """The definition written out (small grids only): a minimum over every
    occupied voxel of the largest per-axis index difference."""
    occ = np.asarray(occ)
    out = np.full(occ.shape, cap, np.uint8)
    L, R = occ.shape[0], occ.shape[1]
    for lev in range(L):
        pts = np.argwhere(occ[lev] != 0)
        if len(pts) == 0:
            continue
        for x in range(R):
            for y in range(R):
                for z in range(R):
                    d = np.abs(pts - np.array([x, y, z])).max(axis=1).min()
                    out[lev, x, y, z] = min(cap, int(d))
    return out
