"""Pins of the oracle's chessboard distances: scipy's transform against the
definition written out on small random grids (cap reached and not), a single
occupied voxel's closed form, and an empty level."""
import numpy as np
import pytest

from oracle import chessboard_distance, chessboard_distance_brute


@pytest.mark.parametrize("seed", range(4))
def test_transform_matches_the_definition(seed):
    rng = np.random.default_rng(900 + seed)
    R = [6, 9, 12, 20][seed]
    occ = (rng.random((2, R, R, R)) < [0.02, 0.1, 0.005, 0.01][seed]).astype(np.uint8)
    for cap in (3, 16):
        np.testing.assert_array_equal(chessboard_distance(occ, cap), chessboard_distance_brute(occ, cap))


def test_single_voxel_closed_form():
    R = 11
    occ = np.zeros((1, R, R, R), np.uint8)
    occ[0, 2, 7, 5] = 1
    i, j, k = np.meshgrid(np.arange(R), np.arange(R), np.arange(R), indexing="ij")
    want = np.minimum(np.maximum(np.maximum(np.abs(i - 2), np.abs(j - 7)), np.abs(k - 5)), 16)
    np.testing.assert_array_equal(chessboard_distance(occ)[0], want)


def test_empty_level_is_capped():
    occ = np.zeros((2, 8, 8, 8), np.uint8)
    occ[1, 0, 0, 0] = 1
    d = chessboard_distance(occ)
    assert np.all(d[0] == 16) and d[1, 7, 7, 7] == 7 and d[1, 0, 0, 0] == 0
