"""Pins of the selector-feature reference on hand-derived values."""
import math

import numpy as np

import graphgen as gg
from oracle import features


def test_path_features_by_hand():
    # path 0-1-2-3 (symmetric): out/in-degrees 1,2,2,1; nnz 6;
    # ld = floor(log2(1+d)) = 1,1,1,1 -> graph mean 1, variance 0.
    g = gg.from_edge_list(4, [(0, 1), (1, 2), (2, 3)], True)
    f = features.level_features(g.row_ptr, g.csc_ptr, np.array([0, 1, 2, 3]))
    exp = np.array([
        [1, 1, 2, math.log2(6), .25, 1 / 6, .75, 1, 0, 1, 0, 0],
        [1, math.log2(3), math.log2(3), 2, .25, 2 / 6, .5, 1, 0, 1, 0, 1],
        [1, math.log2(3), 1, 1, .25, 2 / 6, .25, 1, 0, 1, 0, math.log2(3)],
        [1, 1, 0, 0, .25, 1 / 6, 0, 1, 0, 1, 0, 2],
    ], dtype=np.float64).astype(np.float32)
    np.testing.assert_array_equal(f, exp)


def test_star_variance_by_hand():
    # star with centre 0 and 4 leaves: ld(centre) = floor(log2 5) = 2, leaves 1;
    # graph mean 6/5, mean of squares 8/5 -> variance 8/5 - 36/25 = 4/25.
    g = gg.from_edge_list(5, [(0, i) for i in range(1, 5)], True)
    f = features.level_features(g.row_ptr, g.csc_ptr, np.array([1, 2, 0, 2, 2]))
    assert f.shape == (3, 12)
    np.testing.assert_array_equal(f[:, 9], np.float32(6 / 5))
    np.testing.assert_array_equal(f[:, 10], np.float32(8 / 5 - 36 / 25))
    # level 1 frontier = {centre}: mean 2, variance 0; level 2 = three leaves
    assert f[1, 7] == 2 and f[1, 8] == 0
    assert f[2, 7] == 1 and f[2, 8] == 0
    # unvisited after level 1: the three leaves other than the source
    assert f[1, 6] == np.float32(3 / 5)


def test_floor_log2_is_exact_at_powers_of_two():
    # out-degrees 3 and 7 make 1+d a power of two: ld must be exactly 2 and 3
    edges = [(0, i) for i in range(1, 4)] + [(4, i) for i in range(5, 12)]
    g = gg.from_edge_list(12, edges, False)
    lv = np.full(12, -1)
    lv[0] = 0
    lv[1:4] = 1
    f = features.level_features(g.row_ptr, g.csc_ptr, lv)
    assert f[0, 7] == 2.0
