"""Seeded input generators (CPU): the tiled camera order holds the same rays as the row-major
one, and each run of tile^2 rays is one square screen tile."""
import numpy as np

import nif_synth as S


def test_tiled_camera_rays_are_a_permutation_of_the_row_major_rays():
    res, tile = 64, 8
    o0, d0 = S.rays_camera(res, 30.0)
    o1, d1 = S.rays_camera(res, 30.0, tile=tile)
    assert o1.shape == o0.shape and d1.shape == d0.shape
    # pixel index of every tiled ray from the row-major direction it equals
    key0 = {tuple(np.round(d0[:, i], 6)): i for i in range(res * res)}
    pix = np.array([key0[tuple(np.round(d1[:, i], 6))] for i in range(res * res)])
    assert sorted(pix.tolist()) == list(range(res * res))
    np.testing.assert_array_equal(d1, d0[:, pix])
    np.testing.assert_array_equal(o1, o0[:, pix])
    px, py = pix % res, pix // res
    for b in range(0, res * res, tile * tile):
        x, y = px[b:b + tile * tile], py[b:b + tile * tile]
        assert x.max() - x.min() == tile - 1 and y.max() - y.min() == tile - 1
        assert x.min() % tile == 0 and y.min() % tile == 0
    # tiles are row-major: the first res / tile tiles cover the top tile row
    assert py[:res * tile].max() == tile - 1


def test_tiled_camera_subset_strides_the_tiled_order():
    o, d = S.rays_camera(32, 0.0, tile=8)
    o2, d2 = S.rays_camera(32, 0.0, tile=8, sub=5, sub_index=3)
    np.testing.assert_array_equal(d2, d[:, 3::5])
