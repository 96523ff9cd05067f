"""The geometry suite's seeded inputs (Sec. 5, App. F): shapes, phase ids,
the z-extrusions equal their 2D sections, non-overlapping spots, and the
Voronoi inclusion fraction at least Phi_vol = 0.9."""
import numpy as np
import pytest

import microstructures as M


@pytest.mark.parametrize("name", M.SUITE_2D)
def test_2d_geometries(name):
    g = M.geometry(name, 32, 2, seed=1)
    assert g.shape == (32, 32) and g.dtype == np.uint8 and set(np.unique(g)) <= {0, 1}
    assert np.array_equal(g, M.geometry(name, 32, 2, seed=1))     # seeded


@pytest.mark.parametrize("name,base", [("laminate3", "laminate"), ("pillar", "square"),
                                       ("circular_pillar", "circle"), ("fibres", "spots"),
                                       ("reduced_checkerboard", "checkerboard")])
def test_extrusions_are_their_sections(name, base):
    g3 = M.geometry(name, 16, 3, seed=2)
    g2 = M.geometry(base, 16, 2, seed=2)
    assert g3.shape == (16, 16, 16)
    assert all(np.array_equal(g3[:, :, k], g2) for k in range(16))


def test_same_from_every_direction():
    for name in ("box", "sphere", "checkerboard3"):
        g = M.geometry(name, 16, 3)
        assert np.array_equal(g, g.transpose(1, 2, 0)) and np.array_equal(g, g.transpose(2, 0, 1))


def test_spots_do_not_overlap_and_voronoi_fraction():
    g = M.geometry("spots", 256, 2, seed=3)
    # 10 discs of radius 0.08: area fraction 10 pi 0.08^2 up to pixelation
    assert abs(g.mean() - 10 * np.pi * 0.08 ** 2) < 0.01
    for dim, N in ((2, 64), (3, 16)):
        v = M.geometry("voronoi" if dim == 2 else "voronoi3", N, dim, seed=4)
        assert v.mean() >= 0.9 - 1e-12
