"""Pins of the oracle's region contours simplified into polygons: closed forms
for rectangles, an L, a triangle and single pixels, the area of a disc's
polygon, the two degenerate tolerances, and that every vertex is a boundary
pixel of its region on random blobs."""
import math

import numpy as np
import pytest
from scipy import ndimage


@pytest.mark.parametrize("x0,y0,w,h", [(3, 2, 5, 4), (0, 0, 10, 8), (4, 1, 2, 2), (1, 5, 7, 1), (6, 0, 1, 6)])
def test_rectangle_gives_its_corners_clockwise(orc, x0, y0, w, h):
    r = np.full((8, 10), -1, np.int16)
    r[y0:y0 + h, x0:x0 + w] = 0
    poly = orc.region_polygons(r, 1, 0.5)[0].tolist()
    x1, y1 = x0 + w - 1, y0 + h - 1
    want = [[x0, y0], [x1, y0], [x1, y1], [x0, y1]]
    dedup = [p for i, p in enumerate(want) if p not in want[:i]]
    assert poly == dedup


def test_l_shape_and_its_cut_inner_corner(orc):
    r = np.full((9, 9), -1, np.int16)
    r[1:8, 1:4] = 0
    r[5:8, 1:8] = 0
    poly = orc.region_polygons(r, 1, 0.5)[0].tolist()
    # the 8-connected trace steps diagonally past the inner corner (3, 5)
    assert poly == [[1, 1], [3, 1], [3, 4], [4, 5], [7, 5], [7, 7], [1, 7]]


def test_triangle(orc):
    n = 12
    yy, xx = np.mgrid[0:n, 0:n]
    r = np.where(xx <= yy, 0, -1).astype(np.int16)
    poly = orc.region_polygons(r, 1, 1.0)[0].tolist()
    assert poly == [[0, 0], [n - 1, n - 1], [0, n - 1]]


def test_single_pixels_ring_and_empty_regions(orc):
    r = np.full((6, 7), -1, np.int16)
    r[1:5, 1:5] = 0
    r[2:4, 2:4] = -1      # a hole: only the outer boundary counts
    r[0, 6] = 2           # one pixel; region 1 has none
    polys = orc.region_polygons(r, 3, 0.5)
    assert polys[0].tolist() == [[1, 1], [4, 1], [4, 4], [1, 4]]
    assert polys[1].shape == (0, 2)
    assert polys[2].tolist() == [[6, 0]]


def test_tolerance_limits(orc):
    r = np.full((12, 12), -1, np.int16)
    yy, xx = np.mgrid[0:12, 0:12]
    r[(xx - 6) ** 2 + (yy - 6) ** 2 <= 20] = 0
    coarse = orc.region_polygons(r, 1, 1e9)[0]
    assert len(coarse) == 2  # only the first point and the one farthest from it
    fine = orc.region_polygons(r, 1, 0.0)[0]
    # eps = 0 keeps every point off the chord: no three consecutive kept vertices are collinear
    k = len(fine)
    for i in range(k):
        a, b, c = fine[i - 1], fine[i], fine[(i + 1) % k]
        assert (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]) != 0


def test_disc_polygon_area(orc):
    rad = 20
    yy, xx = np.mgrid[0:50, 0:50]
    r = np.where((xx - 25) ** 2 + (yy - 25) ** 2 <= rad * rad, 0, -1).astype(np.int16)
    p = orc.region_polygons(r, 1, 0.7)[0].astype(float)
    area = 0.5 * abs(np.dot(p[:, 0], np.roll(p[:, 1], -1)) - np.dot(p[:, 1], np.roll(p[:, 0], -1)))
    assert math.pi * (rad - 1.5) ** 2 < area < math.pi * rad ** 2
    assert 8 <= len(p) <= 60


@pytest.mark.parametrize("seed", [0, 1])
def test_vertices_are_boundary_pixels_of_their_region(orc, seed):
    rng = np.random.default_rng(seed)
    blob = ndimage.binary_opening(rng.random((40, 50)) < 0.6, iterations=1)
    lab, n = ndimage.label(blob, structure=[[0, 1, 0], [1, 1, 1], [0, 1, 0]])
    r = (lab - 1).astype(np.int16)
    polys = orc.region_polygons(r, n, 0.0)
    pad = np.pad(r, 1, constant_values=-1)
    for g in range(n):
        first = np.argwhere(r == g)[0]
        assert polys[g][0].tolist() == [first[1], first[0]]  # starts at the first pixel in row-major order
        for x, y in polys[g]:
            assert r[y, x] == g
            win = pad[y:y + 3, x:x + 3]
            assert (win != g).any() or len(polys[g]) == 1


def test_one_pixel_wide_shapes_close(orc):
    """Thin parts are walked out and back; the trace still closes."""
    r = np.full((8, 12), -1, np.int16)
    r[3, 2:10] = 0                      # a 1-pixel line
    assert orc.region_polygons(r, 1, 0.5)[0].tolist() == [[2, 3], [9, 3]]
    t = np.full((9, 9), -1, np.int16)
    t[1, 1:8] = 0                       # a T of 1-pixel strokes
    t[1:8, 4] = 0
    poly = orc.region_polygons(t, 1, 0.5)[0].tolist()
    assert poly == [[1, 1], [7, 1], [5, 1], [4, 2], [4, 7], [4, 2], [3, 1]]  # out and back along the stem
    blob = np.full((10, 10), -1, np.int16)
    blob[2:6, 2:6] = 0
    blob[5, 6:9] = 0                    # a spur off a square
    poly = orc.region_polygons(blob, 1, 0.5)[0].tolist()
    assert [8, 5] in poly and len(poly) <= 7
