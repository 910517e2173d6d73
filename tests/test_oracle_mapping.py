"""Pins of the oracle's polygon map with vertical drift compensation (Eqs.
4-10): hulls against scipy, overlap areas against closed forms and
rasterisation, the filter's steady state against the closed-form root of its
Riccati fixed point and its limiting cases, the merge rules on hand-made
polygons, and drift tracking on a rendered staircase walk."""
import math

import numpy as np
import pytest
from scipy.spatial import ConvexHull

from oracle import mapping as M

UP = np.eye(3)  # camera frame = world frame (R = I, C = 0) for hand-made polygons


def _square(x0, y0, s, z, sup=100):
    v = np.array([[x0, y0, z], [x0 + s, y0, z], [x0 + s, y0 + s, z], [x0, y0 + s, z]], float)
    return (np.array([0.0, 0.0, 1.0]), -z, v.mean(axis=0), sup, v)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_hull_matches_scipy(seed):
    P = np.random.default_rng(seed).normal(size=(60, 2))
    h = M.convex_hull(P)
    ref = P[ConvexHull(P).vertices]
    assert {tuple(p) for p in h} == {tuple(p) for p in ref}
    assert M.area(h) == pytest.approx(ConvexHull(P).volume, rel=1e-12) and M.area(h) > 0  # counter-clockwise


def test_overlap_of_rectangles_is_the_closed_form():
    a = M.convex_hull(np.array([[0, 0], [4, 0], [4, 3], [0, 3]], float))
    b = M.convex_hull(np.array([[1, 1], [6, 1], [6, 5], [1, 5]], float))
    assert M.overlap_area(a, b) == pytest.approx(3 * 2)
    c = M.convex_hull(np.array([[4, 0], [5, 0], [5, 3], [4, 3]], float))
    assert M.overlap_area(a, c) == 0.0  # touching edges have no area


@pytest.mark.parametrize("seed", [0, 1])
def test_overlap_matches_rasterisation(seed):
    rng = np.random.default_rng(seed)
    a = M.convex_hull(rng.normal(0, 1, (12, 2)))
    b = M.convex_hull(rng.normal(0.5, 1, (12, 2)))
    g = np.linspace(-4, 4, 801)
    X, Y = np.meshgrid(g, g)
    pts = np.stack([X.ravel(), Y.ravel()], 1)

    def inside(h):
        m = np.ones(len(pts), bool)
        for i in range(len(h)):
            p, q = h[i], h[(i + 1) % len(h)]
            m &= (q[0] - p[0]) * (pts[:, 1] - p[1]) - (q[1] - p[1]) * (pts[:, 0] - p[0]) >= 0
        return m
    est = (inside(a) & inside(b)).sum() * (g[1] - g[0]) ** 2
    assert M.overlap_area(a, b) == pytest.approx(est, rel=0.02, abs=0.01)


def test_filter_steady_state_is_the_riccati_root():
    sp, sm = 2e-5, 3e-4
    m = M.DriftMap(sigma_p=sp, sigma_m=sm)
    # a map polygon of overwhelming support: merges leave its height where it is,
    # so every frame measures the same 2 cm
    m.integrate(UP, np.zeros(3), [_square(0, 0, 1, 0.3, sup=10 ** 15)])
    for _ in range(400):
        r = m.integrate(UP, np.zeros(3), [_square(0, 0, 1, 0.32, sup=1)])
    # fixed point of P = (1 - K)(P + sp), K = (P + sp)/(P + sp + sm): P^2 + sp P - sp sm = 0
    Pstar = (-sp + math.sqrt(sp * sp + 4 * sp * sm)) / 2
    assert r.variance == pytest.approx(Pstar, rel=1e-9)
    assert r.drift == pytest.approx(0.02, abs=1e-9) and r.measurement == pytest.approx(0.02, abs=1e-12)


def test_filter_limits():
    # one update after one prediction step
    sp, sm = 1e-4, 3e-4
    m = M.DriftMap(sigma_p=sp, sigma_m=sm)
    m.integrate(UP, np.zeros(3), [_square(0, 0, 1, 0.3)])
    r = m.integrate(UP, np.zeros(3), [_square(0, 0, 1, 0.34)])
    # the first frame (an empty map) only predicts: P = sp, then P_pred = 2 sp
    assert r.drift == pytest.approx(0.04 * 2 * sp / (2 * sp + sm), rel=1e-12)
    # prediction noise far above measurement noise: the estimate follows each measurement
    m = M.DriftMap(sigma_p=1e3, sigma_m=1e-9)
    m.integrate(UP, np.zeros(3), [_square(0, 0, 1, 0.3)])
    for dz in (0.01, 0.03, 0.02, -0.015):  # each within the tolerance of the corrected height
        r = m.integrate(UP, np.zeros(3), [_square(0.1, 0, 1, 0.3 + dz)])
        assert r.drift == pytest.approx(dz, abs=1e-9) and m.polys[0].height == pytest.approx(0.3, abs=1e-9)
    # no match: prediction only
    m = M.DriftMap(sigma_p=sp, sigma_m=sm)
    m.integrate(UP, np.zeros(3), [_square(0, 0, 1, 0.3)])
    r = m.integrate(UP, np.zeros(3), [_square(5, 5, 1, 0.3)])
    assert r.matched == 0 and r.drift == 0.0 and r.variance == pytest.approx(2 * sp) and math.isnan(r.measurement)


def test_merge_rules():
    m = M.DriftMap(sigma_p=0.0, sigma_m=1.0)  # K = 0: no drift correction
    r = m.integrate(UP, np.zeros(3), [_square(0, 0, 1, 0.30, 100), _square(3, 0, 1, 0.30, 100)])
    assert r.added == 2 and len(m.polys) == 2
    wall = (np.array([1.0, 0, 0]), -2.0, np.array([2.0, 0, 1]), 50, np.array([[2, 0, 0], [2, 1, 0], [2, 1, 2.0]]))
    r = m.integrate(UP, np.zeros(3), [_square(0.5, 0, 1, 0.34, 300),   # 4 cm above, overlapping: merged
                                      _square(3.5, 0, 1, 0.36, 100),   # 6 cm above: a new polygon
                                      _square(8.0, 0, 1, 0.30, 100),   # same height, no overlap: new
                                      wall])                           # not horizontal: skipped
    assert r.matched == 1 and r.added == 2 and r.skipped == 1 and r.match_of == [0, -1, -1, -2]
    p0 = m.polys[0]
    assert p0.support == 400 and p0.height == pytest.approx((0.30 * 100 + 0.34 * 300) / 400)
    assert M.area(p0.hull) == pytest.approx(1.5)  # the hull of the two unit squares
    assert len(m.polys) == 4


def test_drift_is_tracked_on_a_staircase_walk(orc):
    """Treads of the straight staircase seen from a random-walk camera whose
    reported height drifts by 1 cm a frame: the estimate follows the drift
    and the mapped tread heights stay at their true values."""
    import scenes
    from oracle.mapping import lift_polygon
    m = M.DriftMap(sigma_p=1e-4, sigma_m=1e-5)
    errs = []
    for k in range(12):
        f = scenes.make_frame(2, k, size=(320, 240))
        R, Cc = f.pose
        drift = 0.01 * k
        polys = []
        for g in range(len(f.gt_planes)):
            if (f.gt_labels == g).sum() < 400:
                continue
            xy = orc.region_polygons(np.where(f.gt_labels == g, 0, -1).astype(np.int16), 1, 1.0)[0]
            n, d = f.gt_planes[g][:3], f.gt_planes[g][3]
            verts = lift_polygon(xy, n, d, (f.K.fx, f.K.fy, f.K.cx, f.K.cy))
            polys.append((n, d, verts.mean(axis=0), int((f.gt_labels == g).sum()), verts))
        r = m.integrate(R, Cc + np.array([0, 0, drift]), polys)
        if k >= 3:
            errs.append(abs(r.drift - drift))
    assert max(errs) < 0.006
    treads = sorted({round(p.height, 2) for p in m.polys if p.support > 2000})
    true = {round(0.15 * i, 2) for i in range(0, 9)}
    assert all(min(abs(h - t) for t in true) < 0.01 for h in treads)
