"""Pins of the oracle's region-mode RANSAC (Alg. 2 as printed: per region, the
model with the smallest summed distance, stored iff more than 90 % of the
region's points are inliers): exact recovery of noise-free regions, an
independent numpy re-derivation of every draw and score, the strict ratio
rule, and the small and degenerate regions."""
import math

import numpy as np
import pytest

import oracle as O
from test_oracle_ransac import _numpy_philox_block, _plane_numpy

def _plane_depth(W, H, K, planes, region):
    """Depth (m) of pixel rays hitting plane region[v,u] (n.p + d = 0)."""
    fx, fy, cx, cy = K
    u, v = np.meshgrid(np.arange(W), np.arange(H))
    ray = np.stack([(u - cx) / fx, (v - cy) / fy, np.ones_like(u, dtype=float)])
    z = np.zeros((H, W))
    for g, (n, d) in enumerate(planes):
        m = region == g
        z[m] = -d / np.tensordot(n, ray, axes=1)[m]
    return z


def _points_from_depth_m(z, K):
    fx, fy, cx, cy = K
    H, W = z.shape
    u, v = np.meshgrid(np.arange(W), np.arange(H))
    P = np.stack([z * (u - cx) / fx, z * (v - cy) / fy, z])
    return P, (z > 0).astype(np.uint8)


def _prm(hyps, seed=7, frame=3, t=0.01):
    return O.RansacParams(hyps=hyps, max_planes=1, min_inliers=1, thresh=t, seed=seed, frame=frame)


def test_noise_free_regions_are_each_stored_exactly(orc):
    W, H, Kp = 48, 36, (40.0, 40.0, 24.0, 18.0)
    region = np.full((H, W), -1, np.int16)
    region[:, :16] = 0
    region[:, 16:32] = 1
    region[:20, 32:] = 2
    planes = [(np.array([0.0, -0.8, -0.6]), 1.2), (np.array([0.0, 0.0, -1.0]), 2.0), (np.array([0.6, 0.0, -0.8]), 1.5)]
    z = _plane_depth(W, H, Kp, planes, region)
    z[region < 0] = 1.0  # points outside every region do not count
    P, valid = _points_from_depth_m(z, Kp)
    res = orc.ransac_regions(P, valid, region, 3, _prm(16))
    assert res.n_stored == 3 and res.stored.all()
    for g, (n, d) in enumerate(planes):
        want = np.append(-n, -d) if d < 0 else np.append(n, d)
        assert np.max(np.abs(res.planes[g, res.jstar[g]] - want)) < 1e-9
        m = region == g
        assert res.npts[g] == m.sum()
        assert res.counts[g, res.jstar[g]] == m.sum()
        assert np.max(np.abs(res.centroids[g] - P[:, m].mean(axis=1))) < 1e-12
    assert np.array_equal(res.labels, np.where(region >= 0, region, -1).astype(np.int8))


def _numpy_regions(P, valid, region, R, hyps, seed, frame, t):
    """Alg. 2 per region, written again with numpy's Philox and numpy sums."""
    H, W = region.shape
    flat_r = region.reshape(-1)
    flat_v = valid.reshape(-1)
    pts = P.reshape(3, -1)
    out = []
    for g in range(R):
        lst = np.nonzero((flat_v & 1).astype(bool) & (flat_r == g))[0]
        m = len(lst)
        hyp = []
        for j in range(hyps):
            got = []
            for b in range(16):
                if len(got) == 3 or m == 0:
                    break
                for w in _numpy_philox_block([j, g, b, 1], [seed, frame]):
                    k = (w * m) >> 64
                    if k not in got:
                        got.append(k)
                    if len(got) == 3:
                        break
            pl = None
            if len(got) == 3:
                pl = _plane_numpy(*(pts[:, lst[k]] for k in got))
            if pl is None:
                hyp.append((got if len(got) == 3 else None, None, math.inf, 0))
                continue
            dist = np.abs(pl[:3] @ pts[:, lst] + pl[3])
            hyp.append((got, pl, float(dist.sum()), int((dist < t).sum())))
        errs = [h[2] for h in hyp]
        js = int(np.argmin(errs)) if any(h[1] is not None for h in hyp) else -1
        stored = js >= 0 and hyp[js][3] / m > 0.9
        out.append((lst, hyp, js, stored))
    return out


def _check_against_rederivation(orc, seed):
    rng = np.random.default_rng(seed)
    W, H, R, hyps, t = 24, 18, 4, 12, 0.01
    Kp = (20.0, 20.0, 12.0, 9.0)
    region = rng.integers(-1, R + 1, size=(H, W)).astype(np.int16)  # includes -1 and an out-of-range label R
    region[:, :6] = 0  # a large region
    planes = [(np.array([0.0, -0.6, -0.8]), 1.0), (np.array([0.0, 0.0, -1.0]), 1.5),
              (np.array([0.3, 0.0, -0.954]), 1.2), (np.array([0.0, 0.5, -0.866]), 2.0)]
    z = _plane_depth(W, H, Kp, planes, np.clip(region, 0, R - 1))
    z += rng.normal(0, 0.006, z.shape) * (rng.random(z.shape) < 0.9) + rng.normal(0, 0.05, z.shape) * (
        rng.random(z.shape) < 0.1)
    z[rng.random(z.shape) < 0.05] = 0.0
    P, valid = _points_from_depth_m(z, Kp)
    res = orc.ransac_regions(P, valid, region, R, _prm(hyps, seed=seed, t=t))
    ref = _numpy_regions(P, valid, region, R, hyps, seed, 3, t)
    differ = 0
    for g, (lst, hyp, js, stored) in enumerate(ref):
        assert res.npts[g] == len(lst)
        for j, (got, pl, err, cnt) in enumerate(hyp):
            if got is None:
                assert list(res.triples[g, j]) == [-1, -1, -1]
            else:
                assert list(res.triples[g, j]) == got
            assert res.hvalid[g, j] == (pl is not None)
            if pl is not None:
                assert np.max(np.abs(res.planes[g, j] - pl)) < 1e-12
                assert res.errors[g, j] == pytest.approx(err, rel=1e-12)
                assert res.counts[g, j] == cnt
        assert res.jstar[g] == js and res.stored[g] == stored
        cnts = [h[3] for h in hyp]
        differ += js >= 0 and int(np.argmax(cnts)) != js
    # labels: inliers of the stored regions
    lab = np.full((H, W), -1, np.int8)
    for g, (lst, hyp, js, stored) in enumerate(ref):
        if stored:
            pl = hyp[js][1]
            for px in lst:
                p = P.reshape(3, -1)[:, px]
                if abs(pl[:3] @ p + pl[3]) < t:
                    lab.reshape(-1)[px] = g
    assert np.array_equal(res.labels, lab)
    assert res.n_stored == sum(r[3] for r in ref)
    return differ


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_regions_match_an_independent_rederivation(orc, seed):
    _check_against_rederivation(orc, seed)


def test_selection_is_the_smallest_error_not_the_most_inliers(orc):
    """Over these draws, some region's smallest-error model is not its
    most-inlier model: the pin above separates the two criteria."""
    assert sum(_check_against_rederivation(orc, s) for s in (1, 2, 3, 4, 5)) > 0


def _ratio_region(n_on):
    """A region of n_on points on z = 1 m (spread out) plus one point 0.5 m off."""
    W, H = 8, 8
    Kp = (10.0, 10.0, 4.0, 4.0)
    region = np.full((H, W), -1, np.int16)
    on = [(1, 1), (1, 4), (1, 6), (4, 1), (4, 6), (6, 1), (6, 4), (6, 6), (3, 3), (2, 5), (5, 2)][:n_on]
    z = np.zeros((H, W))
    for (v, u) in on:
        region[v, u] = 0
        z[v, u] = 1.0
    region[4, 4] = 0
    z[4, 4] = 1.5
    return _points_from_depth_m(z, Kp) + (region,)


@pytest.mark.parametrize("n_on,want", [(9, False), (10, True)])
def test_ratio_rule_is_strict(orc, n_on, want):
    P, valid, region = _ratio_region(n_on)
    res = orc.ransac_regions(P, valid, region, 1, _prm(64))
    js = res.jstar[0]
    assert np.max(np.abs(res.planes[0, js] - [0, 0, -1, 1])) < 1e-12  # the z = 1 plane wins
    assert res.counts[0, js] == n_on and res.npts[0] == n_on + 1
    assert bool(res.stored[0]) == want  # 9/10 is not > 0.9; 10/11 is
    if want:  # the centroid is the mean of the inliers only, without the outlier
        on = (region == 0) & (res.labels == 0)
        assert on.sum() == n_on
        assert np.max(np.abs(res.centroids[0] - P[:, on].mean(axis=1))) < 1e-12


def test_small_and_empty_regions_store_nothing(orc):
    W, H = 10, 6
    Kp = (10.0, 10.0, 5.0, 3.0)
    z = np.ones((H, W))
    region = np.full((H, W), -1, np.int16)
    region[0, 0] = 1          # 1 point
    region[1, 1:3] = 2        # 2 points
    region[2, 0:4] = 3        # 4 collinear points: no plane
    region[3, 3] = 2
    z[3, 3] = 0.0             # a hole: not a point of region 2
    P, valid = _points_from_depth_m(z, Kp)
    res = orc.ransac_regions(P, valid, region, 4, _prm(8))
    assert list(res.npts) == [0, 1, 2, 4]
    assert res.n_stored == 0 and not res.stored.any()
    assert list(res.jstar) == [-1, -1, -1, -1]
    assert (res.triples[:3] == -1).all()
    assert not res.hvalid.any() and np.isinf(res.errors).all()
    assert (res.labels == -1).all()


def test_equal_errors_keep_the_first_hypothesis(orc):
    """Points on z = 1 with dyadic coordinates: every non-degenerate triple gives
    exactly n = (0, 0, -1), d = 1 and error 0, so the first valid hypothesis wins."""
    W, H = 8, 8
    Kp = (8.0, 8.0, 4.0, 4.0)
    region = np.zeros((H, W), np.int16)
    P, valid = _points_from_depth_m(np.ones((H, W)), Kp)
    res = orc.ransac_regions(P, valid, region, 1, _prm(24))
    assert (res.errors[0][res.hvalid[0]] == 0.0).all() and res.hvalid[0].sum() > 2
    assert res.jstar[0] == int(np.argmax(res.hvalid[0]))
    assert list(res.planes[0, res.jstar[0]]) == [0.0, 0.0, -1.0, 1.0]


def test_threshold_is_strict_at_an_exact_distance(orc):
    """Nine points on z = 1 and two at z = 1.25 with t = 0.25: the two lie at
    exactly t and are not inliers."""
    W, H = 8, 8
    Kp = (8.0, 8.0, 4.0, 4.0)
    region = np.full((H, W), -1, np.int16)
    z = np.zeros((H, W))
    for (v, u) in [(1, 1), (1, 4), (1, 6), (4, 1), (4, 6), (6, 1), (6, 4), (6, 6), (3, 3)]:
        region[v, u], z[v, u] = 0, 1.0
    for (v, u) in [(2, 5), (5, 2)]:
        region[v, u], z[v, u] = 0, 1.25
    P, valid = _points_from_depth_m(z, Kp)
    res = orc.ransac_regions(P, valid, region, 1, _prm(64, t=0.25))
    js = res.jstar[0]
    assert list(res.planes[0, js]) == [0.0, 0.0, -1.0, 1.0]
    assert res.counts[0, js] == 9 and res.errors[0, js] == 0.5


@pytest.mark.parametrize("delta,valid_plane", [(1e-3, False), (4e-3, True)])
def test_degeneracy_threshold(orc, delta, valid_plane):
    """A three-point region (0,0,1), (1,0,1), (2,delta,1): |e1 x e2| / (|e1||e2|)
    is about delta / 2, against the 1e-3 cut."""
    P = np.zeros((3, 1, 3))
    P[:, 0, 0] = (0.0, 0.0, 1.0)
    P[:, 0, 1] = (1.0, 0.0, 1.0)
    P[:, 0, 2] = (2.0, delta, 1.0)
    valid = np.ones((1, 3), np.uint8)
    res = orc.ransac_regions(P, valid, np.zeros((1, 3), np.int16), 1, _prm(4))
    assert res.hvalid[0].all() == valid_plane and res.hvalid[0].any() == valid_plane
    assert (res.jstar[0] >= 0) == valid_plane
