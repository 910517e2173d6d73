"""Pins of the oracle's segmentation of the normal image (Canny edges, then
regions): closed forms at a step between two normals, one-pixel-wide
suppression, hysteresis and strict thresholds on hand-made magnitude images,
components against scipy's labelling, and regions that fall inside single
planes of a rendered scene."""
import numpy as np
import pytest
from scipy import ndimage

import scenes


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def _two_normals(W, H, inside, n1, n2):
    N = np.empty((3, H, W), np.float32)
    for c in range(3):
        N[c] = np.where(inside, n2[c], n1[c])
    return N, np.ones((H, W), np.uint8)


def test_gradient_at_a_vertical_step_is_the_closed_form(orc):
    W, H, c = 20, 9, 11
    n1, n2 = _unit([0, -1, -1]), _unit([0.3, -1, -0.2])
    u = np.arange(W)[None, :] * np.ones((H, 1), int)
    N, nv = _two_normals(W, H, u >= c, n1, n2)
    m2, sec, bar = orc.seg_grad(N, nv)
    d = N[:, 0, c].astype(np.float64) - N[:, 0, c - 1].astype(np.float64)
    want = 16.0 * (d @ d)  # Sobel sums 4 (n2 - n1) across the step, 0 along it
    inner = bar == 0
    assert (bar[0] == 1).all() and (bar[:, 0] == 1).all() and (bar[:, -1] == 1).all()
    for col in (c - 1, c):
        assert np.allclose(m2[1:-1, col], want, rtol=1e-6) and (sec[1:-1, col] == 0).all()
    others = inner.copy()
    others[:, c - 1:c + 1] = False
    assert (m2[others] == 0).all()


@pytest.mark.parametrize("kind,sector", [("rows", 2), ("diag", 3), ("anti", 1)])
def test_sector_follows_the_edge_orientation(orc, kind, sector):
    W = H = 24
    u = np.arange(W)[None, :] * np.ones((H, 1), int)
    v = np.arange(H)[:, None] * np.ones((1, W), int)
    inside = {"rows": v >= 12, "diag": u > v, "anti": u + v > 23}[kind]
    N, nv = _two_normals(W, H, inside, _unit([0, -1, -1]), _unit([0.4, -0.9, -0.3]))
    m2, sec, bar = orc.seg_grad(N, nv)
    top = m2 == m2[bar == 0].max()
    assert top.sum() >= 4 and (sec[top] == sector).all()


def test_nms_leaves_a_one_pixel_edge_and_two_regions(orc):
    W, H, c = 30, 12, 14
    u = np.arange(W)[None, :] * np.ones((H, 1), int)
    N, nv = _two_normals(W, H, u >= c, _unit([0, -1, -1]), _unit([0.5, -1, -0.2]))
    reg, n, edge = orc.segment(N, nv, 0.5, 1.0, 1, 10)
    assert np.array_equal(np.nonzero(edge.any(axis=0))[0], [c - 1])
    assert (edge[1:-1, c - 1] == 1).all()
    # regions: columns 1..c-3 and c+1..W-2 of rows 1..H-2 (the 1-pixel border is a
    # barrier; pixels next to the edge are dropped by the closing dilation)
    sizes = sorted([(c - 3) * (H - 2), (W - 2 - c) * (H - 2)], reverse=True)
    assert n == 2 and [(reg == k).sum() for k in range(2)] == sizes
    assert (reg[:, c - 2:c + 1] == -1).all() and (reg[0] == -1).all()


def _line_image(W=16, H=9):
    m2 = np.zeros((H, W), np.float32)
    sec = np.full((H, W), 2, np.uint8)  # gradients across rows: a row is a ridge
    return m2, sec, np.zeros((H, W), np.uint8)


def test_hysteresis_keeps_weak_pixels_connected_to_a_strong_one(orc):
    m2, sec, bar = _line_image()
    low, high = 1.0, 2.0
    m2[2, 2:12] = 2.0           # weak ridge ...
    m2[2, 12] = 5.0             # ... ending in a strong pixel
    m2[3, 1] = 2.0              # weak, touches the ridge diagonally
    m2[6, 3:9] = 2.0            # weak ridge with no strong pixel
    cls, edge = orc.seg_edges(m2, sec, bar, low, high)
    assert (cls[2, 2:12] == 1).all() and cls[2, 12] == 2
    want = np.zeros_like(edge)
    want[2, 2:13] = 1
    want[3, 1] = 1
    assert np.array_equal(edge, want)


def test_thresholds_are_strict(orc):
    m2, sec, bar = _line_image()
    low, high = 1.5, 2.5
    m2[2, 2] = np.float32(low) * np.float32(low)     # exactly low^2: not weak
    m2[4, 2] = np.float32(high) * np.float32(high)   # exactly high^2: weak, not strong
    m2[6, 2] = np.nextafter(np.float32(high) * np.float32(high), np.float32(np.inf))
    cls, _ = orc.seg_edges(m2, sec, bar, low, high)
    assert cls[2, 2] == 0 and cls[4, 2] == 1 and cls[6, 2] == 2


def test_nms_tie_rule(orc):
    """Equal magnitudes side by side along the gradient: only the first (the one
    with the equal neighbour ahead) survives."""
    m2, sec, bar = _line_image()
    sec[:] = 0
    m2[4, 5] = m2[4, 6] = 9.0
    cls, _ = orc.seg_edges(m2, sec, bar, 1.0, 2.0)
    assert cls[4, 5] == 2 and cls[4, 6] == 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_components_match_scipy_labelling(orc, seed):
    rng = np.random.default_rng(seed)
    mask = rng.random((37, 53)) < 0.55
    reg, n = orc.seg_regions(mask, 1, 1 << 15)
    lab, nl = ndimage.label(mask, structure=[[0, 1, 0], [1, 1, 1], [0, 1, 0]])
    assert n == nl
    sizes = np.bincount(lab.ravel())[1:]
    first = np.array([np.flatnonzero(lab.ravel() == k + 1)[0] for k in range(nl)])
    order = sorted(range(nl), key=lambda k: (-sizes[k], first[k]))
    for rank, k in enumerate(order):
        assert np.array_equal(reg == rank, lab == k + 1)
    reg2, n2 = orc.seg_regions(mask, 5, 3)
    keep = [k for k in order if sizes[k] >= 5][:3]
    assert n2 == len(keep)
    for rank, k in enumerate(keep):
        assert np.array_equal(reg2 == rank, lab == k + 1)
    assert ((reg2 >= 0) == np.isin(lab, [k + 1 for k in keep])).all()


def test_invalid_normals_make_barriers(orc):
    W, H = 12, 10
    N, nv = _two_normals(W, H, np.zeros((H, W), bool), _unit([0, -1, -1]), _unit([0, -1, -1]))
    nv[4, 6] = 0
    m2, sec, bar = orc.seg_grad(N, nv)
    assert (bar[3:6, 5:8] == 1).all() and bar[2, 6] == 0 and bar[4, 9] == 0
    reg, n, edge = orc.segment(N, nv, 0.5, 1.0, 1, 5)
    assert n == 1 and (reg[3:6, 5:8] == -1).all() and edge.sum() == 0


def test_regions_of_a_scene_lie_inside_single_planes(orc):
    f = scenes.make_frame(2, 0)
    P, valid = orc.backproject(f.depth_m * 1000.0, f.K)
    N, nvalid = orc.normals(P, valid)
    reg, n, edge = orc.segment(N.astype(np.float32), nvalid, 0.35, 0.7, 200, 127)
    assert n >= 8
    for k in range(n):
        gt = f.gt_labels[reg == k]
        top = np.bincount(gt[gt >= 0]).max() if (gt >= 0).any() else 0
        assert top >= 0.97 * gt.size, k


def test_impulse_response_shows_the_sobel_weights(orc):
    """One pixel with another normal d away: its 4-neighbours see one Sobel sum
    of 2 d (m2 = 4 |d|^2), its diagonal neighbours one 1 d in each direction
    (m2 = 2 |d|^2)."""
    W = H = 9
    n1, n2 = _unit([0, -1, -1]), _unit([0.6, -0.2, -1])
    inside = np.zeros((H, W), bool)
    inside[4, 4] = True
    N, nv = _two_normals(W, H, inside, n1, n2)
    m2, sec, bar = orc.seg_grad(N, nv)
    d = N[:, 4, 4].astype(np.float64) - N[:, 0, 0].astype(np.float64)
    dd = d @ d
    for (v, u) in ((3, 4), (5, 4), (4, 3), (4, 5)):
        assert m2[v, u] == pytest.approx(4 * dd, rel=1e-6)
    for (v, u) in ((3, 3), (3, 5), (5, 3), (5, 5)):
        assert m2[v, u] == pytest.approx(2 * dd, rel=1e-6)
    assert m2[4, 4] == 0.0 and sec[3, 4] == 2 and sec[4, 3] == 0 and sec[3, 3] == 1 and sec[3, 5] == 3
