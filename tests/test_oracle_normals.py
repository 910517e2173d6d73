"""Pins of the oracle's back-projection (Alg. 2) and normal image (Eq. 2,
Alg. 1): points land on the scene generator's ray-cast planes, Sobel normals
of analytic planes are exact, validity rules, mirror symmetry."""
import numpy as np
import pytest

import scenes


def _float_depth_mm(frame):
    return frame.depth_m * 1000.0


@pytest.mark.parametrize("cid,k", [(1, 0), (2, 0), (3, 1)])
def test_backprojected_points_lie_on_the_ray_cast_planes(orc, cid, k):
    f = scenes.make_frame(cid, k, noise="none", hole_frac=0.0)
    P, valid = orc.backproject(_float_depth_mm(f), f.K)
    lab = f.gt_labels
    npl = len(f.gt_planes)
    m = (lab >= 0) & (lab < npl)
    assert m.sum() > 1000
    n = f.gt_planes[lab[m], :3]
    d = f.gt_planes[lab[m], 3]
    pts = P[:, m].T
    r = np.einsum("ij,ij->i", n, pts) + d
    assert np.max(np.abs(r)) < 1e-12 * 10
    assert np.array_equal(valid.astype(bool), f.depth_m > 0)


def test_backprojection_closed_form_on_the_principal_axis(orc):
    K = scenes.Intrinsics(100.0, 120.0, 3.0, 2.0)
    d = np.full((5, 7), 2500.0)
    d[0, 0] = 0.0
    P, valid = orc.backproject(d, K)
    assert P[0, 2, 3] == 0.0 and P[1, 2, 3] == 0.0 and P[2, 2, 3] == 2.5
    assert P[0, 2, 4] == pytest.approx(2.5 / 100.0)
    assert P[1, 3, 3] == pytest.approx(2.5 / 120.0)
    assert valid[0, 0] == 0 and np.all(P[:, 0, 0] == 0.0)


@pytest.mark.parametrize("cid,k", [(1, 0), (2, 0), (2, 2), (3, 2)])
def test_normals_of_analytic_planes_are_exact(orc, cid, k):
    """Each Sobel sum is a weighted sum of chords with weights summing to zero,
    so for points on one plane Gx and Gy lie in the plane and their cross
    product is the plane normal exactly; the minus sign makes it face the camera."""
    f = scenes.make_frame(cid, k, noise="none", hole_frac=0.0)
    P, valid = orc.backproject(_float_depth_mm(f), f.K)
    N, nv = orc.normals(P, valid)
    lab = f.gt_labels
    H, W = lab.shape
    same = np.zeros((H, W), bool)
    same[1:-1, 1:-1] = True
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            same[1:-1, 1:-1] &= lab[1 + dj:H - 1 + dj, 1 + di:W - 1 + di] == lab[1:-1, 1:-1]
    same &= (lab >= 0) & (lab < len(f.gt_planes))
    assert same.sum() > 1000
    assert np.all(nv[same] == 1)
    gt = f.gt_planes[lab[same], :3]
    got = N[:, same].T
    cosang = np.clip(np.einsum("ij,ij->i", gt, got), -1, 1)
    ang = np.arccos(cosang)
    assert np.max(ang) < 1e-7  # arccos near 1 amplifies rounding; 1e-7 rad ~ 1e-14 in cos
    assert np.max(np.abs(got - gt)) < 1e-10
    # camera-facing: n . P < 0
    assert np.all(np.einsum("ij,ji->i", got, P[:, same]) < 0)


def test_sobel_weights_on_a_fronto_parallel_plane(orc):
    """On z = const the point image is linear in (u, v), so the 3x3 Sobel sums
    are 8 times the per-pixel steps: Gx = (8z/fx, 0, 0), Gy = (0, 8z/fy, 0)."""
    K = scenes.Intrinsics(90.0, 110.0, 6.5, 4.0)
    d = np.full((9, 12), 1800.0)
    P, valid = orc.backproject(d, K)
    N, nv, gx, gy = orc.normals(P, valid, with_grad=True)
    z = 1.8
    inner = (slice(1, -1), slice(1, -1))
    assert np.allclose(gx[0][inner], 8 * z / K.fx, atol=1e-14, rtol=0)
    assert np.allclose(gx[1][inner], 0.0, atol=1e-14) and np.allclose(gx[2][inner], 0.0, atol=1e-14)
    assert np.allclose(gy[1][inner], 8 * z / K.fy, atol=1e-14, rtol=0)
    assert np.allclose(gy[0][inner], 0.0, atol=1e-14) and np.allclose(gy[2][inner], 0.0, atol=1e-14)
    assert np.allclose(N[2][inner], -1.0, atol=1e-15)


def test_sobel_smoothing_weights_on_a_bilinear_surface(orc):
    """For a component equal to u*v the Sobel x sum is 2 (1 (v-1) + 2 v + (v+1)) = 8 v
    (the 1-2-1 smoothing across rows), and the y sum is 8 u."""
    H, W = 6, 7
    v, u = np.mgrid[0:H, 0:W].astype(float)
    P = np.stack([u * v, u + 2 * v, np.full((H, W), 3.0)])
    valid = np.ones((H, W), np.uint8)
    _, _, gx, gy = orc.normals(P, valid, with_grad=True)
    inner = (slice(1, -1), slice(1, -1))
    assert np.allclose(gx[0][inner], 8 * v[inner], atol=1e-12)
    assert np.allclose(gy[0][inner], 8 * u[inner], atol=1e-12)
    assert np.allclose(gx[1][inner], 8.0, atol=1e-12) and np.allclose(gy[1][inner], 16.0, atol=1e-12)


def test_normal_validity_rules(orc):
    f = scenes.make_frame(1, 0)
    P, valid = orc.backproject(f.depth.astype(float), f.K)
    N, nv = orc.normals(P, valid)
    assert not nv[0].any() and not nv[-1].any() and not nv[:, 0].any() and not nv[:, -1].any()
    H, W = valid.shape
    ok = np.zeros_like(valid, dtype=bool)
    ok[1:-1, 1:-1] = True
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            ok[1:-1, 1:-1] &= valid[1 + dj:H - 1 + dj, 1 + di:W - 1 + di] > 0
    assert np.array_equal(nv.astype(bool), ok)
    nn = np.linalg.norm(N[:, ok], axis=0)
    assert np.max(np.abs(nn - 1.0)) < 1e-12
    assert np.all(N[:, ~ok] == 0.0)


def test_mirror_symmetry_of_normals(orc):
    f = scenes.make_frame(1, 2)
    d = f.depth.astype(float)
    H, W = d.shape
    K = f.K
    Km = scenes.Intrinsics(K.fx, K.fy, (W - 1) - K.cx, K.cy)
    P, v = orc.backproject(d, K)
    N, nv = orc.normals(P, v)
    Pm, vm = orc.backproject(d[:, ::-1].copy(), Km)
    Nm, nvm = orc.normals(Pm, vm)
    assert np.array_equal(nvm, nv[:, ::-1])
    assert np.max(np.abs(Nm[0] + N[0][:, ::-1])) < 1e-9
    assert np.max(np.abs(Nm[1] - N[1][:, ::-1])) < 1e-9
    assert np.max(np.abs(Nm[2] - N[2][:, ::-1])) < 1e-9
