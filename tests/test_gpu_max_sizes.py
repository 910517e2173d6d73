"""Frames at the size limits of the ABI (width and height up to 16384, at most
2^27 pixels), through the plain calls.

The oracle cannot run whole frames this large, so it checks windows: each
output pixel of diffusion depends only on the input within `iters` pixels of
it, and back-projection and normals only on the diffused depth within one
pixel, so a window cut out with that margin (or up to the image border) gives
the oracle the same result there as on the whole frame.  Windows sit at the
corners and the centre, where indexing and clamping go wrong first.  The
planes are checked over the whole frame by the float64 invariants of
sequential removal.

Shapes: 16384 x 64 and 64 x 16384 (each axis at its maximum), and 16384 x 8192
(2^27 pixels).  The last is a 2048 x 2048 rendering of the 640x480 staircase
with every pixel repeated 8 times across and 4 times down, with the focal
lengths and principal point scaled to match, so it back-projects to the same
scene at 2^27 pixels (rendering it directly would take minutes).
"""
import numpy as np
import pytest

import scenes
from gpu_util import cfg_params, check_removal, log, to_dev

pytestmark = pytest.mark.gpu

WIN = 40


@pytest.fixture(scope="module")
def pp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_01919_amd as pp
    pp.default_context(0)
    return pp


def _frame(W, H):
    if W * H <= 1 << 21:
        f = scenes.make_frame(2, 0, size=(W, H))
        return f.depth, f.K
    sx, sy = W // 2048, H // 2048
    base = scenes.make_frame(2, 0, size=(2048, 2048))
    depth = np.repeat(np.repeat(base.depth, sy, axis=0), sx, axis=1)
    K = base.K
    return depth, scenes.Intrinsics(K.fx * sx, K.fy * sy, K.cx * sx, K.cy * sy)


def _windows(W, H):
    w, h = min(WIN, W), min(WIN, H)
    return [(0, 0), ((W - w) // 2, (H - h) // 2), (W - w, H - h)], w, h


def _crop(a, x0, y0, w, h, m, W, H):
    """a[..., y0-m : y0+h+m, x0-m : x0+w+m] clipped to the image, and the
    window's offset inside the crop."""
    cx0, cy0 = max(0, x0 - m), max(0, y0 - m)
    cx1, cy1 = min(W, x0 + w + m), min(H, y0 + h + m)
    return a[..., cy0:cy1, cx0:cx1], x0 - cx0, y0 - cy0, cx0, cy0


def _normals_angle(orc, nrm, valid_bits, P, v, win):
    """Oracle normals of the crop (P, v), compared on the window `win` with the
    GPU's normals and normal-validity bits there; returns the largest angle
    over well-conditioned pixels (atan2 of |a x b| and a.b)."""
    N, nv, gx, gy = orc.normals(P, v, with_grad=True)
    N, nv, gx, gy = N[:, win[0], win[1]], nv[win], gx[:, win[0], win[1]], gy[:, win[0], win[1]]
    assert np.array_equal(valid_bits, nv)
    both = nv > 0
    m = np.linalg.norm(np.cross(gx.reshape(3, -1).T, gy.reshape(3, -1).T), axis=1).reshape(nv.shape)
    well = both & (m >= 1e-2 * np.linalg.norm(gx, axis=0) * np.linalg.norm(gy, axis=0))
    g = nrm.astype(np.float64)
    g = g / np.where(both, np.linalg.norm(g, axis=0), 1.0)
    cr = np.linalg.norm(np.cross(N.reshape(3, -1).T, g.reshape(3, -1).T), axis=1).reshape(nv.shape)
    ang = np.arctan2(cr, np.einsum("chw,chw->hw", N, g))[well]
    return float(ang.max()) if ang.size else 0.0


@pytest.mark.parametrize("W,H", [(16384, 64), (64, 16384), (16384, 8192)])
def test_frames_at_the_size_limits(pp, orc, W, H):
    import torch
    log(f"maximum size {W}x{H} ({W * H} px)")
    depth, K = _frame(W, H)
    assert depth.shape == (H, W)
    cfg = scenes.CONFIGS[2]
    dc, rc = cfg_params(2, W, H, 0)
    dmm = pp.diffuse(to_dev(depth), dc.iters, dc.lam, dc.kappa_mm)
    pts, nrm, valid = pp.normals(dmm, (K.fx, K.fy, K.cx, K.cy))
    planes, n_planes, labels = pp.ransac_planes(pts, valid, rc)
    torch.cuda.synchronize()
    n = int(n_planes.cpu().item())
    dmm, pts, nrm, valid, labels = (t.cpu().numpy() for t in (dmm, pts, nrm, valid, labels))
    log(f"  {n} planes, {int((valid & 1).sum())} valid px")

    wins, w, h = _windows(W, H)
    for x0, y0 in wins:
        # diffusion: the oracle on the window plus its dependency margin
        sub, ox, oy, _, _ = _crop(depth, x0, y0, w, h, dc.iters + 1, W, H)
        ref = orc.diffuse(sub, dc.iters, dc.lam, dc.kappa_mm)[oy:oy + h, ox:ox + w]
        assert np.abs(dmm[y0:y0 + h, x0:x0 + w].astype(np.float64) - ref).max() <= 1e-3, (x0, y0)
        # points and normals: the oracle on the GPU's depth, one pixel of margin
        sub, ox, oy, cx0, cy0 = _crop(dmm, x0, y0, w, h, 1, W, H)
        Kc = scenes.Intrinsics(K.fx, K.fy, K.cx - cx0, K.cy - cy0)
        P, v = orc.backproject(sub.astype(np.float64), Kc)
        win = (slice(oy, oy + h), slice(ox, ox + w))
        g_pts = pts[:, y0:y0 + h, x0:x0 + w]
        assert np.array_equal(valid[y0:y0 + h, x0:x0 + w] & 1, v[win]), (x0, y0)
        assert np.abs(g_pts - P[:, win[0], win[1]]).max() <= 1e-6, (x0, y0)
        # normals: the crop holds the window's one-pixel ring (or the image border)
        ang = _normals_angle(orc, nrm[:, y0:y0 + h, x0:x0 + w], (valid[y0:y0 + h, x0:x0 + w] >> 1) & 1, P, v, win)
        assert ang <= 1e-4, (x0, y0, ang)
        log(f"  window ({x0},{y0}): diffusion, points, normals ok (max angle {ang:.1e} rad)")

    check_removal(pts, labels, valid & 1, pp.planes_to_numpy(planes, n), rc.thresh_m, rc.min_inliers, rc.hyps)
    if W * H == 1 << 27:
        assert n >= 3
