"""Segmentation of the normal image on the GPU against the oracle, through the
C ABI: both sides take the same FP32 normals, and every floating-point
decision is FP32 on both, so edges, region labels and their count must be
bit-exact.  Then the paper's whole chain on the GPU (diffusion, normals,
segmentation, region-mode RANSAC) against the scene's planes."""
import numpy as np
import pytest

import scenes
from gpu_util import log, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_01919_amd as pp
    pp.default_context(0)
    return pp


def _normals(orc, f, noisy):
    # noisy: the sensor-like depth after the oracle's diffusion (the paper segments smoothed depth)
    cfg = scenes.CONFIGS[f.meta["config"]]
    d = orc.diffuse(f.depth, cfg.diffuse_iters, cfg.lam, cfg.kappa_mm) if noisy else f.depth_m * 1000.0
    P, valid = orc.backproject(d, f.K)
    N, nvalid = orc.normals(P, valid)
    return N.astype(np.float32), (valid.astype(np.uint8) | (nvalid.astype(np.uint8) << 1))


def _gpu(pp, N, vbyte, low, high, min_area, max_regions):
    import torch
    reg, n, edge = pp.segment(torch.from_numpy(N).cuda(), torch.from_numpy(vbyte).cuda(), low, high, min_area,
                              max_regions, edges=True)
    torch.cuda.synchronize()
    return reg.cpu().numpy(), int(n.cpu().item()), edge.cpu().numpy()


CASES = [(1, 0, None, False), (1, 1, None, True), (2, 0, None, False), (2, 3, None, True), (3, 1, (424, 240), True),
         (3, 2, (848, 480), False), (4, 0, (1280, 720), True), (2, 5, (301, 97), True)]


@pytest.mark.parametrize("cid,k,size,noisy", CASES)
def test_segmentation_matches_the_oracle(pp, orc, cid, k, size, noisy):
    f = scenes.make_frame(cid, k, size=size)
    H, W = f.depth.shape
    N, vbyte = _normals(orc, f, noisy)
    min_area = max(50, -(-2 * W * H // 1000))
    log(f"segmentation cfg={cid} k={k} {W}x{H} noisy={noisy} min_area={min_area}")
    for low, high in ((0.35, 0.7), (0.2, 1.5)):
        reg, n, edge = _gpu(pp, N, vbyte, low, high, min_area, 127)
        ref, nr, eref = orc.segment(N, vbyte >> 1 & 1, low, high, min_area, 127)
        log(f"  low={low} high={high}: {n} regions, {int(edge.sum())} edge pixels")
        assert np.array_equal(edge, eref)
        assert n == nr and np.array_equal(reg, ref)
        again = _gpu(pp, N, vbyte, low, high, min_area, 127)
        assert np.array_equal(again[0], reg) and again[1] == n and np.array_equal(again[2], edge)


def test_segmentation_edge_cases(pp, orc):
    f = scenes.make_frame(1, 0)
    N, vbyte = _normals(orc, f, False)
    # at most one region; every normal invalid; a 3x3 image
    reg, n, _ = _gpu(pp, N, vbyte, 0.35, 0.7, 50, 1)
    ref, nr, _ = orc.segment(N, vbyte >> 1 & 1, 0.35, 0.7, 50, 1)
    assert n == nr == 1 and np.array_equal(reg, ref)
    zero = vbyte & 1
    reg, n, edge = _gpu(pp, N, zero, 0.35, 0.7, 50, 10)
    assert n == 0 and (reg == -1).all() and edge.sum() == 0
    small = np.ascontiguousarray(N[:, :3, :3])
    reg, n, _ = _gpu(pp, small, np.full((3, 3), 3, np.uint8), 0.3, 0.6, 1, 5)
    ref, nr, _ = orc.segment(small, np.ones((3, 3), np.uint8), 0.3, 0.6, 1, 5)
    assert n == nr and np.array_equal(reg, ref)


def test_segmentation_argument_checks(pp):
    import torch
    N = torch.zeros((3, 64, 64), dtype=torch.float32, device="cuda")
    v = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    for kw in (dict(low=0.5, high=0.2), dict(low=-1.0), dict(max_regions=0), dict(min_area=0), dict(min_area=0)):
        with pytest.raises(pp.PPError):
            pp.segment(N, v, **kw)
    with pytest.raises(pp.PPError):  # 4096 x min_area must cover the image
        pp.segment(torch.zeros((3, 256, 256), dtype=torch.float32, device="cuda"),
                   torch.zeros((256, 256), dtype=torch.uint8, device="cuda"), min_area=10)


def test_paper_chain_on_the_gpu_finds_the_scene_planes(pp, orc):
    """Diffusion -> normals -> segmentation -> region-mode RANSAC, all on the
    GPU; stored planes lie on the scene's planes."""
    import torch
    f = scenes.make_frame(2, 0)
    H, W = f.depth.shape
    K = (f.K.fx, f.K.fy, f.K.cx, f.K.cy)
    dmm = pp.diffuse(to_dev(f.depth), 20, 0.2, 30.0)
    pts, nrm, valid = pp.normals(dmm, K)
    reg, nreg = pp.segment(nrm, valid, 0.35, 0.7, 615, 127)
    R = 127
    cfg = pp.RansacConfig(max_planes=R, hyps=10, min_inliers=1, thresh_m=0.01, seed=7, frame_id=0)
    planes, n, labels = pp.ransac_regions(pts, valid, reg, cfg)
    torch.cuda.synchronize()
    nreg = int(nreg.cpu().item())
    recs = pp.planes_to_numpy(planes, R)
    stored = [g for g in range(nreg) if recs[g]["hyp_index"] >= 0]
    log(f"  chain: {nreg} regions, {len(stored)} planes stored")
    assert nreg >= 8 and len(stored) >= 6
    reg_np, lab = reg.cpu().numpy(), labels.cpu().numpy()
    assert ((lab < 0) | (lab == reg_np)).all()
    gt = np.array(f.gt_planes)
    for g in stored:
        nvec, d = recs[g]["n"], recs[g]["d"]
        lab_g = f.gt_labels[reg_np == g]
        best = gt[np.bincount(lab_g[lab_g >= 0]).argmax()]  # the scene plane the region lies on
        assert abs(best[:3] @ nvec) > np.cos(np.radians(5.0)), g
        assert abs(abs(best[3]) - d) < 0.03, g
