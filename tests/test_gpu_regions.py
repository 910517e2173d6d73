"""Region-mode RANSAC (Alg. 2 as printed) on the GPU against the oracle,
through the C ABI.  Both sides take the same FP32 points and the scene
generator's ground-truth plane labels as regions.

Integer work is compared exactly (region sizes, drawn triples).  Floating
point is compared to its rounding band: FP32 hypothesis planes within eps_j
of the oracle's FP64 planes (the band of the whole-frame tests), inlier
counts between the oracle's counts at t - eps_j and t + eps_j, summed
errors within n_g eps_j.  The kept hypothesis must be a legitimate minimum
under those bands (and the oracle's own when its minimum is separated by
more), the store decision must agree wherever the band does not straddle
the 90 % rule, labels must be exactly the GPU plane's inliers outside
1e-6 m of t, and centroids the FP64 mean of the labelled points."""
import numpy as np
import pytest

import scenes
from gpu_util import EPS32, hyp_eps, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_01919_amd as pp
    pp.default_context(0)
    return pp


def _inputs(orc, f):
    P, valid = orc.backproject(f.depth.astype(float), f.K)
    P32 = P.astype(np.float32)
    return P32, valid


def _run(pp, P32, valid, region, R, hyps, seed, frame_id, t=0.01):
    import torch
    cfg = pp.RansacConfig(max_planes=R, hyps=hyps, min_inliers=1, thresh_m=t, seed=seed, frame_id=frame_id)
    pts = torch.from_numpy(P32).cuda()
    val = torch.from_numpy(valid.astype(np.uint8)).cuda()
    reg = torch.from_numpy(region.astype(np.int16)).cuda()
    planes, n, labels, dbg = pp.ransac_regions(pts, val, reg, cfg, debug=True)
    torch.cuda.synchronize()
    out = dict(planes=pp.planes_to_numpy(planes, R), raw=planes.cpu().numpy(), n=int(n.cpu().item()),
               labels=labels.cpu().numpy(), **{k: v.cpu().numpy() for k, v in dbg.items()})
    return out


def _check(orc, P32, valid, region, R, hyps, seed, frame_id, got, t=0.01):
    import oracle
    P = P32.astype(np.float64)
    H, W = region.shape
    prm = oracle.RansacParams(hyps=hyps, max_planes=1, min_inliers=1, thresh=t, seed=seed, frame=frame_id)
    ref0 = orc.ransac_regions(P, valid, region, R, prm)
    assert np.array_equal(got["npts"], ref0.npts)
    assert np.array_equal(got["triples"], ref0.triples)
    pmax = float(np.abs(P.reshape(3, -1)).sum(axis=0).max())
    flat_r, flat_v = region.reshape(-1), valid.reshape(-1)
    eps = np.zeros((R, hyps))
    for g in range(R):
        L = np.nonzero((flat_v & 1).astype(bool) & (flat_r == g))[0]
        # plane bound plus the canonical FP32 residual's own rounding, 16u (P1 + |d|)
        eps[g] = hyp_eps(ref0.planes[g], ref0.triples[g], L, P, pmax) + \
            16.0 * EPS32 * (pmax + np.abs(np.nan_to_num(ref0.planes[g][:, 3])))
    ref = orc.ransac_regions(P, valid, region, R, prm, eps=eps)
    hv = ~np.isnan(got["hyps"][..., 3])
    assert np.array_equal(hv, ref.hvalid)
    X = P.reshape(3, -1)
    stored_gpu = 0
    for g in range(R):
        n = int(ref.npts[g])
        v = ref.hvalid[g]
        if v.any():
            q, o = got["hyps"][g][v].astype(np.float64), ref.planes[g][v]
            dpl = np.abs(q - o).max(axis=1)
            # a plane through the camera centre (|d| inside the band) is camera-facing either way round
            flip = np.abs(o[:, 3]) <= eps[g][v]
            dpl[flip] = np.minimum(dpl[flip], np.abs(q + o).max(axis=1)[flip])
            assert (dpl <= eps[g][v]).all(), g
            c = got["counts"][g][v]
            assert (ref.counts_lo[g][v] <= c).all() and (c <= ref.counts_hi[g][v]).all(), g
            de = np.abs(got["errors"][g][v] - ref.errors[g][v])
            assert (de <= n * eps[g][v] + 1e-9 * ref.errors[g][v]).all(), g
        assert np.isinf(got["errors"][g][~v]).all()
        js = int(got["jstar"][g])
        assert (js >= 0) == v.any()
        pl = got["planes"][g]
        if js < 0:
            assert pl["hyp_index"] == -1 and pl["inliers"] == 0
            continue
        assert v[js]
        # the GPU's choice is its own first minimum, and a legitimate oracle minimum
        eg = got["errors"][g]
        assert eg[js] == eg[v].min() and js == int(np.flatnonzero(v & (eg == eg[js]))[0])
        band = n * eps[g]
        assert ref.errors[g][js] - band[js] <= (ref.errors[g][v] + band[v]).min(), g
        jo = int(ref.jstar[g])
        others = v.copy()
        others[jo] = False
        if others.any() and ref.errors[g][jo] + band[jo] < (ref.errors[g][others] - band[others]).min():
            assert js == jo, g
        cnt = int(got["counts"][g][js])
        stored = 10 * cnt > 9 * n
        assert (pl["hyp_index"] == js) == stored and pl["inliers"] == cnt
        if 10 * ref.counts_lo[g][js] > 9 * n:
            assert stored, g
        if 10 * ref.counts_hi[g][js] <= 9 * n:
            assert not stored, g
        assert np.array_equal(pl["n"], got["hyps"][g][js][:3].astype(np.float64))
        assert pl["d"] == np.float64(got["hyps"][g][js][3])
        mine = (got["labels"].reshape(-1) == g)
        if not stored:
            assert not mine.any()
            continue
        stored_gpu += 1
        h = got["hyps"][g][js].astype(np.float64)
        L = np.nonzero((flat_v & 1).astype(bool) & (flat_r == g))[0]
        r = np.abs(h[:3] @ X[:, L] + h[3])
        sure = np.abs(r - t) > 1e-6
        assert np.array_equal(mine[L][sure], (r < t)[sure]), g
        assert mine.sum() == cnt and not (mine & ~np.isin(np.arange(H * W), L)).any()
        assert np.max(np.abs(pl["centroid"] - X[:, mine].mean(axis=1))) < 1e-9
    assert got["n"] == stored_gpu
    outside = ~np.isin(got["labels"], np.arange(R))
    assert (got["labels"][outside] == -1).all()
    return stored_gpu


CASES = [(1, 0, None, 10), (1, 1, None, 64), (2, 0, None, 10), (2, 2, None, 256), (3, 1, (424, 240), 10),
         (4, 0, (1280, 720), 10), (3, 2, (301, 97), 32)]


@pytest.mark.parametrize("cid,k,size,hyps", CASES)
def test_regions_match_the_oracle(pp, orc, cid, k, size, hyps):
    f = scenes.make_frame(cid, k, size=size)
    H, W = f.depth.shape
    R = int(f.gt_labels.max()) + 1
    log(f"region mode cfg={cid} k={k} {W}x{H} regions={R} hyps={hyps}")
    P32, valid = _inputs(orc, f)
    seed = 0x5EED0000 + cid
    got = _run(pp, P32, valid, f.gt_labels, R, hyps, seed, k)
    ns = _check(orc, P32, valid, f.gt_labels, R, hyps, seed, k, got)
    log(f"  stored {ns} of {R} regions")
    again = _run(pp, P32, valid, f.gt_labels, R, hyps, seed, k)
    for key in got:
        if key != "planes":
            assert np.array_equal(got[key], again[key], equal_nan=key == "hyps"), key


def test_region_edge_cases(pp, orc):
    """Empty, one- and two-point regions, labels beyond max_planes, holes,
    every label negative, one hypothesis, and the largest region count."""
    f = scenes.make_frame(1, 2)
    P32, valid = _inputs(orc, f)
    H, W = valid.shape
    reg = f.gt_labels.copy()
    reg[reg == 2] = 50                     # beyond max_planes: no region; region 2 is empty
    reg[reg == 3] = -1
    vy, vx = np.nonzero(valid)
    reg[vy[0], vx[0]] = 3                  # region 3: one point
    reg[vy[1], vx[1]] = reg[vy[2], vx[2]] = 6  # region 6: two points
    hy, hx = np.nonzero(valid == 0)
    if len(hy):
        reg[hy[0], hx[0]] = 7              # a hole labelled 7 is no point
    R = 8
    log("region edge cases")
    for hyps in (16, 1):
        got = _run(pp, P32, valid, reg, R, hyps, 11, 0)
        _check(orc, P32, valid, reg, R, hyps, 11, 0, got)
        assert got["npts"][2] == 0 and got["jstar"][2] == -1
        assert got["npts"][3] == 1 and got["npts"][6] == 2 and got["npts"][7] == 0
        assert (got["jstar"][[3, 6, 7]] == -1).all()
    neg = np.full((H, W), -1, np.int16)
    got = _run(pp, P32, valid, neg, 5, 8, 1, 0)
    assert got["n"] == 0 and (got["labels"] == -1).all() and (got["npts"] == 0).all()
    # 127 regions: 8x8-pixel cells of the 160x120 frame
    cells = (((np.arange(H)[:, None] // 8) * 20 + np.arange(W)[None, :] // 8) % 127).astype(np.int16)
    got = _run(pp, P32, valid, cells, 127, 8, 5, 1)
    _check(orc, P32, valid, cells, 127, 8, 5, 1, got)


def test_region_mode_argument_checks(pp):
    import torch
    pts = torch.zeros((3, 8, 8), dtype=torch.float32, device="cuda")
    val = torch.zeros((8, 8), dtype=torch.uint8, device="cuda")
    reg = torch.zeros((8, 8), dtype=torch.int16, device="cuda")
    with pytest.raises(pp.PPError) as e:
        pp.ransac_regions(pts, val, reg, pp.RansacConfig(max_planes=4, hyps=8, precision=pp.PP_SCORE_BF16))
    assert e.value.status == -7
    with pytest.raises(pp.PPError):
        pp.ransac_regions(pts, val, reg, pp.RansacConfig(max_planes=128, hyps=8))
