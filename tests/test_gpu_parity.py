"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Tolerances: diffused depth <= 1e-3 mm max-abs with holes exactly 0; points
<= 1e-6 m; normals <= 1e-4 rad where both are valid and well conditioned;
hypothesis triples bit-exact; counts within the band of residuals whose side
of t FP32 rounding may flip; refit planes 1e-9 against the oracle's refit of
the GPU's own inlier set; inlier masks bit-exact outside the near-threshold
band.
"""
import numpy as np
import pytest

import scenes
from gpu_util import cfg_params, hyp_eps, labels_explained, log, run_plain, score_margin, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_01919_amd as pp
    pp.default_context(0)
    return pp


# ------------------------------------------------------------------ diffusion
@pytest.mark.parametrize("cid,k,edge", [(1, 0, 0), (1, 1, 1), (2, 0, 0), (3, 2, 0)])
def test_diffusion_matches_oracle(pp, orc, cid, k, edge):
    log(f"diffusion parity cfg={cid} k={k} edge={edge}")
    f = scenes.make_frame(cid, k)
    cfg = scenes.CONFIGS[cid]
    out = pp.diffuse(to_dev(f.depth), cfg.diffuse_iters, cfg.lam, cfg.kappa_mm, edge).cpu().numpy()
    ref = orc.diffuse(f.depth, cfg.diffuse_iters, cfg.lam, cfg.kappa_mm, edge)
    holes = f.depth == 0
    assert np.all(out[holes] == 0.0)
    err = np.abs(out.astype(np.float64) - ref)
    log(f"  max |dI| = {err.max():.3e} mm")
    assert err.max() <= 1e-3
    # conservation at rounding level: the summed change is bounded by one ulp per pixel
    drift = abs(out.astype(np.float64).sum() - f.depth.astype(np.float64).sum())
    assert drift <= np.spacing(out[~holes]).astype(np.float64).sum()


@pytest.mark.parametrize("iters", [1, 7, 20])
def test_constant_image_is_a_fixed_point(pp, iters):
    img = np.full((61, 97), 2345, np.uint16)
    img[np.random.default_rng(iters).random(img.shape) < 0.1] = 0
    out = pp.diffuse(to_dev(img), iters, 0.25, 30.0).cpu().numpy()
    assert np.array_equal(out, img.astype(np.float32))


def test_all_tunings_give_bitwise_identical_diffusion(pp):
    f = scenes.make_frame(2, 1)
    ctx = pp.Context(0)
    outs = []
    for tile in (1, 2, 3, 4, 5, 6):
        for T in (1, 3, 5, 10):
            ctx.set_tuning(diffuse_tile=tile, diffuse_t=T)
            outs.append(pp.diffuse(to_dev(f.depth), 20, ctx=ctx).cpu().numpy())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    ctx.close()


@pytest.mark.parametrize("H,W", [(3, 3), (3, 300), (300, 3), (4, 57), (17, 57), (33, 130), (65, 129)])
def test_register_diffusion_on_small_and_ragged_shapes(pp, orc, H, W):
    """The register-resident kernel (one wave per 64 - 2T columns and 16 rows)
    on frames narrower or shorter than one of its tiles: bitwise the LDS
    tiles' result at every fusion depth, and the oracle's within 1e-3 mm."""
    rng = np.random.default_rng(1000 * H + W)
    y, x = np.mgrid[0:H, 0:W]
    img = np.rint(1500 + 2.0 * x + 3.0 * y + rng.normal(0.0, 10.0, (H, W))).astype(np.uint16)
    img[rng.random((H, W)) < 0.05] = 0
    ctx = pp.Context(0)
    outs = []
    for tile, T in ((1, 3), (6, 1), (6, 4), (6, 10), (5, 5)):
        ctx.set_tuning(diffuse_tile=tile, diffuse_t=T)
        outs.append(pp.diffuse(to_dev(img), 20, 0.2, 30.0, ctx=ctx).cpu().numpy())
    ctx.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    ref = orc.diffuse(img, 20, 0.2, 30.0)
    assert np.abs(outs[0].astype(np.float64) - ref).max() <= 1e-3


# ------------------------------------------------------------------ normals
@pytest.mark.parametrize("cid,k", [(1, 0), (2, 0), (3, 1)])
def test_points_and_normals_match_oracle(pp, orc, cid, k):
    log(f"normals parity cfg={cid} k={k}")
    f = scenes.make_frame(cid, k)
    cfg = scenes.CONFIGS[cid]
    K = f.K
    dmm = pp.diffuse(to_dev(f.depth), cfg.diffuse_iters, cfg.lam, cfg.kappa_mm)
    pts, nrm, valid = pp.normals(dmm, (K.fx, K.fy, K.cx, K.cy))
    dmm, pts, nrm, valid = (t.cpu().numpy() for t in (dmm, pts, nrm, valid))
    P, v = orc.backproject(dmm.astype(np.float64), K)
    assert np.array_equal(valid & 1, v)
    assert np.max(np.abs(pts - P)) <= 1e-6
    N, nv, gx, gy = orc.normals(P, v, with_grad=True)
    assert np.array_equal((valid >> 1) & 1, nv)
    both = nv > 0
    m = np.linalg.norm(np.cross(gx.reshape(3, -1).T, gy.reshape(3, -1).T), axis=1).reshape(nv.shape)
    well = both & (m >= 1e-2 * np.linalg.norm(gx, axis=0) * np.linalg.norm(gy, axis=0))
    # angle between unit vectors as atan2(|a x b|, a.b): arccos of a dot product
    # would read the 1e-7 norm error of an FP32 unit vector as 5e-4 rad
    g = nrm.astype(np.float64)
    g = g / np.where(both, np.linalg.norm(g, axis=0), 1.0)
    cr = np.linalg.norm(np.cross(N.reshape(3, -1).T, g.reshape(3, -1).T), axis=1).reshape(nv.shape)
    ang = np.arctan2(cr, np.einsum("chw,chw->hw", N, g))[well]
    log(f"  normals: {well.sum()} well-conditioned of {both.sum()}, max angle {ang.max():.2e} rad, "
        f"grazing {both.sum() - well.sum()} reported apart")
    assert ang.max() <= 1e-4
    # end to end against the oracle's own diffusion
    Po, _ = orc.backproject(orc.diffuse(f.depth, cfg.diffuse_iters, cfg.lam, cfg.kappa_mm), K)
    assert np.max(np.abs(pts - Po)) <= 2e-6


# ------------------------------------------------------------------ RANSAC, round by round
def _follow(pp, orc, frame, cid, k, rounds=None, **over):
    """Follow mode (R22): the oracle is handed the GPU's assignment state
    before round r and round r is checked alone.

    - triples bit-exact, hypothesis validity equal;
    - each FP32 hypothesis plane within the derived bound hyp_eps of the
      float64 plane through the same three points;
    - scoring: every count equals the float64 recount of the GPU's own FP32
      plane except for points within the canonical residual's rounding
      margin 16u (P1 + |d|) of t, and S (the inliers of j*) equals that
      recount exactly outside the margin;
    - counts also lie between the oracle planes' counts at t -+ (bound +
      margin), and j* is the GPU's own argmax and a legitimate winner;
    - refit, F and labels as the oracle's refit of the GPU's own S."""
    H, W = frame.depth.shape
    dc, rc = cfg_params(cid, W, H, k, **over)
    g = run_plain(frame, dc, rc)
    P = g["points"].astype(np.float64)
    valid = g["valid"] & 1
    L = orc.valid_list(valid)
    dbg = g["dbg"]
    assert dbg["n_valid"][0] == len(L)
    assert np.array_equal(dbg["valid_list"][:len(L)], L)
    prm = orc.RansacParams(rc.hyps, rc.max_planes, rc.min_inliers, rc.thresh_m, rc.seed, rc.frame_id)
    labels = g["labels"]
    Xall = P.reshape(3, -1)
    pmax = float(np.max(np.linalg.norm(Xall[:, L], axis=0))) if len(L) else 0.0
    p1max = float(np.max(np.abs(Xall[:, L]).sum(axis=0))) if len(L) else 0.0
    t = rc.thresh_m
    n_rounds = rounds or rc.max_planes
    ran = 0
    worst = dict(plane_ratio=0.0, plane_bound=0.0, margin=0.0, margin_px=0)
    for r in range(n_rounds):
        info = dbg["round_info"][r]
        if info[3] < 0:
            assert r == g["n_planes"]  # rounds stop right after the last emitted plane
            break
        ran += 1
        assigned = ((labels >= 0) & (labels < r)).astype(np.uint8)
        free = assigned.reshape(-1)[L] == 0
        tr_g = dbg["triples"][r]
        hy_g = dbg["hyps"][r].astype(np.float64)
        ct_g = dbg["counts"][r]
        # hypotheses: triples bit-exact; FP32 planes within the derived bound
        tr_o, pl_o, hv_o = orc.hypotheses(P, L, assigned, prm, r)
        gave_up = (tr_o < 0).any(axis=1)
        assert np.array_equal(tr_g[~gave_up], tr_o[~gave_up])
        assert np.all(tr_g[gave_up] == -1)
        hv_g = ~np.isnan(hy_g[:, 3])
        assert np.array_equal(hv_g, hv_o > 0)
        bound = hyp_eps(pl_o, tr_o, L, P, pmax)
        # a plane through the camera centre (d ~ 0) may come out with either sign
        dn = np.minimum(np.linalg.norm(hy_g[:, :3] - pl_o[:, :3], axis=1) * pmax + np.abs(hy_g[:, 3] - pl_o[:, 3]),
                        np.linalg.norm(hy_g[:, :3] + pl_o[:, :3], axis=1) * pmax + np.abs(hy_g[:, 3] + pl_o[:, 3]))
        assert np.all(dn[hv_g] <= bound[hv_g]), (r, np.flatnonzero(hv_g & (dn > bound))[:5])
        if hv_g.any():
            worst["plane_ratio"] = max(worst["plane_ratio"], float(np.max(dn[hv_g] / bound[hv_g])))
            worst["plane_bound"] = max(worst["plane_bound"], float(np.max(bound[hv_g])))
        if info[3] == 1:
            assert not hv_o.any()
            break
        # counts: the GPU's own FP32 planes recounted in float64, exact outside the residual margin
        marg = score_margin(hy_g, p1max)
        hv8 = hv_g.astype(np.uint8)
        c64, lo, hi, _ = orc.score(P, L, assigned, np.nan_to_num(hy_g), hv8, t, marg)
        bad = hv_g & ((ct_g < lo) | (ct_g > hi))
        assert not bad.any(), (r, np.flatnonzero(bad)[:5], ct_g[bad][:5], lo[bad][:5], hi[bad][:5])
        assert np.all(ct_g[~hv_g] == 0)
        worst["margin"] = max(worst["margin"], float(marg[hv_g].max()))
        worst["margin_px"] = max(worst["margin_px"], int((hi - lo)[hv_g].max()))
        # and between the oracle planes' counts at t -+ (plane bound + margin)
        res = orc.ransac_round(P, L, assigned, prm, r, bound + marg)
        assert res.jstar >= 0
        bad = hv_g & ((ct_g < res.counts_lo) | (ct_g > res.counts_hi))
        assert not bad.any(), (r, np.flatnonzero(bad)[:5])
        js = int(info[0])
        assert js == int(np.flatnonzero(hv_g & (ct_g == ct_g[hv_g].max()))[0])
        assert res.counts_hi[js] >= res.counts_lo[hv_o > 0].max()  # a legitimate winner
        # S = inliers of j*: exactly the float64 inliers of the GPU's plane outside the margin
        S = (dbg["masks"][r].reshape(H, W) & 1) > 0
        assert S.sum() == ct_g[js] == info[1]
        Xr = Xall[:, L]
        d_g = np.abs(hy_g[js, :3] @ Xr + hy_g[js, 3])
        S64 = np.zeros(H * W, bool)
        S64[L] = (d_g < t) & free
        nearS = np.zeros(H * W, bool)
        nearS[L] = np.abs(d_g - t) <= marg[js]
        assert not ((S.reshape(-1) != S64) & ~nearS).any()
        # refit: the GPU plane is the least-squares plane of its own S
        pl_ref, ce_ref = orc.refit(P, np.flatnonzero(S.reshape(-1)).astype(np.int32))
        Fm = (dbg["masks"][r].reshape(H, W) & 2) > 0
        if info[3] == 0:
            gp = g["planes"][r]
            gpl = np.append(gp["n"], gp["d"])
            assert np.max(np.abs(gpl - pl_ref)) <= 1e-9 * max(1.0, abs(pl_ref[3]))
            assert np.max(np.abs(gp["centroid"] - ce_ref)) <= 1e-9
            assert gp["hyp_index"] == js and gp["inliers"] == Fm.sum() == info[2]
            # F: the refit plane's inliers (compensated FP32) agree with float64 away from t
            dist = np.abs(gpl[:3] @ Xr + gpl[3])
            F64 = np.zeros(H * W, bool)
            F64[L] = (dist < t) & free
            nearF = np.zeros(H * W, bool)
            nearF[L] = np.abs(dist - t) <= 1e-7
            assert not ((Fm.reshape(-1) != F64) & ~nearF).any()
            assert np.array_equal(labels == r, Fm)
            # and with the oracle's own round when both picked the same hypothesis and set
            if res.jstar == js and np.array_equal(S.reshape(-1), res.smask.reshape(-1)):
                assert np.max(np.abs(gpl - res.plane)) <= 1e-6 * max(1.0, res.plane[3])
                dF = Fm.reshape(-1) != res.fmask.reshape(-1)
                dist_or = np.zeros(H * W)
                dist_or[L] = np.abs(res.plane[:3] @ Xr + res.plane[3])
                assert not (dF & (np.abs(dist_or - t) > 1e-6)).any()
        else:
            assert info[2] < rc.min_inliers and g["n_planes"] == r
            assert not (labels == r).any()
            break
    log(f"  followed {ran} rounds, {g['n_planes']} planes; largest plane bound {worst['plane_bound']:.2e} m "
        f"(used up to {worst['plane_ratio']:.2f} of it), largest residual margin {worst['margin']:.2e} m "
        f"({worst['margin_px']} px inside it at most)")
    return g


@pytest.mark.parametrize("k", [0, 1, 2])
def test_ransac_follow_mode_160x120(pp, orc, k):
    log(f"ransac follow mode cfg=1 k={k}")
    f = scenes.make_frame(1, k)
    g = _follow(pp, orc, f, 1, k)
    assert g["n_planes"] >= 3


def test_ransac_follow_mode_640x480(pp, orc):
    log("ransac follow mode cfg=2 k=0")
    f = scenes.make_frame(2, 0)
    g = _follow(pp, orc, f, 2, 0)
    assert g["n_planes"] >= 6


def test_ransac_follow_mode_spiral_mixed_size(pp, orc):
    log("ransac follow mode cfg=3 k=0 (424x240, 1024 hypotheses)")
    f = scenes.make_frame(3, 0)
    _follow(pp, orc, f, 3, 0)


def test_ransac_follow_mode_1280x720(pp, orc):
    """The 720p frames of the large-batch workload: 4096 hypotheses a round,
    921600 pixels, every round followed."""
    log("ransac follow mode cfg=4 k=0 (1280x720, 4096 hypotheses)")
    f = scenes.make_frame(4, 0)
    assert f.depth.shape == (720, 1280)
    g = _follow(pp, orc, f, 4, 0)
    assert g["n_planes"] >= 6


def test_ransac_few_hypotheses_and_one_plane(pp, orc):
    f = scenes.make_frame(1, 3)
    _follow(pp, orc, f, 1, 3, hyps=1, max_planes=1)
    _follow(pp, orc, f, 1, 3, hyps=37, max_planes=3)


def test_min_inliers_above_every_plane_emits_nothing(pp, orc):
    f = scenes.make_frame(1, 0)
    g = _follow(pp, orc, f, 1, 0, min_inliers=10 ** 6)
    assert g["n_planes"] == 0 and np.all(g["labels"] == -1)
    assert g["dbg"]["round_info"][0][3] == 2


# ------------------------------------------------------------------ free-running against the oracle pipeline
@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_full_pipeline_matches_the_oracle_pipeline(pp, orc, k):
    log(f"free-running pipeline cfg=1 k={k}")
    f = scenes.make_frame(1, k)
    H, W = f.depth.shape
    dc, rc = cfg_params(1, W, H, k)
    g = run_plain(f, dc, rc)
    prm = orc.RansacParams(rc.hyps, rc.max_planes, rc.min_inliers, rc.thresh_m, rc.seed, rc.frame_id)
    o = orc.pipeline(f.depth, f.K, dc.iters, dc.lam, dc.kappa_mm, prm)
    n = min(g["n_planes"], o.ransac.n_planes)
    same = 0
    for r in range(n):
        gp = np.append(g["planes"][r]["n"], g["planes"][r]["d"])
        if np.max(np.abs(gp - o.ransac.planes[r])) <= 1e-6 * max(1.0, o.ransac.planes[r][3]):
            same += 1
        else:
            break
    log(f"  planes gpu={g['n_planes']} oracle={o.ransac.n_planes} identical-prefix={same}")
    assert g["n_planes"] == o.ransac.n_planes and same == n
    # labels exact except near t (R20), judged with the planes of the round that claimed the pixel
    pg = [np.append(q["n"], q["d"]) for q in g["planes"]]
    ndiff, used = labels_explained(g["points"], o.P, g["labels"], o.ransac.labels, pg, o.ransac.planes,
                                  rc.thresh_m)
    log(f"  {ndiff} labels differ, each within {used:.2e} m of t")


# ------------------------------------------------------------------ brute force over triples
def test_scored_triples_match_brute_force(pp, orc):
    """Every triple of a 9x8 crop scored against its points: counts within the
    near-threshold band of the float64 counts, planes close."""
    import itertools
    import torch
    f = scenes.make_frame(1, 0)
    crop = f.depth[70:78, 60:69].copy()
    K = scenes.Intrinsics(f.K.fx, f.K.fy, f.K.cx - 60, f.K.cy - 70)
    dmm = pp.diffuse(to_dev(crop), 0)
    pts, nrm, valid = pp.normals(dmm, (K.fx, K.fy, K.cx, K.cy))
    P = pts.cpu().numpy().astype(np.float64)
    v = valid.cpu().numpy() & 1
    L = orc.valid_list(v)
    trip = np.array(list(itertools.combinations(range(len(L)), 3)), dtype=np.int32)
    offs = L[trip].astype(np.int32)
    planes, counts = pp.score_triples(pts, valid, torch.from_numpy(offs).cuda(), 0.01)
    planes, counts = planes.cpu().numpy().astype(np.float64), counts.cpu().numpy()
    X = P.reshape(3, -1)[:, L]
    e1 = X[:, trip[:, 1]] - X[:, trip[:, 0]]
    e2 = X[:, trip[:, 2]] - X[:, trip[:, 0]]
    m = np.cross(e1.T, e2.T)
    mn = np.linalg.norm(m, axis=1)
    ok = mn > 1e-3 * np.linalg.norm(e1, axis=0) * np.linalg.norm(e2, axis=0)
    nrm64 = m / np.where(mn > 0, mn, 1)[:, None]
    d64 = -np.einsum("ij,ji->i", nrm64, X[:, trip[:, 0]])
    flip = d64 < 0
    nrm64[flip] *= -1
    d64[flip] *= -1
    pl64 = np.column_stack([nrm64, d64])
    hv = ~np.isnan(planes[:, 3])
    assert np.array_equal(hv, ok)
    # triples on one image row span a plane through the camera centre (d ~ 0): sign is free
    dpl = np.minimum(np.abs(planes - pl64).max(1), np.abs(planes + pl64).max(1))
    assert np.max(dpl[ok]) <= 1e-4
    pmax = float(np.max(np.linalg.norm(X, axis=0)))
    eps = hyp_eps(pl64, trip, np.arange(len(L)), X.reshape(3, 1, -1), pmax)
    c, lo, hi, _ = orc.score(X.reshape(3, 1, -1).copy(), np.arange(len(L), dtype=np.int32),
                             np.zeros((1, len(L)), np.uint8), pl64, ok.astype(np.uint8), 0.01, eps)
    assert np.all((counts >= lo) & (counts <= hi))
    log(f"  {len(trip)} triples, {int((counts != c).sum())} differ from float64 within the band")


# ------------------------------------------------------------------ equivalence of the execution forms
def _batch_frames(pp, frames_spec):
    outs = []
    for cid, k in frames_spec:
        f = scenes.make_frame(cid, k)
        H, W = f.depth.shape
        dc, rc = cfg_params(cid, W, H, k)
        outs.append((f, pp.make_outputs(to_dev(f.depth), (f.K.fx, f.K.fy, f.K.cx, f.K.cy), dc, rc)))
    return outs


def _snapshot(fo):
    return [t.cpu().numpy().copy() for t in (fo.depth_mm, fo.points, fo.normals, fo.valid, fo.planes, fo.n_planes,
                                              fo.labels)]


def test_batch_graph_eager_and_plain_are_bitwise_equal(pp):
    import torch
    spec = [(1, 0), (2, 0), (3, 0), (1, 1), (3, 2), (2, 1)]
    frames = _batch_frames(pp, spec)
    for _, fo in frames:
        pp.run_frame(fo)
    torch.cuda.synchronize()
    plain = [_snapshot(fo) for _, fo in frames]
    for mode in ("eager", "graph", "graph"):
        for _, fo in frames:
            for t in (fo.depth_mm, fo.points, fo.normals, fo.planes, fo.labels):
                t.zero_()
        pp.batch_run([fo for _, fo in frames], graph=(mode == "graph"))
        torch.cuda.synchronize()
        for (f, fo), ref in zip(frames, plain):
            got = _snapshot(fo)
            for a, b in zip(got, ref):
                assert np.array_equal(a, b), mode
    log(f"  batch of {len(spec)} ragged frames: plain == eager == graph (x2)")


def test_batch_of_odd_widths_equals_the_plain_path(pp):
    """Widths that are not multiples of 4 (groups of 4 row-major pixels wrap
    into the next row in the normals, valid-list and round-0 list passes), in
    a ragged graph batch and one by one: every output bitwise equal."""
    import torch
    sizes = [(301, 97), (57, 33), (130, 65), (421, 240), (98, 77)]
    frames = []
    for i, (W, H) in enumerate(sizes):
        f = scenes.make_frame(3, i, size=(W, H))
        dc, rc = cfg_params(3, W, H, i)
        frames.append(pp.make_outputs(to_dev(f.depth), (f.K.fx, f.K.fy, f.K.cx, f.K.cy), dc, rc))
    for fo in frames:
        pp.run_frame(fo)
    torch.cuda.synchronize()
    plain = [_snapshot(fo) for fo in frames]
    for fo in frames:
        for t in (fo.depth_mm, fo.points, fo.normals, fo.planes, fo.labels):
            t.zero_()
    pp.batch_run(frames, graph=True)
    torch.cuda.synchronize()
    for i, (fo, ref) in enumerate(zip(frames, plain)):
        for a, b in zip(_snapshot(fo), ref):
            assert np.array_equal(a, b), (i, sizes[i])
    log(f"  odd widths {sizes}: graph batch == plain, {[int(r[5][0]) for r in plain]} planes")


def test_large_batch_with_capped_grids_equals_the_plain_path(pp):
    """96 frames of 1280x720 in one batch (4 kernel chains of 24 frames): the
    per-chunk passes (valid-list scatter, moments, final count, removal) run
    capped, odd grids whose blocks take several chunks each, which no smaller
    batch reaches; every output of every frame, after a graph and an eager
    run, is bitwise the plain path's."""
    import torch
    base = [scenes.make_frame(4, k) for k in range(8)]
    frames = []
    for i in range(96):
        f = base[i % 8]
        H, W = f.depth.shape
        dc, rc = cfg_params(4, W, H, i, hyps=1024)
        frames.append(pp.make_outputs(to_dev(f.depth), (f.K.fx, f.K.fy, f.K.cx, f.K.cy), dc, rc))
    for fo in frames:
        pp.run_frame(fo)
    torch.cuda.synchronize()
    keys = ("depth_mm", "points", "normals", "valid", "planes", "n_planes", "labels")
    plain = [[getattr(fo, k).clone() for k in keys] for fo in frames]
    for graph in (True, False):
        for fo in frames:
            for t in (fo.depth_mm, fo.points, fo.normals, fo.planes, fo.labels):
                t.zero_()
        pp.batch_run(frames, graph=graph)
        torch.cuda.synchronize()
        for i, (fo, ref) in enumerate(zip(frames, plain)):
            for k, a in zip(keys, ref):
                assert torch.equal(getattr(fo, k), a), (graph, i, k)
    log(f"  96 x 1280x720 batch: graph and eager runs bitwise the plain path "
        f"({sum(int(fo.n_planes.item()) for fo in frames)} planes)")


def test_batch_of_nine_frames_equals_the_plain_path(pp):
    """More frames than XCDs and not a multiple of 8: the XCD-ordered grid of
    the hypothesis kernel still covers every (frame, block) once."""
    import torch
    spec = [(1, 0), (1, 1), (1, 2), (3, 0), (3, 1), (3, 2), (2, 0), (2, 1), (2, 2)]
    frames = _batch_frames(pp, spec)
    for _, fo in frames:
        pp.run_frame(fo)
    torch.cuda.synchronize()
    plain = [_snapshot(fo) for _, fo in frames]
    for _, fo in frames:
        for t in (fo.depth_mm, fo.points, fo.normals, fo.planes, fo.labels):
            t.zero_()
    pp.batch_run([fo for _, fo in frames], graph=True)
    torch.cuda.synchronize()
    for (f, fo), ref in zip(frames, plain):
        for a, b in zip(_snapshot(fo), ref):
            assert np.array_equal(a, b)


def test_shuffled_batch_and_repeats_are_deterministic(pp):
    import torch
    spec = [(3, 1), (1, 2), (2, 2), (1, 3)]
    frames = _batch_frames(pp, spec)
    pp.batch_run([fo for _, fo in frames])
    torch.cuda.synchronize()
    ref = [_snapshot(fo) for _, fo in frames]
    order = [2, 0, 3, 1]
    pp.batch_run([frames[i][1] for i in order])
    pp.batch_run([frames[i][1] for i in order])
    torch.cuda.synchronize()
    for (f, fo), r in zip(frames, ref):
        for a, b in zip(_snapshot(fo), r):
            assert np.array_equal(a, b)


def test_scoring_tunings_give_identical_planes(pp):
    import torch
    f = scenes.make_frame(2, 2)
    H, W = f.depth.shape
    dc, rc = cfg_params(2, W, H, 2)
    ref = None
    ctx = pp.Context(0)
    for hb in (1, 2, 3, 4, 5, 6):
        for ch in (1, 4):
            ctx.set_tuning(score_hb=hb, score_chunk=ch)
            fo = pp.make_outputs(to_dev(f.depth), (f.K.fx, f.K.fy, f.K.cx, f.K.cy), dc, rc)
            pp.run_frame(fo, ctx=ctx)
            torch.cuda.synchronize()
            snap = _snapshot(fo)
            if ref is None:
                ref = snap
            for a, b in zip(snap, ref):
                assert np.array_equal(a, b)
    ctx.close()


@pytest.mark.parametrize("cid,k,size,hyps", [(1, 0, None, 256), (2, 1, None, 1024), (3, 2, (301, 97), 5),
                                              (3, 0, (848, 480), 100), (4, 1, (1280, 720), 1024)])
def test_culled_scorer_counts_equal_the_plain_scorer(pp, cid, k, size, hyps):
    """Tile culling decides whole tiles only where the canonical residual
    cannot change side: every count of every round is bitwise the plain one."""
    f = scenes.make_frame(cid, k, size=size)
    H, W = f.depth.shape
    dc, rc = cfg_params(cid, W, H, k, hyps=hyps)
    log(f"culled scorer cfg={cid} k={k} {W}x{H} hyps={hyps}")
    runs = []
    for hb in (1, 4, 5, 6):  # every point; tiles with 1, 2, 4 hypotheses per lane
        ctx = pp.Context(0)
        ctx.set_tuning(score_hb=hb)
        runs.append(run_plain(f, dc, rc, ctx=ctx))
        ctx.close()
    a = runs[0]
    for b in runs[1:]:
        assert a["n_planes"] == b["n_planes"] and np.array_equal(a["labels"], b["labels"])
        for key in ("counts", "triples", "round_info"):
            assert np.array_equal(a["dbg"][key], b["dbg"][key]), key
        assert np.array_equal(a["dbg"]["hyps"], b["dbg"]["hyps"], equal_nan=True)
        for pa, pb in zip(a["planes"], b["planes"]):
            assert np.array_equal(pa["n"], pb["n"]) and pa["d"] == pb["d"] and pa["inliers"] == pb["inliers"]
    log(f"  {a['n_planes']} planes, counts of {int((a['dbg']['round_info'][:, 0] > 0).sum())} rounds equal")


# ------------------------------------------------------------------ edge cases
def test_empty_and_tiny_frames(pp):
    import torch
    dc_args = dict(iters=5)
    for shape, fill in [((120, 160), 0), ((3, 3), 1500), ((3, 5), 0), ((61, 97), None)]:
        if fill is None:
            img = scenes.make_frame(1, 0).depth[:61, :97].copy()
        else:
            img = np.full(shape, fill, np.uint16)
        H, W = img.shape
        dc, rc = cfg_params(1, W, H, 0, **dc_args)
        fo = pp.make_outputs(to_dev(img), (100.0, 100.0, W / 2, H / 2), dc, rc)
        pp.run_frame(fo)
        torch.cuda.synchronize()
        n = int(fo.n_planes.cpu().item())
        lab = fo.labels.cpu().numpy()
        if fill == 0:
            assert n == 0 and np.all(lab == -1)
        assert np.all(lab[img == 0] == -1)
        log(f"  {shape} fill={fill}: {n} planes")


def test_invalid_arguments_are_rejected_before_launch(pp):
    import torch
    from paper_2411_01919_amd import _native as N
    d = torch.zeros((10, 10), dtype=torch.int16, device="cuda")
    with pytest.raises(pp.PPError) as e:
        pp.diffuse(d, 5, lam=0.3)
    assert e.value.status == N.PP_E_INVAL
    with pytest.raises(pp.PPError) as e:
        pp.diffuse(d[:2, :2].contiguous(), 5)
    assert e.value.status == N.PP_E_INVAL
    pts = torch.zeros((3, 10, 10), device="cuda")
    valid = torch.zeros((10, 10), dtype=torch.uint8, device="cuda")
    with pytest.raises(pp.PPError) as e:
        pp.ransac_planes(pts, valid, pp.RansacConfig(max_planes=200))
    assert e.value.status == N.PP_E_INVAL
    # the context is still usable afterwards
    out = pp.diffuse(d, 1)
    torch.cuda.synchronize()
    assert float(out.abs().sum().item()) == 0.0


# ------------------------------------------------------------------ precision forms
@pytest.mark.parametrize("cid,k,size,hb", [(1, 0, None, 4), (2, 1, None, 4), (3, 1, None, 5), (2, 2, None, 6),
                                            (4, 0, (1280, 720), 5)])
def test_matrix_core_forms_equal_the_fp32_path_bitwise(pp, cid, k, size, hb):
    """FP32-MFMA, BF16 and FP16 scoring (with the recheck band, or the
    derived bound alone) return the canonical FP32 counts of every round,
    hence identical planes and labels, at 1, 2 and 4 hypotheses per lane."""
    f = scenes.make_frame(cid, k, size=size)
    H, W = f.depth.shape
    runs = {}
    for prec, band in [(pp.PP_SCORE_FP32, 0.0), (pp.PP_SCORE_MFMA_F32, 0.0), (pp.PP_SCORE_BF16, 0.002),
                       (pp.PP_SCORE_FP16, 0.002), (pp.PP_SCORE_BF16, 1e-4), (pp.PP_SCORE_FP16, 0.0),
                       (pp.PP_SCORE_BF16, 0.0)]:
        dc, rc = cfg_params(cid, W, H, k, precision=prec, recheck_band_m=band)
        ctx = pp.Context(0)
        ctx.set_tuning(score_hb=hb if prec != pp.PP_SCORE_FP32 else 1)
        runs[(prec, band)] = run_plain(f, dc, rc, ctx=ctx)
        ctx.close()
    ref = runs[(pp.PP_SCORE_FP32, 0.0)]
    for key, g in runs.items():
        assert g["n_planes"] == ref["n_planes"], key
        assert np.array_equal(g["dbg"]["counts"], ref["dbg"]["counts"]), key
        assert np.array_equal(g["labels"], ref["labels"]), key
        for a, b in zip(g["planes"], ref["planes"]):
            assert np.array_equal(a["n"], b["n"]) and a["d"] == b["d"], key
    # residuals evaluated on the matrix cores (dbg scored[2]) among those evaluated point by point ([1])
    share = {key: int(g["dbg"]["scored"][2]) / max(1, int(g["dbg"]["scored"][1])) for key, g in runs.items()}
    assert share[(pp.PP_SCORE_FP32, 0.0)] == 0.0
    if hb == 4 or size is not None:  # 64 hypotheses a block, or 4096 hypotheses a round: dense tiles exist
        assert all(v > 0.0 for key, v in share.items() if key[0] != pp.PP_SCORE_FP32), share
    log(f"  cfg={cid} k={k}: {ref['n_planes']} planes identical under every scoring form; matrix-core share "
        + ", ".join(f"{v:.2f}" for key, v in share.items() if key[0] != pp.PP_SCORE_FP32))


@pytest.mark.parametrize("prec,band", [(1, 0.0), (2, 0.002), (3, 0.002), (2, 0.0)])
def test_matrix_core_counts_of_scored_triples(pp, prec, band):
    import torch
    f = scenes.make_frame(2, 0)
    K = f.K
    dmm = pp.diffuse(to_dev(f.depth), 20)
    pts, nrm, valid = pp.normals(dmm, (K.fx, K.fy, K.cx, K.cy))
    v = valid.cpu().numpy() & 1
    L = np.flatnonzero(v.reshape(-1))
    rng = np.random.default_rng(prec)
    offs = torch.from_numpy(rng.choice(L, size=(777, 3)).astype(np.int32)).cuda()
    pl_ref, c_ref = pp.score_triples(pts, valid, offs, 0.01)
    pl, c = pp.score_triples(pts, valid, offs, 0.01, precision=prec, recheck_band_m=band)
    assert torch.equal(c, c_ref) and torch.equal(pl.isnan(), pl_ref.isnan())


def test_batched_bf16_form_equals_plain_fp32(pp):
    import torch
    spec = [(2, 3), (3, 0), (4, 1)]
    ref, outs = [], []
    for cid, k in spec:
        f = scenes.make_frame(cid, k)
        H, W = f.depth.shape
        dc, rc = cfg_params(cid, W, H, k)
        fo = pp.make_outputs(to_dev(f.depth), (f.K.fx, f.K.fy, f.K.cx, f.K.cy), dc, rc)
        pp.run_frame(fo)
        torch.cuda.synchronize()
        ref.append(_snapshot(fo))
        dc, rc = cfg_params(cid, W, H, k, precision=pp.PP_SCORE_BF16, recheck_band_m=0.002)
        outs.append(pp.make_outputs(to_dev(f.depth), (f.K.fx, f.K.fy, f.K.cx, f.K.cy), dc, rc))
    pp.batch_run(outs)
    torch.cuda.synchronize()
    for fo, r in zip(outs, ref):
        for a, b in zip(_snapshot(fo), r):
            assert np.array_equal(a, b)


def test_autotuner_picks_a_valid_tuning_and_caches_it(pp, tmp_path):
    import torch
    from paper_2411_01919_amd import autotune
    frames = [fo for _, fo in _batch_frames(pp, [(1, 0), (1, 1), (3, 0)])]
    ctx = pp.Context(0)
    p = str(tmp_path / "tune.json")
    t = autotune.tune(frames, ctx=ctx, reps=1, path=p)
    assert not t["cached"] and t["diffuse_tile"] in autotune.TILES and t["diffuse_t"] in autotune.DEPTHS
    assert t["diffusion_ms"] <= t["diffusion_default_ms"] + 1e-6
    t2 = autotune.tune(frames, ctx=ctx, reps=1, path=p)
    assert t2["cached"] and t2["diffuse_t"] == t["diffuse_t"]
    assert ctx.get_tuning()["diffuse_t"] == t["diffuse_t"]
    ctx.close()
