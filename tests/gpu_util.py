"""Helpers shared by the GPU tests: run frames through the HIP path and bring
results back, build oracle inputs, and the near-threshold bands used when
several results are correct (values within rounding of the threshold)."""
import sys

import numpy as np

import scenes

EPS32 = 2.0 ** -24


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def torch_dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    if a.dtype == np.uint16:
        a = a.view(np.int16)
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch_dev())


def cfg_params(cid, W, H, frame_k=0, **over):
    import paper_2411_01919_amd as pp
    cfg = scenes.CONFIGS[cid]
    dc = pp.DiffuseConfig(cfg.diffuse_iters, cfg.lam, cfg.kappa_mm)
    rc = pp.RansacConfig(cfg.max_planes, cfg.hyps, cfg.min_inliers(W, H), cfg.thresh_m, cfg.ransac_seed, frame_k)
    for k, v in over.items():
        if hasattr(dc, k):
            setattr(dc, k, v)
        else:
            setattr(rc, k, v)
    return dc, rc


def run_plain(frame, dc, rc, ctx=None):
    """pp_diffuse -> pp_normals -> pp_ransac_planes_dbg on one frame."""
    import torch
    import paper_2411_01919_amd as pp
    K = frame.K
    d = to_dev(frame.depth)
    dmm = pp.diffuse(d, dc.iters, dc.lam, dc.kappa_mm, dc.edge_stop, ctx=ctx)
    pts, nrm, valid = pp.normals(dmm, (K.fx, K.fy, K.cx, K.cy), ctx=ctx)
    planes, n, labels, dbg = pp.ransac_planes_debug(pts, valid, rc, ctx=ctx)
    torch.cuda.synchronize()
    out = dict(depth_mm=dmm.cpu().numpy(), points=pts.cpu().numpy(), normals=nrm.cpu().numpy(),
               valid=valid.cpu().numpy(), n_planes=int(n.cpu().item()), labels=labels.cpu().numpy(),
               planes=pp.planes_to_numpy(planes, int(n.cpu().item())))
    out["dbg"] = {k: v.cpu().numpy() for k, v in dbg.items()}
    return out


def hyp_eps(planes_or, triples, L, P, pmax):
    """Derived bound on how far the residual implied by an FP32 hypothesis
    plane may sit from the float64 plane through the same three FP32 points,
    anywhere within |p| <= pmax.  With u = 2^-24 and exact inputs:
    e = fl(p1 - p0) is off by u|e| per component; each component of
    m = e1 x e2 (two products and a difference) by at most
    5u (|e1a e2b| + |e1b e2a|), so |dm| <= 15u |e1||e2|; normalising adds 5u,
    so |n32 - n| <= 30u cond + 5u with cond = |e1||e2| / |e1 x e2| = 1/sin;
    d = -fl(n.p0) adds 3u |p0|.  At a point p the residuals then differ by at
    most |n32 - n| (|p| + |p0|) + |d32 - d| <=
    u ((30 cond + 5)(pmax + |p0|) + 4 |p0|)."""
    X = P.reshape(3, -1)
    eps = np.full(len(planes_or), 0.0)
    for j, t in enumerate(triples):
        if t[0] < 0:
            continue
        p0, p1, p2 = (X[:, L[k]] for k in t)
        e1, e2 = p1 - p0, p2 - p0
        l1, l2 = np.linalg.norm(e1), np.linalg.norm(e2)
        m = np.linalg.norm(np.cross(e1, e2))
        if m <= 0 or l1 <= 0 or l2 <= 0:
            continue
        cond = l1 * l2 / m
        n0 = np.linalg.norm(p0)
        eps[j] = EPS32 * ((30.0 * cond + 5.0) * (pmax + n0) + 4.0 * n0)
    return eps


def score_margin(hyps32, p1max):
    """Band around t inside which the canonical FP32 residual
    fmaf(nx, x, fmaf(ny, y, fmaf(nz, z, d))) may fall on the other side of t
    than the exact residual of the same FP32 plane: three roundings, each at
    most u (|d| + |x|+|y|+|z|) since |n_i| <= 1; 16u (P1 + |d|) is the margin
    the culled scorer itself keeps (P1 = max |x|+|y|+|z| over the frame)."""
    d = np.abs(np.nan_to_num(np.asarray(hyps32, np.float64)[:, 3]))
    return 16.0 * EPS32 * (p1max + d)


def labels_explained(P_g, P_o, lab_g, lab_o, planes_g, planes_o, t, band=1e-6):
    """Free-running labels against the oracle's (R20): every pixel whose
    label differs must be near t for the plane of the first round that
    claimed it on either side, k = min(lab_g, lab_o): its oracle residual
    (oracle plane k, oracle point) within `band` of t, or on the other side
    of t from the GPU's residual (GPU plane k, GPU point) -- the two sides'
    planes and points are both legitimate and agree to their own tolerances
    (planes 1e-6 relative, points 2e-6 m), so between them they may split a
    pixel lying that close to t.  Returns (number of differing pixels,
    largest band used)."""
    Xg = np.asarray(P_g, np.float64).reshape(3, -1)
    Xo = np.asarray(P_o, np.float64).reshape(3, -1)
    lg = np.asarray(lab_g).reshape(-1).astype(np.int64)
    lo = np.asarray(lab_o).reshape(-1).astype(np.int64)
    diff = np.flatnonzero(lg != lo)
    if diff.size == 0:
        return 0, 0.0
    big = 1 << 20
    k = np.minimum(np.where(lg[diff] >= 0, lg[diff], big), np.where(lo[diff] >= 0, lo[diff], big))
    assert np.all(k < min(len(planes_g), len(planes_o))), "a differing pixel lies beyond the common planes"
    used = 0.0
    for i, kk in zip(diff, k):
        po, pg = np.asarray(planes_o[kk], np.float64), np.asarray(planes_g[kk], np.float64)
        ro = abs(po[:3] @ Xo[:, i] + po[3])
        rg = abs(pg[:3] @ Xg[:, i] + pg[3])
        allow = band + abs(rg - ro)
        assert abs(ro - t) <= allow, (int(i), int(kk), ro, rg)
        used = max(used, allow)
    return int(diff.size), used


def check_removal(points, labels, valid, planes, t, min_inliers, hyps, band=1e-6):
    """Invariants of sequential removal (Alg. 2) in float64 for one frame:
    points [3][H][W], labels [H][W] int8 (-1 none), valid [H][W] 0/1, planes as
    dicts with n, d, inliers, hyp_index in emission order.  Pixels within
    `band` of t are exempt: the path decides them in compensated FP32 against
    the FP64 plane."""
    X = np.asarray(points, np.float64).reshape(3, -1)
    lab = np.asarray(labels).reshape(-1)
    val = np.asarray(valid).reshape(-1) > 0
    assert np.all(lab[~val] == -1) and np.all(lab < len(planes))
    earlier_far = np.ones(X.shape[1], bool)  # at least t from every plane so far
    for r, pl in enumerate(planes):
        dist = np.abs(np.asarray(pl["n"]) @ X + pl["d"])
        decided = np.abs(dist - t) > band
        mine = lab == r
        assert pl["inliers"] == mine.sum() >= min_inliers, r
        assert 0 <= pl["hyp_index"] < hyps, r
        assert np.all(dist[mine & decided] < t), r
        assert not np.any(mine & ~earlier_far), r
        earlier_far &= (dist >= t) | ~decided
    assert not np.any(val & (lab == -1) & ~earlier_far)
