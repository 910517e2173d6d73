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
    """Band inside which an FP32 hypothesis residual may legitimately sit on
    the other side of t than the float64 one: FP32 rounding of the three
    points' differences, of the cross product (amplified by the triple's
    conditioning 1/sin(angle) and lever arm pmax/|e|), and of the canonical
    residual evaluation."""
    X = P.reshape(3, -1)
    eps = np.full(len(planes_or), 1e-6)
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
        lever = pmax / min(l1, l2)
        eps[j] = 1e-6 + 64 * EPS32 * (pmax + abs(planes_or[j, 3])) * (1.0 + lever * cond)
    return eps


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
