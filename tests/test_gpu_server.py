"""The serving runtime on the GPU: results served in a mix of camera streams
(different sizes, bursts, several lanes, admission under a tight budget) are
bitwise the same as the plain per-frame path, alone."""
import time

import numpy as np
import pytest

import scenes
from gpu_util import cfg_params, log, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_01919_amd as pp
    pp.default_context(0)
    return pp


def _plain(pp, f, cid, k):
    import torch
    H, W = f.depth.shape
    dc, rc = cfg_params(cid, W, H, k)
    fo = pp.make_outputs(to_dev(f.depth), (f.K.fx, f.K.fy, f.K.cx, f.K.cy), dc, rc)
    pp.run_frame(fo)
    torch.cuda.synchronize()
    n = int(fo.n_planes.cpu().item())
    return n, fo.planes.cpu().numpy().tobytes()[:n * pp.PLANE_BYTES], fo.labels.cpu().numpy()


@pytest.mark.parametrize("use_graphs", [True, False])
def test_served_results_equal_the_plain_path(pp, use_graphs):
    cams = [(1, 160, 120), (3, 424, 240), (2, 640, 480), (3, 640, 480), (4, 1280, 720)]
    frames = {}
    for sid, (cid, W, H) in enumerate(cams):
        frames[sid] = [scenes.make_frame(cid, k, size=(W, H)) for k in range(3)]
    # budget for about three 640x480 frames at once: admission must hold frames back
    srv = pp.Server(hbm_budget_bytes=160 << 20, max_batch=8, lanes=3, staging_frames=16, use_graphs=use_graphs)
    for sid, (cid, W, H) in enumerate(cams):
        dc, rc = cfg_params(cid, W, H, 0)
        f0 = frames[sid][0]
        srv.open_stream(sid, W, H, (f0.K.fx, f0.K.fy, f0.K.cx, f0.K.cy), dc, rc)
    tickets = []
    for rep in range(2):  # two bursts over every stream
        for sid in range(len(cams)):
            for k, f in enumerate(frames[sid]):
                tickets.append((sid, k, srv.submit(sid, f.depth, k)))
        time.sleep(0.01)
    got = {}
    t0 = time.time()
    while len(got) < len(tickets) and time.time() - t0 < 120:
        for sid, k, t in tickets:
            if t in got:
                continue
            r = srv.poll(t, sid, timeout_us=5000)
            if r is not None:
                got[t] = r
    assert len(got) == len(tickets)
    st = srv.stats()
    log(f"  served {st['completed']} frames in {st['launches']} launches (mean batch {st['mean_batch']:.2f}), "
        f"p50 {st['p50_us'] / 1e3:.2f} ms p99 {st['p99_us'] / 1e3:.2f} ms, arena peak {st['hbm_peak'] >> 20} MiB")
    assert st["hbm_peak"] <= 160 << 20
    for sid, k, t in tickets:
        cid = cams[sid][0]
        n, planes, labels = _plain(pp, frames[sid][k], cid, k)
        r = got[t]
        assert r["n_planes"] == n, (sid, k)
        assert r["planes"][:len(planes)] == planes, (sid, k)
        assert np.array_equal(r["labels"], labels), (sid, k)
    srv.close()


def test_served_frames_match_the_oracle(pp, orc):
    """Frames of a 160x120 camera served in a mix with a 640x480 camera and
    a tight budget: every served plane equals the float64 oracle pipeline's
    to 1e-6 relative and every label is the oracle's except near t (the
    same check as the plain path's free-running test)."""
    import torch
    from gpu_util import labels_explained
    small = [scenes.make_frame(1, k) for k in range(4)]
    big = [scenes.make_frame(2, k) for k in range(2)]
    srv = pp.Server(hbm_budget_bytes=96 << 20, max_batch=4, lanes=2, staging_frames=16, use_graphs=True)
    for sid, fr in ((0, small[0]), (1, big[0])):
        H, W = fr.depth.shape
        dc, rc = cfg_params(1 if sid == 0 else 2, W, H, 0)
        srv.open_stream(sid, W, H, (fr.K.fx, fr.K.fy, fr.K.cx, fr.K.cy), dc, rc)
    tickets = []
    for k in range(4):
        tickets.append((0, k, srv.submit(0, small[k].depth, k)))
        tickets.append((1, k, srv.submit(1, big[k % 2].depth, k)))
    got = {}
    t0 = time.time()
    while len(got) < len(tickets) and time.time() - t0 < 120:
        for sid, k, t in tickets:
            if t not in got:
                r = srv.poll(t, sid, timeout_us=5000)
                if r is not None:
                    got[t] = r
    assert len(got) == len(tickets)
    srv.close()
    for sid, k, t in tickets:
        if sid != 0:
            continue
        f = small[k]
        H, W = f.depth.shape
        dc, rc = cfg_params(1, W, H, k)
        prm = orc.RansacParams(rc.hyps, rc.max_planes, rc.min_inliers, rc.thresh_m, rc.seed, rc.frame_id)
        o = orc.pipeline(f.depth, f.K, dc.iters, dc.lam, dc.kappa_mm, prm)
        r = got[t]
        planes = pp.planes_to_numpy(torch.frombuffer(bytearray(r["planes"]), dtype=torch.uint8), r["n_planes"])
        assert r["n_planes"] == o.ransac.n_planes, (k, r["n_planes"], o.ransac.n_planes)
        pg = []
        for i in range(r["n_planes"]):
            g = np.append(planes[i]["n"], planes[i]["d"])
            assert np.max(np.abs(g - o.ransac.planes[i])) <= 1e-6 * max(1.0, o.ransac.planes[i][3]), (k, i)
            pg.append(g)
        # the served frame's points are the plain path's (the served results are bitwise the plain ones)
        dmm = pp.diffuse(to_dev(f.depth), dc.iters, dc.lam, dc.kappa_mm)
        pts, _, _ = pp.normals(dmm, (f.K.fx, f.K.fy, f.K.cx, f.K.cy))
        ndiff, used = labels_explained(pts.cpu().numpy(), o.P, r["labels"], o.ransac.labels, pg, o.ransac.planes,
                                       rc.thresh_m)
        log(f"  served 160x120 frame {k}: {r['n_planes']} planes as the oracle's, {ndiff} labels differ "
            f"(each within {used:.1e} m of t)")
