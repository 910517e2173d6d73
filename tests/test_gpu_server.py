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
