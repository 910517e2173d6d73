"""One context used from two streams, and the context's bounded graph cache.

- The plain per-frame calls of several frames alternate between two streams
  on one context with no host synchronisation between them: each call on a
  stream other than the previous call's waits for the previous call's work
  (the frame table and scratch are shared), so every result equals the one
  of the same calls on a single stream, bitwise.
- Batch layouts beyond the cache's 64 graphs evict the least recently used
  one; replaying every layout again (some re-captured) gives the same
  results as eager launches.
"""
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
    return pp


def _outs(pp, frames, cid):
    outs = []
    for f in frames:
        H, W = f.depth.shape
        dc, rc = cfg_params(cid, W, H, f.meta["k"])
        outs.append(pp.make_outputs(to_dev(f.depth), (f.K.fx, f.K.fy, f.K.cx, f.K.cy), dc, rc))
    return outs


def _host(fo):
    n = int(fo.n_planes.cpu().item())
    return (fo.depth_mm.cpu().numpy(), fo.points.cpu().numpy(), fo.valid.cpu().numpy(), fo.labels.cpu().numpy(),
            n, fo.planes.cpu().numpy()[:64 * n])


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def test_plain_calls_alternating_between_two_streams_on_one_context(pp):
    import torch
    frames = [scenes.make_frame(3, k) for k in range(6)]  # 424x240, 640x480, 848x480, ...
    ref = _outs(pp, frames, 3)
    ctx = pp.Context(0)
    for fo in ref:
        pp.run_frame(fo, ctx=ctx)
    torch.cuda.synchronize()
    want = [_host(fo) for fo in ref]
    got = _outs(pp, frames, 3)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for i, fo in enumerate(got):
        # the three calls of one frame on alternating streams, no host wait in between
        H, W = fo.depth.shape
        a, b = (s1, s2) if i % 2 == 0 else (s2, s1)
        pp.diffuse(fo.depth, fo.diffuse.iters, fo.diffuse.lam, fo.diffuse.kappa_mm, out=fo.depth_mm, ctx=ctx,
                   stream=a)
        pp.normals(fo.depth_mm, fo.K, fo.points, fo.normals, fo.valid, ctx=ctx, stream=b)
        pp.ransac_planes(fo.points, fo.valid, fo.ransac, fo.planes, fo.n_planes, fo.labels, ctx=ctx, stream=a)
    torch.cuda.synchronize()
    for i, fo in enumerate(got):
        assert _same(_host(fo), want[i]), i
    log(f"  {len(got)} frames over two streams: bitwise the single-stream results")
    ctx.close()


def test_graph_cache_evicts_beyond_its_bound_and_results_stay_equal(pp):
    import torch
    frames = [scenes.make_frame(1, k) for k in range(70)]
    outs = _outs(pp, frames, 1)
    ctx = pp.Context(0)
    eager = {}
    for n in range(1, 67):  # 66 batch sizes: 66 layouts
        pp.batch_run(outs[:n], graph=False, ctx=ctx)
        torch.cuda.synchronize()
        eager[n] = [_host(fo) for fo in outs[:n]]
    for rep in range(2):
        for n in range(1, 67):
            for fo in outs[:n]:
                fo.labels.fill_(7)
                fo.n_planes.fill_(-3)
            pp.batch_run(outs[:n], graph=True, ctx=ctx)
            torch.cuda.synchronize()
            got = [_host(fo) for fo in outs[:n]]
            assert all(_same(a, b) for a, b in zip(got, eager[n])), (rep, n)
    log("  66 layouts through a 64-graph cache, twice: every replay equals the eager launches")
    ctx.close()
