"""pp_ransac_planes_noalloc: sequential RANSAC on the library's static per-GPU
scratch, with no context and no device allocation.

- Two calls in a row, the second on a smaller frame (640x480 with 1024
  hypotheses, then 160x120 with 256), each give the same planes, plane count
  and labels as pp_ransac_planes on a context at the same (default) tuning,
  bitwise: the same kernels run on the same inputs, and the second call's
  results do not depend on what the first left in the shared array.
- The matrix-core scoring form through the same entry point equals its
  context counterpart too.
- A frame whose scratch exceeds the array's size is refused with
  PP_E_INVAL and a message, before any work; so are bad arguments.
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


def _inputs(pp, cid, k, ctx):
    f = scenes.make_frame(cid, k)
    H, W = f.depth.shape
    dc, rc = cfg_params(cid, W, H, k)
    K = f.K
    dmm = pp.diffuse(to_dev(f.depth), dc.iters, dc.lam, dc.kappa_mm, dc.edge_stop, ctx=ctx)
    pts, _, valid = pp.normals(dmm, (K.fx, K.fy, K.cx, K.cy), ctx=ctx)
    return pts, valid, rc


def _host(planes, n, labels):
    import torch
    torch.cuda.synchronize()
    k = int(n.cpu().item())
    return k, planes.cpu().numpy()[:64 * k].copy(), labels.cpu().numpy().copy()


def _check_equal(got, want, what):
    assert got[0] == want[0], f"{what}: {got[0]} planes, context path {want[0]}"
    assert np.array_equal(got[1], want[1]), f"{what}: plane records differ"
    diff = int((got[2] != want[2]).sum())
    assert diff == 0, f"{what}: {diff} labels differ"


def _alloc_outputs(pp, pts, rc):
    import torch
    _, H, W = pts.shape
    planes = torch.full((rc.max_planes * pp.PLANE_BYTES,), 0xAB, dtype=torch.uint8, device=pts.device)
    n = torch.full((1,), -7, dtype=torch.int32, device=pts.device)
    labels = torch.full((H, W), 99, dtype=torch.int8, device=pts.device)
    return planes, n, labels


def test_noalloc_equals_the_context_path_on_two_calls_the_second_smaller(pp):
    ctx = pp.Context(0)
    cases = [(2, 0), (1, 1)]  # 640x480 x 1024 hypotheses, then 160x120 x 256
    inputs = [_inputs(pp, cid, k, ctx) for cid, k in cases]
    want = []
    for pts, valid, rc in inputs:
        want.append(_host(*pp.ransac_planes(pts, valid, rc, ctx=ctx)))
    outs = [_alloc_outputs(pp, pts, rc) for pts, _, rc in inputs]  # allocated before the calls
    for (cid, k), (pts, valid, rc), o, w in zip(cases, inputs, outs, want):
        log(f"noalloc: config {cid} frame {k}, {tuple(pts.shape)}, {rc.hyps} hypotheses")
        got = _host(*pp.ransac_planes_noalloc(pts, valid, rc, *o))
        assert got[0] >= 1
        _check_equal(got, w, f"config {cid} frame {k}")
    # and once more on the larger frame after the smaller one
    pts, valid, rc = inputs[0]
    o = _alloc_outputs(pp, pts, rc)
    _check_equal(_host(*pp.ransac_planes_noalloc(pts, valid, rc, *o)), want[0], "640x480 again")
    ctx.close()


def test_noalloc_matrix_core_form_equals_the_context_path(pp):
    ctx = pp.Context(0)
    pts, valid, rc = _inputs(pp, 2, 3, ctx)
    rc.precision, rc.recheck_band_m = pp.PP_SCORE_BF16, 0.002
    want = _host(*pp.ransac_planes(pts, valid, rc, ctx=ctx))
    got = _host(*pp.ransac_planes_noalloc(pts, valid, rc, *_alloc_outputs(pp, pts, rc)))
    _check_equal(got, want, "bf16 form")
    ctx.close()


def test_noalloc_refuses_frames_beyond_its_scratch_and_bad_arguments(pp):
    import torch
    from paper_2411_01919_amd import _native as N
    W, H = 2048, 2048  # about 191 MB of scratch at 45.6 bytes a pixel
    pts = torch.zeros((3, H, W), dtype=torch.float32, device="cuda:0")
    valid = torch.zeros((H, W), dtype=torch.uint8, device="cuda:0")
    _, rc = cfg_params(2, W, H)
    o = _alloc_outputs(pp, pts, rc)
    with pytest.raises(pp.PPError) as ei:
        pp.ransac_planes_noalloc(pts, valid, rc, *o)
    assert ei.value.status == N.PP_E_INVAL and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert int(o[1].cpu().item()) == -7  # nothing ran
    small = torch.zeros((3, 8, 8), dtype=torch.float32, device="cuda:0")
    sv = torch.zeros((8, 8), dtype=torch.uint8, device="cuda:0")
    _, rc = cfg_params(1, 8, 8)
    rc.hyps = 0
    with pytest.raises(pp.PPError) as ei:
        pp.ransac_planes_noalloc(small, sv, rc, *_alloc_outputs(pp, small, rc))
    assert ei.value.status == N.PP_E_INVAL
