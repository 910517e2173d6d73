"""Frames stored with a row pitch wider than the image (pitch_px > width).

Every step reads only the first `width` pixels of each row, so a frame stored
with padding columns (filled here with plausible depths that would change the
result if read) gives bitwise the results of the same frame stored densely:
diffused depth, points, normals and valid flags on the image columns, the
planes, and the labels.  Odd pitches misalign the rows for word-wide loads,
even ones keep them aligned; both forms are covered, on the plain calls and
on one ragged batch.
"""
import ctypes

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


def _padded(depth, pitch, seed):
    H, W = depth.shape
    out = np.random.default_rng(seed).integers(800, 4000, (H, pitch)).astype(np.uint16)
    out[:, :W] = depth
    return out


def _buffers(H, pitch, rc):
    import torch
    import paper_2411_01919_amd as pp
    dev = torch.device("cuda:0")
    return dict(depth_mm=torch.full((H, pitch), -7.0, dtype=torch.float32, device=dev),
                points=torch.full((3, H, pitch), -7.0, dtype=torch.float32, device=dev),
                normals=torch.full((3, H, pitch), -7.0, dtype=torch.float32, device=dev),
                valid=torch.full((H, pitch), 0xEE, dtype=torch.uint8, device=dev),
                planes=torch.zeros((rc.max_planes * pp.PLANE_BYTES,), dtype=torch.uint8, device=dev),
                n_planes=torch.zeros((1,), dtype=torch.int32, device=dev),
                labels=torch.full((H, pitch), 77, dtype=torch.int8, device=dev))


def _host(b, W, pp):
    n = int(b["n_planes"].cpu().item())
    return dict(depth_mm=b["depth_mm"].cpu().numpy()[:, :W], points=b["points"].cpu().numpy()[:, :, :W],
                normals=b["normals"].cpu().numpy()[:, :, :W], valid=b["valid"].cpu().numpy()[:, :W],
                labels=b["labels"].cpu().numpy()[:, :W], n=n, planes=b["planes"].cpu().numpy().tobytes())


def _plain(pp, depth_padded, W, K, dc, rc):
    """pp_diffuse -> pp_normals -> pp_ransac_planes on a [H][pitch] frame."""
    import torch
    N = pp._native
    H, pitch = depth_padded.shape
    ctx = pp.default_context(0)
    d = to_dev(depth_padded)
    b = _buffers(H, pitch, rc)
    desc = N.FrameDesc(W, H, pitch)
    p_d, p_r = dc.c(), rc.c()
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    ctx.check(N.lib().pp_diffuse(ctx.h, ptr(d), ptr(b["depth_mm"]), desc, ctypes.byref(p_d), None))
    ctx.check(N.lib().pp_normals(ctx.h, ptr(b["depth_mm"]), desc, N.Intrinsics(K.fx, K.fy, K.cx, K.cy),
                                 ptr(b["points"]), ptr(b["normals"]), ptr(b["valid"]), None))
    ctx.check(N.lib().pp_ransac_planes(ctx.h, ptr(b["points"]), ptr(b["valid"]), None, desc, ctypes.byref(p_r),
                                       ptr(b["planes"]), ptr(b["n_planes"]), ptr(b["labels"]), None))
    torch.cuda.synchronize()
    return _host(b, W, pp)


def _same(a, b, what):
    for key in ("depth_mm", "points", "normals", "valid", "labels"):
        assert np.array_equal(a[key], b[key]), f"{what}: {key} differs"
    assert a["n"] == b["n"], f"{what}: plane counts {a['n']} != {b['n']}"
    assert a["planes"] == b["planes"], f"{what}: plane records differ"


@pytest.mark.parametrize("cid,k,extra", [(1, 0, 13), (1, 1, 16), (2, 0, 1), (2, 1, 16)])
def test_pitched_frame_equals_the_dense_frame(pp, cid, k, extra):
    f = scenes.make_frame(cid, k)
    H, W = f.depth.shape
    log(f"pitched frame cfg={cid} k={k} {W}x{H} pitch={W + extra}")
    dc, rc = cfg_params(cid, W, H, k)
    dense = _plain(pp, f.depth, W, f.K, dc, rc)
    pitched = _plain(pp, _padded(f.depth, W + extra, 7 * cid + k), W, f.K, dc, rc)
    assert dense["n"] >= 1
    _same(pitched, dense, f"cfg {cid} frame {k} pitch {W + extra}")


def test_pitched_ragged_batch_equals_dense_plain_frames(pp):
    """One pp_batch_run over frames of two sizes with odd and even pitches."""
    import torch
    N = pp._native
    cases = [(1, 0, 5), (2, 0, 16), (1, 2, 0), (2, 1, 3)]
    log("pitched ragged batch " + " ".join(f"cfg{c}/k{k}/+{e}" for c, k, e in cases))
    jobs, keep, refs, widths = [], [], [], []
    for cid, k, extra in cases:
        f = scenes.make_frame(cid, k)
        H, W = f.depth.shape
        dc, rc = cfg_params(cid, W, H, k)
        refs.append(_plain(pp, f.depth, W, f.K, dc, rc))
        d = to_dev(_padded(f.depth, W + extra, 11 * cid + k))
        b = _buffers(H, W + extra, rc)
        keep.append((d, b))
        widths.append(W)
        ptr = lambda t: t.data_ptr()
        jobs.append(N.FrameJob(ptr(d), N.FrameDesc(W, H, W + extra), N.Intrinsics(f.K.fx, f.K.fy, f.K.cx, f.K.cy),
                               dc.c(), rc.c(), ptr(b["depth_mm"]), ptr(b["points"]), ptr(b["normals"]),
                               ptr(b["valid"]), ptr(b["planes"]), ptr(b["n_planes"]), ptr(b["labels"])))
    arr = (N.FrameJob * len(jobs))(*jobs)
    ctx = pp.default_context(0)
    for fn in (N.lib().pp_batch_run_eager, N.lib().pp_batch_run):
        ctx.check(fn(ctx.h, len(jobs), arr, None))
        torch.cuda.synchronize()
        for (cid, k, extra), (_, b), W, ref in zip(cases, keep, widths, refs):
            _same(_host(b, W, pp), ref, f"batch cfg {cid} frame {k} pitch +{extra}")
