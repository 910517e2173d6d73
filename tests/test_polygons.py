"""The library's contour polygons (host code behind the C ABI, no GPU needed)
equal the oracle's vertex for vertex, on the oracle's segmentations of the
rendered scenes, on random blobs, and with a pitch wider than the image."""
import numpy as np
import pytest
from scipy import ndimage

import paper_2411_01919_amd as pp
import scenes
from paper_2411_01919_amd import _native as N


def _same(a, b):
    assert len(a) == len(b)
    for g, (p, q) in enumerate(zip(a, b)):
        assert np.array_equal(p, q), g


@pytest.mark.parametrize("cid,k,eps", [(1, 0, 1.0), (2, 0, 1.5), (2, 3, 0.0), (3, 1, 2.5)])
def test_scene_polygons_equal_the_oracle(orc, cid, k, eps):
    f = scenes.make_frame(cid, k)
    cfg = scenes.CONFIGS[cid]
    P, valid = orc.backproject(orc.diffuse(f.depth, cfg.diffuse_iters, cfg.lam, cfg.kappa_mm), f.K)
    Nrm, nvalid = orc.normals(P, valid)
    H, W = f.depth.shape
    reg, n, _ = orc.segment(Nrm.astype(np.float32), nvalid, 0.35, 0.7, max(50, -(-2 * W * H // 1000)), 127)
    assert n > 0
    _same(pp.region_polygons(reg, n, eps), orc.region_polygons(reg, n, eps))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_blob_polygons_equal_the_oracle(orc, seed):
    rng = np.random.default_rng(seed)
    blob = rng.random((61, 83)) < 0.58
    lab, n = ndimage.label(blob, structure=[[0, 1, 0], [1, 1, 1], [0, 1, 0]])
    reg = (lab - 1).astype(np.int16)
    for eps in (0.0, 0.8, 3.0):
        _same(pp.region_polygons(reg, n, eps), orc.region_polygons(reg, n, eps))


def test_pitch_and_buffer_size(orc):
    reg = np.full((20, 30), -1, np.int16)
    reg[2:9, 3:12] = 0
    reg[11:18, 14:27] = 1
    padded = np.full((20, 40), 7, np.int16)
    padded[:, :30] = reg
    off = np.zeros(3, np.int32)
    xy = np.zeros((3, 2), np.int32)
    st = N.lib().pp_region_polygons(padded.ctypes.data, N.FrameDesc(30, 20, 40), 2, 0.5, xy.ctypes.data, 3,
                                    off.ctypes.data)
    assert st == N.PP_E_NOMEM and off[2] == 8
    xy = np.zeros((8, 2), np.int32)
    st = N.lib().pp_region_polygons(padded.ctypes.data, N.FrameDesc(30, 20, 40), 2, 0.5, xy.ctypes.data, 8,
                                    off.ctypes.data)
    assert st == N.PP_OK
    want = orc.region_polygons(reg, 2, 0.5)
    assert np.array_equal(xy[off[0]:off[1]], want[0]) and np.array_equal(xy[off[1]:off[2]], want[1])
    assert N.lib().pp_region_polygons(None, N.FrameDesc(30, 20, 40), 2, 0.5, None, 0, off.ctypes.data) == N.PP_E_INVAL
