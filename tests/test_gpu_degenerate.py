"""Degenerate inputs of the method, through the whole path on the GPU, against
closed forms and the oracle.

- Every point on one 3-D line: one image row of constant depth, holes
  elsewhere.  Diffusion keeps the row constant, the row back-projects to
  points with equal y and z, so every triple is collinear and no hypothesis
  of round 0 is valid (Alg. 2 draws three points that must span a plane).
  No plane is emitted, every label stays -1, and the oracle draws the same
  triples and finds none of them valid either.
- Every point on one plane: constant depth over the whole image.  The first
  round's refit is exactly the plane z = depth (n = (0, 0, -1), d = depth in
  metres, d >= 0 by the sign rule), every pixel is its inlier, and no second
  round runs because no point is left.
"""
from types import SimpleNamespace

import numpy as np
import pytest

import scenes
from gpu_util import cfg_params, log, run_plain

pytestmark = pytest.mark.gpu

H, W = 61, 97


@pytest.fixture(scope="module")
def pp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_01919_amd as pp
    pp.default_context(0)
    return pp


def _frame(depth):
    return SimpleNamespace(depth=depth, K=scenes.Intrinsics(100.0, 100.0, W / 2.0, H / 2.0))


@pytest.mark.parametrize("row", [0, 30, H - 1])
def test_collinear_points_give_no_valid_hypothesis(pp, orc, row):
    log(f"collinear points: row {row} of a {W}x{H} frame")
    depth = np.zeros((H, W), np.uint16)
    depth[row, :] = 1500
    dc, rc = cfg_params(1, W, H, 0)
    g = run_plain(_frame(depth), dc, rc)
    assert np.all(g["depth_mm"][row] == 1500.0) and np.all(g["depth_mm"][np.arange(H) != row] == 0.0)
    assert g["n_planes"] == 0
    assert np.all(g["labels"] == -1)
    dbg = g["dbg"]
    assert dbg["n_valid"][0] == W
    info = dbg["round_info"]
    assert info[0][3] == 1 and info[0][0] == -1  # no valid hypothesis
    assert np.all(info[1:, 3] == -1)  # nothing after it ran
    assert np.all(np.isnan(dbg["hyps"][0][:, 3]))
    # the oracle draws the same triples and finds every one degenerate
    P = g["points"].astype(np.float64)
    valid = g["valid"] & 1
    L = orc.valid_list(valid)
    prm = orc.RansacParams(rc.hyps, rc.max_planes, rc.min_inliers, rc.thresh_m, rc.seed, rc.frame_id)
    tr_o, _, hv_o = orc.hypotheses(P, L, np.zeros_like(valid), prm, 0)
    assert not hv_o.any()
    assert np.array_equal(dbg["triples"][0], tr_o)


@pytest.mark.parametrize("z_mm", [500, 1500, 4000])
def test_one_plane_is_found_exactly_with_every_pixel(pp, z_mm):
    log(f"one plane: constant depth {z_mm} mm over {W}x{H}")
    depth = np.full((H, W), z_mm, np.uint16)
    dc, rc = cfg_params(1, W, H, 0)
    g = run_plain(_frame(depth), dc, rc)
    assert np.all(g["depth_mm"] == float(z_mm))
    assert g["n_planes"] == 1
    pl = g["planes"][0]
    assert np.abs(pl["n"] - np.array([0.0, 0.0, -1.0])).max() <= 1e-12
    assert abs(pl["d"] - z_mm / 1000.0) <= 1e-12
    assert abs(pl["centroid"][2] - z_mm / 1000.0) <= 1e-12
    assert pl["inliers"] == W * H
    assert np.all(g["labels"] == 0)
    info = g["dbg"]["round_info"]
    assert info[0][3] == 0 and info[0][2] == W * H
    assert np.all(info[1:, 3] == -1)
