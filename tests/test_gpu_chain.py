"""The paper's whole per-frame chain on the GPU (diffusion, normals,
segmentation, region-mode RANSAC) feeding the host polygons and the drift-
compensated map, over a walk along the straight staircase whose reported
camera height drifts: the drift estimate follows the injected drift and the
mapped treads sit at their true heights.  (A validity check: the stages
themselves are compared with the oracle in the other GPU tests.)"""
import numpy as np
import pytest

import scenes
from gpu_util import log, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_01919_amd as pp
    pp.default_context(0)
    return pp


def test_chain_tracks_vertical_drift(pp):
    m = pp.DriftMap(0.05, 1e-4, 1e-5, 15.0)
    errs = []
    times = {}
    for k in range(12):
        f = scenes.make_frame(2, k)
        R, C = f.pose
        drift = 0.008 * k
        out = pp.paper_chain(to_dev(f.depth), (f.K.fx, f.K.fy, f.K.cx, f.K.cy), m, (R, C + np.array([0, 0, drift])),
                             seed=11, frame_id=k, times=times)
        r = out["map"]
        log(f"  frame {k}: {out['n_regions']} regions, {len(out['planes'])} planes, matched {r['matched']}, "
            f"drift {r['drift'] * 100:.2f} cm (true {drift * 100:.2f})")
        if k >= 3:
            errs.append(abs(r["drift"] - drift))
    log(f"  per-frame ms (12 frames): { {k: round(v / 12, 3) for k, v in times.items()} }")
    assert max(errs) < 0.01
    heights = [p["height"] for p in m.polygons() if p["support"] > 20000]
    true = [0.15 * i for i in range(9)]
    assert len(heights) >= 4
    assert all(min(abs(h - t) for t in true) < 0.015 for h in heights), heights
