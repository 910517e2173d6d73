"""The seeded scene generator: deterministic, holes and noise as configured,
labels consistent with the depth image."""
import numpy as np
import pytest

import scenes


@pytest.mark.parametrize("cid,k", [(1, 0), (2, 1), (3, 2), (4, 1)])
def test_frames_are_deterministic(cid, k):
    a = scenes.make_frame(cid, k)
    b = scenes.make_frame(cid, k)
    assert np.array_equal(a.depth, b.depth) and np.array_equal(a.gt_labels, b.gt_labels)
    c = scenes.make_frame(cid, k + 1)
    assert not np.array_equal(a.depth, c.depth)


@pytest.mark.parametrize("cid", [1, 2, 3])
def test_holes_labels_and_noise(cid):
    cfg = scenes.CONFIGS[cid]
    f = scenes.make_frame(cid, 0)
    W, H = cfg.sizes[0]
    assert f.depth.shape == (H, W) and f.depth.dtype == np.uint16
    hit = f.depth_m > 0
    dropped = hit & (f.depth == 0)
    assert abs(dropped.sum() / f.depth.size - cfg.hole_frac) < 0.01
    assert np.array_equal(f.gt_labels >= 0, f.depth > 0)
    assert f.depth_m.max() <= scenes.MAX_RANGE_M
    v = f.depth > 0
    err = f.depth[v].astype(float) - 1000.0 * f.depth_m[v]
    sig = cfg.sigma if cfg.noise == "const" else 1000.0 * cfg.sigma * f.depth_m[v] ** 2
    z = err / sig
    assert abs(z.mean()) < 0.05 and 0.9 < z.std() < 1.1


def test_noise_free_variant_rounds_only():
    f = scenes.make_frame(2, 0, noise="none", hole_frac=0.0)
    v = f.depth_m > 0
    assert np.all(f.depth[v] == np.rint(1000.0 * f.depth_m[v]))
    assert np.all(f.depth[~v] == 0)


def test_spiral_scene_has_many_planes_and_the_column():
    f = scenes.make_frame(3, 1)
    lab = f.gt_labels
    names = f.meta["patch_names"]
    present = {names[i] for i in np.unique(lab[lab >= 0])}
    assert "floor" in present and sum(n.startswith("tread") for n in present) >= 3
