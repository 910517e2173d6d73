"""Pin of the oracle's valid list (the fixed per-frame point set Alg. 2
samples from): the row-major positions of the depth-valid pixels, checked
against numpy's own flat-index search on random masks, the edge cases, and
on a frame's back-projection, where each listed position must hold a point
with positive depth and the positions must be strictly increasing."""
import numpy as np
import pytest

import scenes


@pytest.mark.parametrize("H,W,frac", [(1, 1, 0.5), (3, 3, 0.5), (7, 13, 0.3), (64, 64, 0.98), (97, 61, 0.02),
                                      (480, 640, 0.98)])
def test_valid_list_is_flatnonzero(orc, H, W, frac):
    rng = np.random.default_rng(H * 1000 + W)
    v = (rng.random((H, W)) < frac).astype(np.uint8)
    L = orc.valid_list(v)
    assert L.dtype == np.int32
    assert np.array_equal(L, np.flatnonzero(v))


def test_valid_list_edge_cases(orc):
    z = np.zeros((5, 7), np.uint8)
    assert orc.valid_list(z).size == 0
    o = np.ones((5, 7), np.uint8)
    assert np.array_equal(orc.valid_list(o), np.arange(35))
    only = np.zeros((5, 7), np.uint8)
    only[0, 0] = only[4, 6] = 1
    assert np.array_equal(orc.valid_list(only), [0, 34])
    # row-major, not column-major: (row 0, col 2) precedes (row 1, col 0)
    rc = np.zeros((3, 4), np.uint8)
    rc[1, 0] = rc[0, 2] = 1
    assert np.array_equal(orc.valid_list(rc), [2, 4])
    # any non-zero byte counts as valid
    b = np.array([[0, 1, 2], [255, 0, 3]], np.uint8)
    assert np.array_equal(orc.valid_list(b), np.flatnonzero(b))


def test_valid_list_of_a_frame(orc):
    f = scenes.make_frame(1, 0)
    P, valid = orc.backproject(f.depth.astype(np.float64), f.K)
    L = orc.valid_list(valid)
    assert np.array_equal(L, np.flatnonzero(f.depth > 0))
    assert np.all(np.diff(L) > 0)
    assert np.all(P[2].reshape(-1)[L] > 0)
    assert len(L) == int((f.depth > 0).sum())
