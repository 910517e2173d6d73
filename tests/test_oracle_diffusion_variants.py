"""Pins of the oracle's diffusion variants beside the hot path's form: Alg. 1's
pixel-centred update as printed, and an 8-neighbour per-edge flux."""
import math

import numpy as np
import pytest

import scenes

PIXEL, EDGE8 = 1, 2


@pytest.mark.parametrize("scheme", [PIXEL, EDGE8])
def test_constant_image_is_a_fixed_point(orc, scheme):
    img = np.full((13, 17), 1500, np.uint16)
    img[np.random.default_rng(0).random(img.shape) < 0.15] = 0
    out = orc.diffuse_variant(img, 7, 0.15, 30.0, scheme)
    assert np.array_equal(out, img.astype(float))


def test_pixel_centred_form_is_not_conservative_but_edge_forms_are(orc):
    """The property that separates Alg. 1 as printed from the divergence form of Eq. 1."""
    f = scenes.make_frame(1, 0)
    s0 = f.depth.astype(float).sum()
    pix = orc.diffuse_variant(f.depth, 10, 0.2, 30.0, PIXEL)
    e8 = orc.diffuse_variant(f.depth, 10, 1 / 6, 30.0, EDGE8)
    assert abs(pix.sum() - s0) > 1e-6 * s0
    assert abs(e8.sum() - s0) <= 1e-12 * s0


def test_pixel_centred_form_reduces_to_the_heat_step_when_g_is_one(orc):
    """With kappa -> inf, c_p == 1 and Alg. 1's update is the 5-point heat step:
    the same closed-form mode decay as the per-edge form."""
    W, H, lam, N, k = 40, 9, 0.2, 15, 3
    u = np.arange(W)[None, :]
    img = 1000.0 + 40.0 * np.cos(math.pi * k * (u + 0.5) / W) * np.ones((H, 1))
    out = orc.diffuse_variant(img, N, lam, 1e30, PIXEL)
    fac = 1 - 4 * lam * math.sin(math.pi * k / (2 * W)) ** 2
    assert np.max(np.abs(out - (1000.0 + 40.0 * fac ** N * np.cos(math.pi * k * (u + 0.5) / W)))) < 1e-9
    assert np.max(np.abs(out - orc.diffuse(img, N, lam, 1e30))) < 1e-9


def test_maximum_principle(orc):
    f = scenes.make_frame(1, 2)
    v = f.depth > 0
    lo, hi = f.depth[v].min(), f.depth[v].max()
    for scheme, lam in [(PIXEL, 0.25), (EDGE8, 1 / 6)]:
        out = orc.diffuse_variant(f.depth, 12, lam, 30.0, scheme)
        assert out[v].min() >= lo - 1e-9 and out[v].max() <= hi + 1e-9


@pytest.mark.parametrize("a,b", [(1000, 1020), (1500, 1400)])
def test_diagonal_pair_isolates_weight_and_distance(orc, a, b):
    """Two valid pixels on a diagonal of a 2x2 image (the other two are holes):
    one step moves each by lam * 1/2 * g(|b-a| / sqrt 2) (b - a)."""
    lam, kappa = 0.15, 30.0
    img = np.array([[a, 0], [0, b]], np.uint16)
    out = orc.diffuse_variant(img, 1, lam, kappa, EDGE8)
    g = math.exp(-((abs(b - a) / math.sqrt(2) / kappa) ** 2))
    assert out[0, 0] == pytest.approx(a + lam * 0.5 * g * (b - a), abs=1e-12)
    assert out[1, 1] == pytest.approx(b - lam * 0.5 * g * (b - a), abs=1e-12)
    assert out[0, 1] == 0.0 and out[1, 0] == 0.0


def test_pixel_centred_gradient_uses_central_differences(orc):
    """A 1x3 row a, b, c: the middle pixel's c_p uses |c - a| / 2; the ends use
    one-sided differences; the update is lam c_p times the 2-neighbour Laplacian."""
    lam, kappa = 0.2, 30.0
    a, b, c = 1000.0, 1010.0, 1050.0
    out = orc.diffuse_variant(np.array([[a, b, c]]), 1, lam, kappa, PIXEL)
    g = lambda x: math.exp(-((x / kappa) ** 2))
    assert out[0, 1] == pytest.approx(b + lam * g(abs(c - a) / 2) * ((a - b) + (c - b)), abs=1e-12)
    assert out[0, 0] == pytest.approx(a + lam * g(abs(b - a)) * (b - a), abs=1e-12)
    assert out[0, 2] == pytest.approx(c + lam * g(abs(c - b)) * (b - c), abs=1e-12)


@pytest.mark.parametrize("scheme", [PIXEL, EDGE8])
def test_variants_commute_with_flips(orc, scheme):
    f = scenes.make_frame(1, 1)
    d = f.depth
    lam = 0.2 if scheme == PIXEL else 1 / 6
    out = orc.diffuse_variant(d, 6, lam, 30.0, scheme)
    assert np.max(np.abs(orc.diffuse_variant(d[::-1], 6, lam, 30.0, scheme) - out[::-1])) < 1e-9
    assert np.max(np.abs(orc.diffuse_variant(d.T, 6, lam, 30.0, scheme) - out.T)) < 1e-9
