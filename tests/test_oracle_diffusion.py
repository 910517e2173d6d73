"""Pins of the oracle's Perona-Malik diffusion (Eq. 1, Alg. 1) against facts the
mathematics fixes: fixed points, conservation, the maximum principle, the
closed-form heat-equation mode decay, symmetry, and the edge-stopping
function isolated on a two-pixel image."""
import math

import numpy as np
import pytest

import scenes


@pytest.mark.parametrize("shape", [(7, 9), (33, 40)])
@pytest.mark.parametrize("val", [1, 1234, 65535])
def test_constant_image_is_a_fixed_point_bit_exact(orc, shape, val):
    rng = np.random.default_rng(val)
    img = np.full(shape, val, np.uint16)
    img[rng.random(shape) < 0.2] = 0  # holes must not disturb the fixed point
    for iters, lam, kappa in [(1, 0.2, 30.0), (10, 0.25, 5.0), (20, 0.1, 1e30)]:
        out = orc.diffuse(img, iters, lam, kappa)
        assert np.array_equal(out, img.astype(np.float64))


@pytest.mark.parametrize("edge_stop", [0, 1])
def test_sum_is_conserved_and_holes_stay_zero(orc, edge_stop):
    f = scenes.make_frame(1, 0)
    out = orc.diffuse(f.depth, 10, 0.2, 30.0, edge_stop)
    s0 = f.depth.astype(np.float64).sum()
    assert abs(out.sum() - s0) <= 1e-12 * s0
    assert np.all(out[f.depth == 0] == 0.0)
    assert np.all(out[f.depth > 0] > 0.0)


def test_discrete_maximum_principle(orc):
    f = scenes.make_frame(1, 3)
    v = f.depth > 0
    lo, hi = f.depth[v].min(), f.depth[v].max()
    for n in (1, 5, 20):
        out = orc.diffuse(f.depth, n, 0.25, 30.0)
        assert out[v].min() >= lo - 1e-9 and out[v].max() <= hi + 1e-9
    # and the spread of a noisy flat patch shrinks
    flat = np.full((32, 32), 2000.0) + np.random.default_rng(1).normal(0, 3, (32, 32))
    out = orc.diffuse(flat, 10, 0.2, 30.0)
    assert out.std() < 0.5 * flat.std()


@pytest.mark.parametrize("k,l", [(1, 0), (3, 0), (2, 1), (5, 3)])
def test_heat_mode_decay_closed_form(orc, k, l):
    """With kappa -> inf, g == 1 and one step is the 5-point heat step with zero
    flux at the border; cos(pi k (u+1/2)/W) cos(pi l (v+1/2)/H) is its
    eigenvector with factor 1 - 4 lam (sin^2(pi k/2W) + sin^2(pi l/2H))."""
    W, H, lam, N = 48, 20, 0.2, 25
    A, B = 1000.0, 50.0
    u = np.arange(W)[None, :]
    v = np.arange(H)[:, None]
    mode = np.cos(math.pi * k * (u + 0.5) / W) * np.cos(math.pi * l * (v + 0.5) / H)
    img = A + B * mode
    out = orc.diffuse(img, N, lam, 1e30)
    fac = 1.0 - 4.0 * lam * (math.sin(math.pi * k / (2 * W)) ** 2 + math.sin(math.pi * l / (2 * H)) ** 2)
    expected = A + B * fac ** N * mode
    assert np.max(np.abs(out - expected)) < 1e-9


def test_flips_and_transpose_commute(orc):
    f = scenes.make_frame(1, 1)
    d = f.depth
    out = orc.diffuse(d, 10, 0.2, 30.0)
    assert np.max(np.abs(orc.diffuse(d[::-1], 10, 0.2, 30.0) - out[::-1])) < 1e-9
    assert np.max(np.abs(orc.diffuse(d[:, ::-1], 10, 0.2, 30.0) - out[:, ::-1])) < 1e-9
    assert np.max(np.abs(orc.diffuse(d.T, 10, 0.2, 30.0) - out.T)) < 1e-9


@pytest.mark.parametrize("a,b", [(1000, 1010), (1000, 1030), (2000, 1900), (500, 501)])
def test_edge_stopping_function_on_two_pixels(orc, a, b):
    """Alg. 1 prints c = exp(-(|grad I|/k)^2); on a 1x2 image one step moves each
    pixel by lam * g(b-a) * (b-a) towards the other (the per-edge flux)."""
    lam, kappa = 0.2, 30.0
    img = np.array([[a, b]], np.uint16)
    out = orc.diffuse(img, 1, lam, kappa)
    g = math.exp(-(((b - a) / kappa) ** 2))
    assert out[0, 0] == pytest.approx(a + lam * g * (b - a), abs=1e-12)
    assert out[0, 1] == pytest.approx(b - lam * g * (b - a), abs=1e-12)
    out = orc.diffuse(img, 1, lam, kappa, edge_stop=1)
    g = 1.0 / (1.0 + ((b - a) / kappa) ** 2)
    assert out[0, 0] == pytest.approx(a + lam * g * (b - a), abs=1e-12)


def test_one_step_bump_example(orc):
    """A 3x3 patch with a 100 mm bump in the middle: after one step the centre
    loses 4 lam g(100) 100, each edge pixel gains lam g(100) 100, corners (whose
    neighbours are all equal to them) do not move."""
    lam, kappa = 0.2, 30.0
    img = np.full((3, 3), 1000, np.uint16)
    img[1, 1] = 1100
    out = orc.diffuse(img, 1, lam, kappa)
    g = math.exp(-((100.0 / kappa) ** 2))
    assert out[1, 1] == pytest.approx(1100 - 4 * lam * g * 100, abs=1e-12)
    for (i, j) in [(0, 1), (1, 0), (1, 2), (2, 1)]:
        assert out[i, j] == pytest.approx(1000 + lam * g * 100, abs=1e-12)
    for (i, j) in [(0, 0), (0, 2), (2, 0), (2, 2)]:
        assert out[i, j] == 1000.0


def test_hole_blocks_flux(orc):
    img = np.array([[1000, 0, 2000]], np.uint16)
    out = orc.diffuse(img, 5, 0.25, 1e30)
    assert np.array_equal(out, img.astype(float))
