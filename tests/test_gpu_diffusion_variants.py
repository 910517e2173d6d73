"""Parity of the other discretisations of Eq. 1 (Alg. 1 as printed, pixel-centred;
8-neighbour per-edge flux) with the oracle's, through the C ABI, and their
grouping in ragged batches.  Tolerance: 1e-3 mm max-abs, holes exactly 0."""
import numpy as np
import pytest

import scenes
from gpu_util import cfg_params, log, to_dev

pytestmark = pytest.mark.gpu

PIXEL, EDGE8 = 1, 2


@pytest.fixture(scope="module")
def pp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_01919_amd as pp
    pp.default_context(0)
    return pp


CASES = [
    # scheme, edge_stop, config, frame, size, iters, lambda
    (PIXEL, 0, 1, 0, None, 10, 0.2),
    (PIXEL, 1, 2, 0, None, 20, 0.25),
    (PIXEL, 0, 3, 1, (200, 77), 12, 0.2),
    (EDGE8, 0, 1, 1, None, 10, 1 / 6),
    (EDGE8, 1, 2, 1, None, 20, 0.15),
    (EDGE8, 0, 3, 2, (131, 45), 7, 0.1),
    (PIXEL, 0, 1, 2, None, 1, 0.2),
    (EDGE8, 0, 1, 2, None, 0, 0.1),
]


@pytest.mark.parametrize("scheme,edge,cid,k,size,iters,lam", CASES)
def test_variant_matches_oracle(pp, orc, scheme, edge, cid, k, size, iters, lam):
    log(f"diffusion variant scheme={scheme} edge={edge} cfg={cid} k={k} size={size} iters={iters} lam={lam:.4f}")
    f = scenes.make_frame(cid, k, size=size)
    out = pp.diffuse(to_dev(f.depth), iters, lam, 30.0, edge, scheme=scheme).cpu().numpy()
    ref = orc.diffuse_variant(f.depth, iters, lam, 30.0, scheme, edge)
    holes = f.depth == 0
    assert np.all(out[holes] == 0.0)
    err = np.abs(out.astype(np.float64) - ref)
    log(f"  max |dI| = {err.max():.3e} mm")
    assert err.max() <= 1e-3
    if scheme == EDGE8:  # conservative up to rounding: one ulp per pixel
        drift = abs(out.astype(np.float64).sum() - f.depth.astype(np.float64).sum())
        assert drift <= np.spacing(out[~holes]).astype(np.float64).sum()


@pytest.mark.parametrize("scheme", [PIXEL, EDGE8])
def test_variant_constant_image_is_a_fixed_point(pp, scheme):
    img = np.full((61, 97), 2345, np.uint16)
    img[np.random.default_rng(scheme).random(img.shape) < 0.1] = 0
    out = pp.diffuse(to_dev(img), 11, 0.1, 30.0, scheme=scheme).cpu().numpy()
    assert np.array_equal(out, img.astype(np.float32))


def test_mixed_schemes_in_one_batch_equal_the_plain_path(pp):
    """A ragged batch whose frames use different schemes and iteration counts:
    the batch groups them, and every output equals the frame run alone."""
    import torch
    spec = [(1, 0, PIXEL, 10, 0.2), (2, 0, 0, 20, 0.2), (3, 1, EDGE8, 20, 1 / 6), (1, 1, EDGE8, 10, 0.1),
            (2, 1, PIXEL, 20, 0.2), (1, 2, 0, 10, 0.2)]
    outs = []
    for cid, k, scheme, iters, lam in spec:
        f = scenes.make_frame(cid, k)
        H, W = f.depth.shape
        dc, rc = cfg_params(cid, W, H, k)
        dc.scheme, dc.iters, dc.lam = scheme, iters, lam
        outs.append(pp.make_outputs(to_dev(f.depth), (f.K.fx, f.K.fy, f.K.cx, f.K.cy), dc, rc))
    for fo in outs:
        pp.run_frame(fo)
    torch.cuda.synchronize()
    plain = [(fo.depth_mm.cpu().numpy().copy(), fo.labels.cpu().numpy().copy()) for fo in outs]
    for graph in (False, True):
        for fo in outs:
            fo.depth_mm.zero_()
            fo.labels.zero_()
        pp.batch_run(outs, graph=graph)
        torch.cuda.synchronize()
        for fo, (d, lab) in zip(outs, plain):
            assert np.array_equal(fo.depth_mm.cpu().numpy(), d), graph
            assert np.array_equal(fo.labels.cpu().numpy(), lab), graph


def test_variant_argument_checks(pp):
    img = to_dev(np.full((16, 16), 1000, np.uint16))
    for scheme, lam in [(EDGE8, 0.2), (3, 0.1), (-1, 0.1)]:
        with pytest.raises(pp.PPError):
            pp.diffuse(img, 3, lam, 30.0, scheme=scheme)
