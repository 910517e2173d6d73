"""The library's polygon map with drift compensation (host code behind the C
ABI, no GPU needed) against the oracle: the same observations (the oracle
gets the pixel polygons lifted onto their planes) give the same matches,
measurements, drift estimates, variances and map polygons, frame by frame,
over rendered staircase walks with injected vertical drift."""
import numpy as np
import pytest

import paper_2411_01919_amd as pp
import scenes
from oracle import mapping as M


def _observations(orc, f, min_px=400):
    out = []
    for g in range(len(f.gt_planes)):
        npx = int((f.gt_labels == g).sum())
        if npx < min_px:
            continue
        xy = orc.region_polygons(np.where(f.gt_labels == g, 0, -1).astype(np.int16), 1, 1.0)[0]
        n, d = f.gt_planes[g][:3], f.gt_planes[g][3]
        verts = M.lift_polygon(xy, n, d, (f.K.fx, f.K.fy, f.K.cx, f.K.cy))
        out.append((n, d, verts.mean(axis=0), npx, xy, verts))
    return out


@pytest.mark.parametrize("cid,drift_step,sp,sm", [(2, 0.01, 1e-4, 1e-5), (3, -0.008, 1e-5, 1e-4), (2, 0.0, 1e-5, 1e-4)])
def test_map_equals_the_oracle(orc, cid, drift_step, sp, sm):
    lib = pp.DriftMap(0.05, sp, sm, 15.0)
    ref = M.DriftMap(0.05, sp, sm, 15.0)
    for k in range(10):
        f = scenes.make_frame(cid, k, size=(320, 240))
        R, Cc = f.pose
        C = Cc + np.array([0.0, 0.0, drift_step * k])
        obs = _observations(orc, f)
        K = (f.K.fx, f.K.fy, f.K.cx, f.K.cy)
        a = lib.integrate(K, R, C, [(n, d, c, s, xy) for (n, d, c, s, xy, _) in obs])
        b = ref.integrate(R, C, [(n, d, c, s, v) for (n, d, c, s, _, v) in obs])
        assert (a["matched"], a["added"], a["skipped"]) == (b.matched, b.added, b.skipped), k
        assert a["match_of"] == b.match_of, k
        assert (np.isnan(a["measurement"]) and np.isnan(b.measurement)) or a["measurement"] == pytest.approx(
            b.measurement, abs=1e-12)
        assert a["drift"] == pytest.approx(b.drift, abs=1e-12) and a["variance"] == pytest.approx(b.variance, rel=1e-12)
    mine = lib.polygons()
    assert len(mine) == len(ref.polys)
    for p, q in zip(mine, ref.polys):
        assert p["support"] == q.support and p["height"] == pytest.approx(q.height, abs=1e-12)
        assert {tuple(np.round(v, 9)) for v in p["hull"]} == {tuple(np.round(v, 9)) for v in q.hull}
    lib.close()


def test_map_argument_checks():
    from paper_2411_01919_amd import _native as N
    import ctypes
    h = ctypes.c_void_p()
    for bad in ((0.0, 1e-5, 1e-4, 15.0), (0.05, -1.0, 1e-4, 15.0), (0.05, 1e-5, 0.0, 15.0), (0.05, 1e-5, 1e-4, 90.0)):
        assert N.lib().pp_map_create(ctypes.byref(N.MapParams(*bad)), ctypes.byref(h)) == N.PP_E_INVAL
    m = pp.DriftMap()
    with pytest.raises(pp.PPError):
        m.integrate((0.0, 1.0, 0.0, 0.0), np.eye(3), np.zeros(3), [])
    r = m.integrate((100.0, 100.0, 50.0, 40.0), np.eye(3), np.zeros(3), [])
    assert r["matched"] == 0 and r["added"] == 0 and np.isnan(r["measurement"])
