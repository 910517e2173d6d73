"""Pins of the oracle's sequential RANSAC (Alg. 2, Eq. 3 and the least-squares
refit): an independent numpy re-derivation of the sampling, brute force over
every triple of tiny images, numpy's eigensolver, exact recovery of
noise-free planes, and the round-control rules."""
import itertools

import numpy as np
import pytest

import scenes

MASK = (1 << 64) - 1


def _numpy_philox_block(ctr, key):
    c = sum(int(w) << (64 * i) for i, w in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    words = [(c >> (64 * i)) & MASK for i in range(4)]
    g = np.random.Philox(counter=np.array(words, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return [int(x) for x in g.random_raw(4)]


def _numpy_triple(j, r, seed, frame, L, assigned):
    """Rejection sampling of 3 distinct unassigned list positions, written from
    the sampling reading with numpy's Philox (independent of the oracle's)."""
    M0 = len(L)
    got = []
    for b in range(16):
        for w in _numpy_philox_block([j, r, b, 0], [seed, frame]):
            k = (w * M0) >> 64
            if assigned[L[k]] or k in got:
                continue
            got.append(k)
            if len(got) == 3:
                return got
    return None


def _plane_numpy(p0, p1, p2):
    e1, e2 = p1 - p0, p2 - p0
    m = np.cross(e1, e2)
    mn = np.linalg.norm(m)
    if not mn > 1e-3 * np.linalg.norm(e1) * np.linalg.norm(e2):
        return None
    n = m / mn
    d = -n @ p0
    if d < 0:
        n, d = -n, -d
    return np.append(n, d)


def _points(frame, float_depth=False):
    import oracle
    d = frame.depth_m * 1000.0 if float_depth else frame.depth.astype(float)
    return oracle.backproject(d, frame.K)


# ---------------------------------------------------------------- eigensolver
def test_eig3_matches_numpy_eigh(orc):
    rng = np.random.default_rng(3)
    for _ in range(200):
        B = rng.normal(size=(3, 3)) * rng.choice([1e-3, 1.0, 1e3])
        A = B @ B.T
        if rng.random() < 0.3:
            A[2] = A[:, 2] = 0.0  # rank deficient
            A[2, 2] = 0.0
        w, V = orc.eig3(A)
        wn, Vn = np.linalg.eigh(A)
        scale = max(abs(wn).max(), 1e-300)
        assert np.max(np.abs(w - wn)) <= 1e-12 * scale
        assert np.max(np.abs(A @ V - V * w)) <= 1e-12 * scale
        assert np.max(np.abs(V.T @ V - np.eye(3))) < 1e-12
        # the smallest eigenvector agrees up to sign when it is well separated
        if wn[1] - wn[0] > 1e-6 * scale:
            assert abs(abs(V[:, 0] @ Vn[:, 0]) - 1.0) < 1e-12


# ---------------------------------------------------------------- refit
def test_refit_recovers_a_noise_free_plane_and_is_invariant(orc):
    rng = np.random.default_rng(5)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    d = 1.7
    a = np.cross(n, [1.0, 0, 0]); a /= np.linalg.norm(a)
    b = np.cross(n, a)
    M = 500
    pts = -d * n + rng.uniform(-1, 1, (M, 1)) * a + rng.uniform(-1, 1, (M, 1)) * b
    P = pts.T.reshape(3, 1, M).copy()
    idx = np.arange(M, dtype=np.int32)
    pl, ce = orc.refit(P, idx)
    want = np.append(n, d) if d > 0 else -np.append(n, d)
    assert np.max(np.abs(pl - want)) < 1e-12
    assert np.max(np.abs(ce - pts.mean(0))) < 1e-12
    pl2, _ = orc.refit(P, rng.permutation(idx))
    assert np.max(np.abs(pl2 - pl)) < 1e-12
    # translation by s changes d by -n.s (while the plane stays camera-facing)
    s = np.array([0.1, -0.2, 0.05])
    pl3, _ = orc.refit((pts + s).T.reshape(3, 1, M).copy(), idx)
    assert np.max(np.abs(pl3[:3] - pl[:3])) < 1e-12
    assert abs(pl3[3] - (pl[3] - pl[:3] @ s)) < 1e-12


def test_refit_normal_is_the_smallest_eigenvector_of_the_scatter(orc):
    f = scenes.make_frame(1, 0)
    P, valid = _points(f)
    idx = np.flatnonzero((f.gt_labels.reshape(-1) == 0) & (valid.reshape(-1) > 0)).astype(np.int32)
    pl, ce = orc.refit(P, idx)
    X = P.reshape(3, -1)[:, idx].T
    c = X.mean(0)
    C = (X - c).T @ (X - c)
    w, V = np.linalg.eigh(C)
    v = V[:, 0]
    if -(v @ c) < 0:
        v = -v
    assert np.max(np.abs(pl[:3] - v)) < 1e-10
    assert abs(pl[3] + v @ c) < 1e-10


# ---------------------------------------------------------------- hypotheses
@pytest.mark.parametrize("r", [0, 3])
def test_hypotheses_match_an_independent_rederivation(orc, r):
    f = scenes.make_frame(1, 0)
    P, valid = _points(f)
    L = orc.valid_list(valid)
    rng = np.random.default_rng(r)
    assigned = (rng.random(valid.shape) < 0.6 * (r > 0)).astype(np.uint8)
    prm = orc.RansacParams(hyps=64, seed=0x5EED0001, frame=9)
    tr, pl, hv = orc.hypotheses(P, L, assigned, prm, r)
    Pf = P.reshape(3, -1)
    af = assigned.reshape(-1)
    for j in range(prm.hyps):
        t = _numpy_triple(j, r, prm.seed, prm.frame, L, af)
        if t is None:
            assert hv[j] == 0
            continue
        assert list(tr[j]) == t
        want = _plane_numpy(*(Pf[:, L[k]] for k in t))
        if want is None:
            assert hv[j] == 0
        else:
            assert hv[j] == 1
            assert np.max(np.abs(pl[j] - want)) < 1e-12
            # the plane passes through its three points
            for k in t:
                assert abs(pl[j, :3] @ Pf[:, L[k]] + pl[j, 3]) < 1e-12


def test_tiny_lists_give_distinct_triples(orc):
    """With five valid points repeated draws are frequent: every triple must
    still hold three distinct positions, as the re-derivation does."""
    rng = np.random.default_rng(0)
    P = np.zeros((3, 2, 4))
    P[:, :, :] = rng.normal(size=(3, 2, 4))
    P[2] += 3.0
    valid = np.zeros((2, 4), np.uint8)
    valid.reshape(-1)[[0, 2, 3, 5, 7]] = 1
    L = orc.valid_list(valid)
    prm = orc.RansacParams(hyps=200, seed=1, frame=1)
    tr, pl, hv = orc.hypotheses(P, L, np.zeros_like(valid), prm, 0)
    for j in range(prm.hyps):
        t = _numpy_triple(j, 0, prm.seed, prm.frame, L, np.zeros(8, np.uint8))
        assert list(tr[j]) == t and len(set(t)) == 3


def test_degeneracy_threshold_on_nearly_collinear_triples(orc):
    """Points on a line with perpendicular offsets spread over decades: the
    validity of every hypothesis follows sin(angle) > 1e-3."""
    rng = np.random.default_rng(4)
    W = 64
    P = np.zeros((3, 1, W))
    P[0, 0] = np.linspace(-1, 1, W)
    P[1, 0] = 10 ** rng.uniform(-6, -1, W) * rng.choice([-1, 1], W)
    P[2, 0] = 2.0 + 0.3 * P[0, 0]
    valid = np.ones((1, W), np.uint8)
    L = orc.valid_list(valid)
    prm = orc.RansacParams(hyps=256, seed=2)
    tr, pl, hv = orc.hypotheses(P, L, np.zeros_like(valid), prm, 0)
    X = P.reshape(3, -1)
    n_valid = 0
    for j in range(prm.hyps):
        want = _plane_numpy(*(X[:, L[k]] for k in tr[j]))
        assert hv[j] == (want is not None)
        n_valid += want is not None
    assert 0 < n_valid < prm.hyps  # both sides of the threshold occur


def test_collinear_points_give_only_invalid_hypotheses(orc):
    # a single row of points on one 3-D line: every triple is degenerate
    W = 50
    P = np.zeros((3, 1, W))
    P[0, 0] = np.linspace(-1, 1, W)
    P[2, 0] = 2.0
    valid = np.ones((1, W), np.uint8)
    L = orc.valid_list(valid)
    _, _, hv = orc.hypotheses(P, L, np.zeros((1, W), np.uint8), orc.RansacParams(hyps=32), 0)
    assert not hv.any()
    rr = orc.ransac(P, valid, orc.RansacParams(hyps=32))
    assert rr.n_planes == 0


def test_sampling_gives_up_when_too_few_points_remain(orc):
    f = scenes.make_frame(1, 0)
    P, valid = _points(f)
    L = orc.valid_list(valid)
    assigned = np.ones_like(valid)
    assigned.reshape(-1)[L[:2]] = 0  # only two unassigned points
    _, _, hv = orc.hypotheses(P, L, assigned, orc.RansacParams(hyps=16), 0)
    assert not hv.any()


# ---------------------------------------------------------------- scoring
def test_counts_match_numpy_brute_force(orc):
    f = scenes.make_frame(1, 1)
    P, valid = _points(f)
    L = orc.valid_list(valid)
    assigned = np.zeros_like(valid)
    assigned.reshape(-1)[L[::3]] = 1
    prm = orc.RansacParams(hyps=128, seed=11, frame=2)
    tr, pl, hv = orc.hypotheses(P, L, assigned, prm, 1)
    counts = orc.score(P, L, assigned, pl, hv, 0.01)
    X = P.reshape(3, -1)[:, [p for p in L if not assigned.reshape(-1)[p]]]
    dist = np.abs(pl[:, :3] @ X + pl[:, 3:4])
    want = np.where(hv > 0, (dist < 0.01).sum(1), 0)
    assert np.array_equal(counts, want)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_over_every_triple_of_a_tiny_image(orc, seed):
    """Two noisy planes on a 7x6 image: score every triple; the round's best
    count cannot exceed the brute-force maximum, its own count is exact, and
    scoring the full triple list selects the brute-force argmax."""
    rng = np.random.default_rng(seed)
    H, W = 6, 7
    u, v = np.meshgrid(np.arange(W), np.arange(H))
    z = np.where(u < 4, 1.0 + 0.05 * v, 1.4 - 0.03 * u) + rng.normal(0, 0.002, (H, W))
    K = scenes.Intrinsics(5.0, 5.0, 3.0, 2.5)
    P, valid = orc.backproject(z * 1000.0, K)
    L = orc.valid_list(valid)
    M = len(L)
    X = P.reshape(3, -1)[:, L]
    trip = list(itertools.combinations(range(M), 3))
    planes = np.zeros((len(trip), 4))
    ok = np.zeros(len(trip), np.uint8)
    for i, (a, b, c) in enumerate(trip):
        q = _plane_numpy(X[:, a], X[:, b], X[:, c])
        if q is not None:
            planes[i], ok[i] = q, 1
    bf = np.where(ok > 0, (np.abs(planes[:, :3] @ X + planes[:, 3:4]) < 0.01).sum(1), 0)
    counts = orc.score(P, L, np.zeros_like(valid), planes, ok, 0.01)
    assert np.array_equal(counts, bf)
    # selection over the full list: most inliers, ties to the lowest index
    assert int(np.argmax(counts)) == int(np.flatnonzero(bf == bf.max())[0])
    prm = orc.RansacParams(hyps=256, min_inliers=3, thresh=0.01, seed=seed)
    rr = orc.ransac_round(P, L, np.zeros_like(valid), prm, 0)
    assert rr.counts.max() <= bf.max()
    js = rr.jstar
    # ties go to the lowest hypothesis index
    assert js == int(np.flatnonzero((rr.counts == rr.counts[rr.hvalid > 0].max()) & (rr.hvalid > 0))[0])
    t = tuple(sorted(rr.triples[js]))
    assert rr.counts[js] == bf[trip.index(t)]


# ---------------------------------------------------------------- sequential
def _separated_c1():
    """Noise-free, hole-free C1 with every point closer than 2 t to a second
    ground-truth plane removed, so each plane's slab holds only its own points."""
    import oracle
    f = scenes.make_frame(1, 0, noise="none", hole_frac=0.0)
    P, valid = oracle.backproject(f.depth_m * 1000.0, f.K)
    X = P.reshape(3, -1)
    lab = f.gt_labels.reshape(-1)
    dist = np.abs(f.gt_planes[:, :3] @ X + f.gt_planes[:, 3:4])
    keep = lab >= 0
    for i in range(len(f.gt_planes)):
        keep &= (lab == i) | (dist[i] > 0.02)
    depth = np.where(keep.reshape(f.depth.shape), f.depth_m * 1000.0, 0.0)
    P, valid = oracle.backproject(depth, f.K)
    return f, P, valid, np.where(keep, lab, -1).reshape(f.depth.shape)


def test_sequential_ransac_recovers_every_separated_plane_exactly(orc):
    f, P, valid, lab = _separated_c1()
    prm = orc.RansacParams(hyps=256, max_planes=12, min_inliers=50, thresh=0.01, seed=0x5EED0001, frame=0)
    rr = orc.ransac(P, valid, prm)
    assert rr.n_planes == len(f.gt_planes)
    used = set()
    for i in range(rr.n_planes):
        diff = np.max(np.abs(f.gt_planes - rr.planes[i]), axis=1)
        g = int(np.argmin(diff))
        assert diff[g] < 1e-9
        used.add(g)
        # labels of round i are exactly the pixels of ground-truth plane g
        assert np.array_equal(rr.labels == i, lab == g)
        assert rr.inliers[i] == (lab == g).sum()
    assert len(used) == len(f.gt_planes)
    # planes come out largest first
    assert list(rr.inliers) == sorted(rr.inliers, reverse=True)


def test_full_run_equals_its_rounds_in_follow_mode(orc):
    f = scenes.make_frame(1, 0)
    I = orc.diffuse(f.depth, 10, 0.2, 30.0)
    P, valid = orc.backproject(I, f.K)
    cfg = scenes.CONFIGS[1]
    prm = orc.RansacParams(hyps=256, max_planes=12, min_inliers=cfg.min_inliers(160, 120), seed=cfg.ransac_seed)
    rr = orc.ransac(P, valid, prm)
    assert rr.n_planes >= 4
    L = orc.valid_list(valid)
    assigned = np.zeros_like(valid)
    total = 0.0
    for r in range(rr.n_planes):
        res = orc.ransac_round(P, L, assigned, prm, r)
        assert res.status == 0 and res.jstar == rr.jstar[r]
        assert np.array_equal(res.plane, rr.planes[r])
        assert np.array_equal(res.fmask, rr.labels == r)
        assert res.s_count == res.counts[res.jstar]
        total += res.n_remaining * prm.hyps
        assigned = assigned | res.fmask.astype(np.uint8)
    assert total <= rr.residuals
    # the label image marks each remaining point at most once and holes never
    assert np.all(rr.labels[valid == 0] == -1)


def test_round_control_rules(orc):
    f = scenes.make_frame(1, 0)
    P, valid = _points(f)
    # max_planes caps the rounds
    rr = orc.ransac(P, valid, orc.RansacParams(hyps=64, max_planes=2, min_inliers=10))
    assert rr.n_planes == 2
    # min_inliers above every plane emits nothing
    rr = orc.ransac(P, valid, orc.RansacParams(hyps=64, min_inliers=10 ** 6))
    assert rr.n_planes == 0 and np.all(rr.labels == -1)
    # an empty frame and a frame with two points
    empty = np.zeros_like(valid)
    assert orc.ransac(P * 0, empty, orc.RansacParams()).n_planes == 0
    two = np.zeros_like(valid)
    two.reshape(-1)[[5, 900]] = 1
    assert orc.ransac(P, two, orc.RansacParams()).n_planes == 0


def test_threshold_is_strict(orc):
    """Points at distance exactly t (binary-exact values) are not inliers."""
    W = 8
    P = np.zeros((3, 1, W))
    P[0, 0] = np.arange(W) * 0.25
    P[2, 0] = [1.0, 1.0, 1.5, 0.5, 1.25, 1.0, 2.0, 1.0]
    valid = np.ones((1, W), np.uint8)
    L = orc.valid_list(valid)
    plane = np.array([[0.0, 0.0, -1.0, 1.0]])  # z = 1
    c = orc.score(P, L, np.zeros_like(valid), plane, np.ones(1, np.uint8), 0.5)
    # |1 - z| < 0.5 holds for z in {1, 1, 1.25, 1, 1}; z = 1.5 and z = 0.5 sit exactly at t
    assert c[0] == 5


def test_final_set_is_the_refit_planes_inliers_and_min_inliers_is_inclusive(orc):
    f = scenes.make_frame(1, 0)
    I = orc.diffuse(f.depth, 10, 0.2, 30.0)
    P, valid = orc.backproject(I, f.K)
    L = orc.valid_list(valid)
    prm = orc.RansacParams(hyps=128, min_inliers=50, seed=3)
    res = orc.ransac_round(P, L, np.zeros_like(valid), prm, 0)
    assert (res.smask != res.fmask).sum() > 0  # a case where the refit moves the set
    X = P.reshape(3, -1)[:, L]
    fm = np.zeros(valid.size, bool)
    fm[L] = np.abs(res.plane[:3] @ X + res.plane[3]) < prm.thresh
    assert np.array_equal(res.fmask.reshape(-1), fm)
    sm = np.zeros(valid.size, bool)
    sm[L] = np.abs(res.hyp_plane[:3] @ X + res.hyp_plane[3]) < prm.thresh
    assert np.array_equal(res.smask.reshape(-1), sm)
    assert res.s_count == sm.sum() == res.counts[res.jstar]
    # the refit plane is the least-squares plane of S
    pl, ce = orc.refit(P, np.flatnonzero(sm).astype(np.int32))
    assert np.array_equal(pl, res.plane)
    # min_inliers == |F| still emits; |F| + 1 does not
    for mi, want in [(res.f_count, 0), (res.f_count + 1, 2)]:
        prm2 = orc.RansacParams(hyps=128, min_inliers=mi, seed=3)
        assert orc.ransac_round(P, L, np.zeros_like(valid), prm2, 0).status == want


def test_removal_invariants_hold_on_the_oracle_and_fail_on_planted_mistakes(orc):
    """The float64 removal invariants that the GPU test of the benchmark
    workload applies to every frame hold on the oracle's own result, and each
    planted mistake in a copy of that result breaks them: a plane shifted by
    2t, two pixels of planes 0 and 1 swapped (counts unchanged), an inlier
    dropped, a relabelled pixel."""
    from gpu_util import check_removal
    f = scenes.make_frame(1, 0)
    cfg = scenes.CONFIGS[1]
    H, W = f.depth.shape
    prm = orc.RansacParams(hyps=cfg.hyps, max_planes=cfg.max_planes, min_inliers=cfg.min_inliers(W, H),
                           thresh=cfg.thresh_m, seed=cfg.ransac_seed)
    I = orc.diffuse(f.depth, cfg.diffuse_iters, cfg.lam, cfg.kappa_mm)
    P, valid = orc.backproject(I, f.K)
    rr = orc.ransac(P, valid, prm)
    assert rr.n_planes >= 3
    planes = [dict(n=rr.planes[r, :3], d=rr.planes[r, 3], inliers=int(rr.inliers[r]), hyp_index=int(rr.jstar[r]))
              for r in range(rr.n_planes)]
    args = (prm.thresh, prm.min_inliers, prm.hyps)
    check_removal(P, rr.labels, valid, planes, *args, band=1e-12)

    shifted = [dict(p) for p in planes]
    shifted[1]["d"] += 2 * prm.thresh
    with pytest.raises(AssertionError):
        check_removal(P, rr.labels, valid, shifted, *args, band=1e-12)
    flat = rr.labels.reshape(-1)
    i0, i1 = np.flatnonzero(flat == 0)[0], np.flatnonzero(flat == 1)[0]
    for edit in ({i0: 1, i1: 0}, {i0: -1}, {i0: 1}):
        lab = rr.labels.copy()
        for i, v in edit.items():
            lab.reshape(-1)[i] = v
        with pytest.raises(AssertionError):
            check_removal(P, lab, valid, planes, *args, band=1e-12)


def test_label_comparison_explains_only_near_threshold_differences(orc):
    """The free-running label check of the GPU tests (R20): on the oracle's
    own result against itself nothing differs; a pixel relabelled far from t
    is caught; a pixel that a second, slightly shifted plane puts on the
    other side of t is explained by that shift and caught without it; a
    pixel beyond the common planes is caught."""
    from gpu_util import labels_explained
    f = scenes.make_frame(1, 1)
    cfg = scenes.CONFIGS[1]
    H, W = f.depth.shape
    prm = orc.RansacParams(hyps=cfg.hyps, max_planes=cfg.max_planes, min_inliers=cfg.min_inliers(W, H),
                           thresh=cfg.thresh_m, seed=cfg.ransac_seed, frame=1)
    I = orc.diffuse(f.depth, cfg.diffuse_iters, cfg.lam, cfg.kappa_mm)
    P, valid = orc.backproject(I, f.K)
    rr = orc.ransac(P, valid, prm)
    t = prm.thresh
    planes = [rr.planes[r].copy() for r in range(rr.n_planes)]
    assert labels_explained(P, P, rr.labels, rr.labels, planes, planes, t) == (0, 0.0)
    X = P.reshape(3, -1)
    flat = rr.labels.reshape(-1)
    r0 = np.abs(planes[0][:3] @ X + planes[0][3])
    # far from t: relabelled as unassigned
    far = np.flatnonzero((flat == 0) & (r0 < 0.5 * t))[0]
    lab = rr.labels.copy()
    lab.reshape(-1)[far] = -1
    with pytest.raises(AssertionError):
        labels_explained(P, P, lab, rr.labels, planes, planes, t)
    # the inlier of plane 0 closest to t, pushed out by a shifted plane 0
    mine = np.flatnonzero(flat == 0)
    edge = mine[np.argmax(r0[mine])]
    gap = t - r0[edge]
    assert gap > 1e-6
    shifted = [p.copy() for p in planes]
    side = np.sign(planes[0][:3] @ X[:, edge] + planes[0][3])
    shifted[0][3] += side * 2 * gap
    lab = rr.labels.copy()
    lab.reshape(-1)[edge] = -1
    n, used = labels_explained(P, P, lab, rr.labels, shifted, planes, t)
    assert n == 1 and used >= gap
    with pytest.raises(AssertionError):
        labels_explained(P, P, lab, rr.labels, planes, planes, t)
    # a label no common plane explains
    lab = rr.labels.copy()
    lab.reshape(-1)[far] = rr.n_planes
    with pytest.raises(AssertionError):
        labels_explained(P, P, lab, rr.labels, planes, planes, t)
