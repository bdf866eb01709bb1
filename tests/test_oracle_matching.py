"""Pins of the oracle's matching stage (Section 3.1): eq. (1) cost, exact-NN
initialisation, propagation + random search, consistency check -- against
Parseval, brute force, closed forms and invariants."""
import numpy as np
import pytest

import oracle
from sff_inputs import SceneSpec, make_scene, small_spec, smoothed_noise
from tests import indep


def _descs(imgs, level):
    return [oracle.features(im, level) for im in imgs]


def _bins(imgs, level):
    n = 1 << level
    return [indep.bin_sums(oracle.smooth(im, n), n) for im in imgs]


def _scene(H, W, C, seed, **kw):
    return make_scene(small_spec(H, W, C, seed, **kw))


# ----------------------------------------------------------------- cost ----
@pytest.mark.parametrize("level", [0, 1, 2])
@pytest.mark.parametrize("s", [1, -1])
def test_cost_equals_parseval_route(level, s):
    sc = _scene(24, 36, 3, seed=21 + level)
    imgs = sc.images()
    D = _descs(imgs, level)
    B = _bins(imgs, level)
    rng = np.random.default_rng(level * 10 + (s > 0))
    for _ in range(150):
        y, x = int(rng.integers(0, 24)), int(rng.integers(0, 36))
        h = rng.integers(-40, 41, 4).astype(np.int16)  # includes clamped targets
        assert oracle.cost(D, s, x, y, h) == indep.cost_parseval(B, s, x, y, h)


def test_cost_zero_at_ground_truth():
    """Clean integer translations: at pixels whose whole 8x8 neighbourhood moves
    rigidly and is visible in all three targets, eq. (1) is exactly zero."""
    spec = SceneSpec(H=48, W=80, C=1, seed=5, n_segments=(1, 1), d_range=(3, 9),
                     flow_max=6, slope_max=0.0)
    sc = make_scene(spec)
    D = _descs(sc.images(), 0)
    gt = sc.gt_fwd
    vis = sc.vis_T & sc.vis_S & sc.vis_X
    checked = 0
    for y in range(4, 44):
        for x in range(4, 76):
            win = (slice(max(y - 3, 0), y + 5), slice(max(x - 3, 0), x + 5))
            if not vis[win].all() or not (gt[win] == gt[y, x]).all():
                continue
            u, v, d0, d1 = (int(t) for t in gt[y, x])
            tg = [(x + u, y + v), (x - d0, y), (x + u - d1, y + v)]
            if not all(3 <= tx < 80 - 4 and 3 <= ty < 48 - 4 for tx, ty in tg):
                continue
            assert oracle.cost(D, 1, x, y, gt[y, x]) == 0
            checked += 1
    assert checked > 200


def test_cost_extreme_contrast_fits_uint32():
    chk = ((np.indices((16, 16)).sum(axis=0) % 2) * 255).astype(np.uint8)
    a = np.repeat(chk[..., None], 3, axis=2)
    b = 255 - a
    imgs = [a, b, b, b]
    D = _descs(imgs, 0)
    B = _bins(imgs, 0)
    h = np.zeros(4, np.int16)
    ref = indep.cost_parseval(B, 1, 8, 8, h)
    assert ref < 2 ** 32
    assert oracle.cost(D, 1, 8, 8, h) == ref


# ------------------------------------------------------------------ init ----
@pytest.mark.parametrize("level,s,C", [(0, 1, 1), (0, -1, 2), (1, 1, 3), (1, -1, 1), (2, 1, 2)])
def test_init_matches_brute_force(level, s, C):
    sc = _scene(20, 44, C, seed=31 + level, flow_max=10, d_range=(0, 16))
    imgs = sc.images()
    D = _descs(imgs, level)
    B = _bins(imgs, level)
    fmax, dmax = 9, 14
    hyp, cst = oracle.init_nn(D, level, s, fmax, dmax)
    bh, bc = indep.brute_init(B, s, level, fmax, dmax)
    assert np.array_equal(hyp.astype(np.int64), bh)
    assert np.array_equal(cst.astype(np.int64), bc)


def test_init_ties_go_to_smallest_index():
    const = np.full((16, 24, 1), 90, np.uint8)
    D = _descs([const] * 4, 0)
    for s in (1, -1):
        hyp, cst = oracle.init_nn(D, 0, s, 5, 7)
        assert np.all(cst == 0)
        for i in range(16):
            for j in range(24):
                u, v, d0, d1 = (int(t) for t in hyp[i, j])
                assert v == -min(5, i) and u == -min(5, j)
                # smallest stereo target column
                assert j - s * d0 == (max(j - 7, 0) if s > 0 else j)
                assert j + u - s * d1 == (max(j + u - 7, 0) if s > 0 else j + u)


def test_init_recovers_clean_translation():
    spec = SceneSpec(H=40, W=72, C=1, seed=8, n_segments=(1, 1), d_range=(4, 4),
                     flow_max=5, slope_max=0.0)
    sc = make_scene(spec)
    D = _descs(sc.images(), 0)
    hyp, cst = oracle.init_nn(D, 0, 1, 8, 8)
    gt = sc.gt_fwd
    inner = (slice(10, 30), slice(16, 56))
    assert np.array_equal(hyp[inner], gt[inner])
    assert np.all(cst[inner] == 0)


# ---------------------------------------------------------- match level ----
def _level_case(seed=41, H=24, W=40, C=2, level=0):
    sc = _scene(H, W, C, seed=seed, flow_max=6, d_range=(0, 8))
    D = _descs(sc.images(), level)
    return sc, D


@pytest.mark.parametrize("s", [1, -1])
def test_match_level_cost_field_is_consistent_and_monotone(s):
    sc, D = _level_case()
    B = _bins(sc.images(), 0)
    h0, c0 = oracle.init_nn(D, 0, s, 8, 10)
    h1, c1 = oracle.match_level(D, 0, s, 123, 3, 32, 6, 8, 10, h0, c0)
    assert np.all(c1 <= c0)
    for i in range(h1.shape[0]):
        for j in range(h1.shape[1]):
            assert c1[i, j] == indep.cost_parseval(B, s, j, i, h1[i, j])
    assert np.all(np.abs(h1[..., :2]) <= 8)
    assert np.all((h1[..., 2:] >= 0) & (h1[..., 2:] <= 10))


def test_match_level_order_and_thread_independence():
    sc, D = _level_case(seed=42, C=1)
    h0, c0 = oracle.init_nn(D, 0, 1, 8, 10)
    ref = oracle.match_level(D, 0, 1, 5, 3, 32, 6, 8, 10, h0, c0, order=0, nthreads=1)
    rev = oracle.match_level(D, 0, 1, 5, 3, 32, 6, 8, 10, h0, c0, order=1, nthreads=1)
    par = oracle.match_level(D, 0, 1, 5, 3, 32, 6, 8, 10, h0, c0, order=0, nthreads=4)
    for a, b in ((ref, rev), (ref, par)):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_match_level_never_below_exhaustive_minimum():
    sc = _scene(16, 24, 1, seed=43, flow_max=3, d_range=(0, 5))
    D = _descs(sc.images(), 0)
    B = _bins(sc.images(), 0)
    fmax, dmax = 4, 6
    for s in (1, -1):
        h0, c0 = oracle.init_nn(D, 0, s, fmax, dmax)
        h1, c1 = oracle.match_level(D, 0, s, 77, 8, 8, 6, fmax, dmax, h0, c0)
        ex = indep.exhaustive_min(B, s, 0, fmax, dmax)
        assert np.all(c1.astype(np.int64) >= ex)
        # the search reaches the global minimum at a good share of pixels
        assert (c1.astype(np.int64) == ex).mean() > 0.3


def test_propagation_spreads_as_red_black_diamond():
    """With identical images, (0,0,0,0) has cost 0 and any other vector a
    positive cost.  Start every pixel at a bad vector except one seed pixel, and
    switch off random search: after `it` iterations exactly the pixels within
    Manhattan distance 2*it - 1 (seed red) or 2*it (seed black) carry the seed."""
    rng = np.random.default_rng(9)
    img = rng.integers(0, 256, (30, 30, 1), dtype=np.uint8)
    D = _descs([img] * 4, 0)
    B = _bins([img] * 4, 0)
    bad = np.array([5, 3, 2, 4], np.int16)
    for seed_px, colour in (((14, 14), "red"), ((14, 15), "black")):
        h = np.tile(bad, (30, 30, 1))
        h[seed_px] = 0
        c = np.array([[indep.cost_parseval(B, 1, j, i, h[i, j]) for j in range(30)]
                      for i in range(30)], np.uint32)
        assert np.all(c[h[..., 0] == 5] > 0)
        for it in (1, 2, 3):
            h1, c1 = oracle.match_level(D, 0, 1, 0, it, 32, 0, 16, 16, h, c)
            yy, xx = np.indices((30, 30))
            dist = np.abs(yy - seed_px[0]) + np.abs(xx - seed_px[1])
            reach = 2 * it - 1 if colour == "red" else 2 * it
            assert np.array_equal((h1 == 0).all(axis=-1), dist <= reach)


def test_constant_images_leave_field_unchanged():
    const = np.full((12, 20, 2), 40, np.uint8)
    D = _descs([const] * 4, 0)
    rng = np.random.default_rng(10)
    h = rng.integers(0, 5, (12, 20, 4)).astype(np.int16)
    c = np.zeros((12, 20), np.uint32)
    h1, c1 = oracle.match_level(D, 0, 1, 3, 4, 32, 6, 8, 8, h, c)
    assert np.array_equal(h1, h) and np.all(c1 == 0)


def test_handoff_copies_parent_and_recomputes_cost():
    sc = _scene(22, 34, 2, seed=44)
    D1 = _descs(sc.images(), 1)
    D0 = _descs(sc.images(), 0)
    B0 = _bins(sc.images(), 0)
    hc, cc = oracle.init_nn(D1, 1, 1, 8, 8)
    h, c = oracle.match_level(D0, 0, 1, 1, 0, 32, 6, 8, 8, None, None, hyp_coarse=hc)
    for i in range(22):
        for j in range(34):
            assert np.array_equal(h[i, j], hc[i >> 1, j >> 1])
            assert c[i, j] == indep.cost_parseval(B0, 1, j, i, h[i, j])


def test_random_search_changes_stay_in_radius():
    sc, D = _level_case(seed=45, C=1)
    # uniform starting field: propagation has nothing to offer, only search moves
    h = np.tile(np.array([2, 1, 3, 3], np.int16), (24, 40, 1))
    B = _bins(sc.images(), 0)
    c = np.array([[indep.cost_parseval(B, 1, j, i, h[i, j]) for j in range(40)]
                  for i in range(24)], np.uint32)
    h1, c1 = oracle.match_level(D, 0, 1, 11, 1, 4, 1, 30, 30, h, c)
    moved = ~(h1 == h).all(axis=-1)
    red = (np.indices((24, 40)).sum(axis=0) % 2) == 0
    assert moved[red].any()
    # red pixels move at most 4 px per component; black pixels may also take a
    # red neighbour's searched vector, at most 4 px from the start as well
    assert np.all(np.abs(h1.astype(int) - h.astype(int)) <= 8)
    assert np.all(np.abs(h1[red].astype(int) - h[red].astype(int)) <= 4)
    assert np.all(c1 <= c)


# ---------------------------------------------------------- consistency ----
def test_consistency_accepts_ground_truth():
    spec = SceneSpec(H=40, W=80, C=1, seed=6, n_segments=(3, 3), d_range=(2, 10),
                     flow_max=6, delta_max=2)
    sc = make_scene(spec)
    valid, err = oracle.consistency(sc.gt_fwd, sc.gt_inv, 1)
    H, W = 40, 80
    yy, xx = np.indices((H, W))
    u, v, d0, d1 = (sc.gt_fwd[..., k].astype(int) for k in range(4))
    inb = ((xx + u >= 0) & (xx + u < W) & (yy + v >= 0) & (yy + v < H) & (xx - d0 >= 0)
           & (xx + u - d1 >= 0) & (xx + u - d1 < W))
    ok = inb & sc.vis_X
    assert np.all(valid[ok] == 1) and np.all(err[ok] == 0)
    assert np.all(valid[~inb] == 0) and np.all(err[~inb] == 0xFFFFFFFF)


def test_consistency_thresholds():
    H, W = 6, 10
    fwd = np.zeros((H, W, 4), np.int16)
    fwd[..., 0] = 1      # u
    fwd[..., 2] = 2      # d0
    fwd[..., 3] = 3      # d1
    # exact inverse vector everywhere: (d1 - d0 - u, -v, d1, d0)
    inv = np.zeros((H, W, 4), np.int16)
    inv[..., 0] = 3 - 2 - 1
    inv[..., 2] = 3
    inv[..., 3] = 2
    v, e = oracle.consistency(fwd, inv, 0)
    inb = np.zeros((H, W), bool)
    inb[:, 2:9] = True
    assert np.array_equal(v.astype(bool), inb) and np.all(e[inb] == 0)
    # disparity error of 1 passes at tau = 1, fails at tau = 0; 2 fails at tau = 1
    for delta, tau, expect in ((1, 1, 1), (1, 0, 0), (2, 1, 0)):
        f2 = fwd.copy()
        f2[..., 2] += delta
        inb2 = np.zeros((H, W), bool)
        inb2[:, 2 + delta:9] = True
        v, e = oracle.consistency(f2, inv, tau)
        assert np.all(v[inb2] == expect)
        # d0 error enters e0 and the flow term
        assert np.all(e[inb2] == delta * delta)
    # Euclidean flow check: (1, 1) error fails at tau = 1, passes at tau = 2
    i2 = inv.copy()
    i2[..., 0] += 1
    i2[..., 1] += 1
    assert np.all(oracle.consistency(fwd, i2, 1)[0][inb] == 0)
    assert np.all(oracle.consistency(fwd, i2, 2)[0][inb] == 1)
    assert np.all(oracle.consistency(fwd, i2, 2)[1][inb] == 2)


# ------------------------------------------------------------ whole pair ----
def test_match_pair_tiny_recovers_most_of_ground_truth():
    from sff_inputs import tiny_spec, tiny_params
    sc = make_scene(tiny_spec())
    p = tiny_params()
    out = oracle.match_pair(sc.stack(), p, seed=1)
    valid = out["valid"].astype(bool)
    gt = sc.gt_fwd
    epe = np.abs(out["hyp"][0].astype(int) - gt.astype(int)).max(axis=-1)
    assert valid.mean() > 0.3
    # consistent matches are accurate
    assert (epe[valid] <= 1).mean() > 0.9
    again = oracle.match_pair(sc.stack(), p, seed=1, nthreads=1)
    for k in out:
        assert np.array_equal(out[k], again[k])
