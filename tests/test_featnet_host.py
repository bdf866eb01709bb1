"""Host-side logic of the learned-feature path: triple sampling from consistent
matches and the match-quality summary (no GPU needed)."""
import numpy as np

from paper_1710_10096_amd.featnet import TripletPool, match_quality


def test_triplet_pool_indices_follow_the_vectors():
    H, W = 20, 30
    hyp = np.zeros((H, W, 4), np.int16)
    hyp[..., 0] = 2
    hyp[..., 1] = -1
    hyp[..., 2] = 3
    hyp[..., 3] = 4
    valid = np.zeros((H, W), bool)
    valid[5:15, 8:25] = True
    pool = TripletPool(hyp, valid)
    rng = np.random.default_rng(0)
    t = pool.sample(rng, 5000).astype(np.int64)
    HW = H * W
    a, p, n = t[:, 0], t[:, 1], t[:, 2]
    assert (a < HW).all() and (p >= HW).all() and (p < 4 * HW).all()
    ay, ax = a // W, a % W
    assert valid[ay, ax].all()
    view = p // HW
    py, px = (p % HW) // W, (p % HW) % W
    exp = {1: (ay - 1, ax + 2), 2: (ay, ax - 3), 3: (ay - 1, ax + 2 - 4)}
    for v in (1, 2, 3):
        s = view == v
        assert s.any()
        assert np.array_equal(py[s], exp[v][0][s]) and np.array_equal(px[s], exp[v][1][s])
    # negatives: same view, 3..16 px away (before clamping to the image)
    assert np.array_equal(n // HW, view)
    ny, nx = (n % HW) // W, (n % HW) % W
    dist = np.hypot(ny - py, nx - px)
    inside = (nx > 0) & (nx < W - 1) & (ny > 0) & (ny < H - 1)
    assert (dist[inside] >= 2.0).all() and (dist <= 16.0 + 0.75).all()  # rounding of cos, sin


def test_match_quality_summary():
    gt = np.zeros((4, 5, 4), np.int16)
    hyp = gt.copy()
    hyp[0, 0, 0] = 3
    hyp[0, 0, 1] = 4          # flow error 5 px
    hyp[1, 1, 2] = 2          # d0 error 2
    valid = np.ones((4, 5), np.uint8)
    valid[3] = 0
    ok = np.ones((4, 5), bool)
    q = match_quality(hyp, valid, gt, ok)
    assert q["consistent_frac"] == 15 / 20
    assert np.isclose(q["flow_epe"], 5 / 15)
    assert np.isclose(q["d0_err"], 2 / 15)
    assert np.isclose(q["outliers_3px"], 1 / 15)
