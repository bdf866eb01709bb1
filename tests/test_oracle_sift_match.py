"""Pins of the oracle's full-resolution matcher with the SIFT-PCA cost
(Section 3.1, "Matching Cost", eq. (1), and "Multi-Scale Propagation"): the
FP32 cost against the FP64 definition of eq. (1), the matcher's invariants
(costs never rise, the cost field is the cost of the field, independent of
pixel order and thread count, never below the exhaustive optimum on a tiny
search space), and recovery of a pure translation scene."""
import numpy as np

import oracle
from oracle import sift_pca as sp


def _phi(rng, H, W, smooth=True):
    phi = rng.standard_normal((4, H, W, 3))
    if smooth:
        from scipy.ndimage import gaussian_filter
        phi = np.stack([np.stack([gaussian_filter(phi[m, :, :, c], 1.0, mode="nearest")
                                  for c in range(3)], -1) for m in range(4)])
    return phi.astype(np.float32)


def _hyp(rng, H, W, f, d):
    return np.stack([rng.integers(-f, f + 1, (H, W)), rng.integers(-f, f + 1, (H, W)),
                     rng.integers(0, d + 1, (H, W)), rng.integers(0, d + 1, (H, W))], -1).astype(np.int16)


def test_fp32_cost_matches_the_fp64_definition():
    rng = np.random.default_rng(1)
    H, W = 17, 23
    phi = _phi(rng, H, W, smooth=False)
    hyp = _hyp(rng, H, W, 30, 20)        # many targets clamped at the borders
    for s in (1, -1):
        want = sp.cost(phi.astype(np.float64), hyp, s)
        got = oracle.cost_sift(phi, hyp, s).astype(np.float64)
        # 147 non-negative terms, each a few roundings: relative error < 150 u
        assert np.all(np.abs(got - want) <= 150 * 2.0 ** -24 * want + 1e-6)


def test_matcher_invariants():
    rng = np.random.default_rng(2)
    H, W = 20, 26
    phi = _phi(rng, H, W)
    start = _hyp(rng, H, W, 4, 4)
    c0 = oracle.cost_sift(phi, start, 1)
    h, c = oracle.match_sift(phi, start, 1, 7, iters=3, rs_r0=4, rs_samples=3, fmax=6, dmax=6)
    assert np.all(c <= c0)                                   # own vector is always a candidate
    assert np.array_equal(c, oracle.cost_sift(phi, h, 1))   # stored cost = cost of the field
    assert np.all(np.abs(h[..., :2]) <= 6) and np.all((h[..., 2:] >= 0) & (h[..., 2:] <= 6))
    # red-black schedule: independent of the visiting order and the thread count
    h2, c2 = oracle.match_sift(phi, start, 1, 7, iters=3, rs_r0=4, rs_samples=3, fmax=6, dmax=6,
                               order=1, nthreads=1)
    h3, c3 = oracle.match_sift(phi, start, 1, 7, iters=3, rs_r0=4, rs_samples=3, fmax=6, dmax=6,
                               nthreads=4)
    assert np.array_equal(h, h2) and np.array_equal(c, c2)
    assert np.array_equal(h, h3) and np.array_equal(c, c3)
    # zero iterations: the field is kept and only its cost is computed
    h0, cz = oracle.match_sift(phi, start, 1, 7, iters=0, rs_r0=4, rs_samples=3, fmax=6, dmax=6)
    assert np.array_equal(h0, start) and np.array_equal(cz, c0)


def test_never_below_the_exhaustive_optimum():
    rng = np.random.default_rng(3)
    H, W, F, D = 9, 11, 2, 3
    phi = _phi(rng, H, W)
    best = np.full((H, W), np.inf, np.float32)
    for u in range(-F, F + 1):
        for v in range(-F, F + 1):
            for d0 in range(D + 1):
                for d1 in range(D + 1):
                    hyp = np.zeros((H, W, 4), np.int16) + np.array([u, v, d0, d1], np.int16)
                    best = np.minimum(best, oracle.cost_sift(phi, hyp, -1))
    h, c = oracle.match_sift(phi, np.zeros((H, W, 4), np.int16), -1, 3, iters=6, rs_r0=4,
                             rs_samples=6, fmax=F, dmax=D)
    assert np.all(c >= best)
    assert (c == best).mean() > 0.3          # reported reach, loosely bounded


def test_recovers_a_translation_scene():
    """Four views of one image translated by (u, v), disparities d0, d1; the
    oracle's SIFT-PCA features; a start one pixel off everywhere: the matcher
    finds the true vector at interior pixels, where eq. (1) is zero."""
    rng = np.random.default_rng(11)
    H, W, pad = 36, 48, 24
    big = rng.integers(0, 256, (H + 2 * pad, W + 2 * pad, 3), dtype=np.uint8)
    u, v, d0, d1 = 5, -2, 7, 4

    def crop(dy, dx):
        return big[pad + dy:pad + dy + H, pad + dx:pad + dx + W]
    imgs = np.stack([crop(0, 0), crop(-v, -u), crop(0, d0), crop(-v, -(u - d1))])
    phi = sp.sift_pca_features(imgs)["phi"].astype(np.float32)
    start = np.zeros((H, W, 4), np.int16) + np.array([u + 1, v, d0 - 1, d1 + 1], np.int16)
    h, c = oracle.match_sift(phi, start, 1, 5, iters=4, rs_r0=4, rs_samples=6, fmax=16, dmax=16)
    inner = (slice(12, H - 12), slice(20, W - 20))
    assert np.all(h[inner] == np.array([u, v, d0, d1]))
    assert np.all(c[inner] < 1e-5)
