"""Pins of the initialisation with several temporal leaves (Section 3.1,
"Initialization": all combinations of the leaves compared by eq. (1))."""
import numpy as np
import pytest

import oracle
from sff_inputs import make_scene, small_spec
from tests import indep


def _descs(sc, level):
    imgs = sc.stack()
    return [oracle.features(imgs[m], level) for m in range(4)]


def _bins(sc, level):
    """Bin sums of the level's smoothed images (smoothing is pinned on its own)."""
    n = 1 << level
    return [indep.bin_sums(oracle.smooth(im, n), n) for im in sc.stack()]


@pytest.mark.parametrize("leaves", [1, 2, 4, 7])
@pytest.mark.parametrize("s", [1, -1])
def test_leaves_match_brute_force(leaves, s):
    for (H, W, C, level, seed) in ((18, 26, 1, 0, 3), (21, 33, 3, 1, 4), (16, 40, 2, 1, 5)):
        sc = make_scene(small_spec(H, W, C, seed, flow_max=6, d_range=(0, 8)))
        D = _descs(sc, level)
        B = _bins(sc, level)
        fmax, dmax = 6, 8
        hyp, cost = oracle.init_nn(D, level, s, fmax, dmax, leaves=leaves)
        bh, bj = indep.brute_init_leaves(B, s, level, fmax, dmax, leaves)
        assert np.array_equal(hyp, bh), (H, W, C, level, leaves, s)
        # every target lies in the image, so the stored eq. (1) cost is the
        # combination's T + S + X distance
        assert np.array_equal(cost.astype(np.int64), bj)


def test_more_leaves_never_worse_and_all_leaves_is_the_joint_optimum():
    H, W, C, level, s = 14, 22, 1, 0, 1
    sc = make_scene(small_spec(H, W, C, 9, flow_max=5, d_range=(0, 6)))
    D = _descs(sc, level)
    fmax, dmax = 5, 6
    prev = None
    for leaves in (1, 2, 3, 5, 8, 200):
        _, cost = oracle.init_nn(D, level, s, fmax, dmax, leaves=leaves)
        if prev is not None:
            assert (cost <= prev).all()
        prev = cost
    # 200 leaves exceed the 11 x 11 temporal box: the joint optimum over every
    # (u, v, d1) combination, found by exhaustive search
    B = _bins(sc, level)
    _, bj = indep.brute_init_leaves(B, s, level, fmax, dmax, 10 ** 6)
    assert np.array_equal(prev.astype(np.int64), bj)
