"""Pins of the oracle's region filter (Section 3.1, "Consistency Check",
second step; s_c of Section 5) and sparsification (Section 3.2)."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from tests import indep


def _field(rng, H, W, levels=3):
    """Piecewise-constant vectors from a few values so that neighbours are
    often, but not always, within tau of each other."""
    base = rng.integers(-levels, levels + 1, size=(H, W, 4)).astype(np.int16)
    blocks = rng.integers(0, 3, size=(H // 4 + 1, W // 4 + 1, 4)).astype(np.int16) * 3
    return base // 2 + np.repeat(np.repeat(blocks, 4, 0), 4, 1)[:H, :W]


def test_equal_vectors_reduce_to_connected_components():
    """With one vector everywhere the regions are the 4-connected components
    of the consistent mask (scipy.ndimage.label) and every component that
    touches an inconsistent pixel is 'extendable'."""
    rng = np.random.default_rng(7)
    for H, W, s_c in ((30, 41, 12), (17, 9, 5), (25, 25, 150)):
        valid = (rng.random((H, W)) < 0.7).astype(np.uint8)
        hyp = np.zeros((H, W, 4), np.int16) + np.array([3, -2, 5, 6], np.int16)
        lab, n = ndimage.label(valid)  # default structure = 4-connectivity
        size = np.bincount(lab.ravel(), minlength=n + 1)
        touches = np.zeros(n + 1, bool)
        near_invalid = ndimage.binary_dilation(valid == 0, structure=ndimage.generate_binary_structure(2, 1))
        touches[np.unique(lab[(valid == 1) & near_invalid])] = True
        want = (valid == 1) & ~(touches[lab] & (size[lab] < s_c))
        got = oracle.region_filter(hyp, valid, 1, s_c)
        assert np.array_equal(got, want.astype(np.uint8)), (H, W)


@pytest.mark.parametrize("tau", [0, 1, 2])
def test_matches_union_find(tau):
    rng = np.random.default_rng(11 + tau)
    for H, W in ((23, 31), (1, 40), (40, 1), (12, 12)):
        hyp = _field(rng, H, W)
        valid = (rng.random((H, W)) < 0.8).astype(np.uint8)
        for s_c in (1, 4, 20, 150):
            got = oracle.region_filter(hyp, valid, tau, s_c)
            want = indep.region_filter_union_find(hyp, valid, tau, s_c)
            assert np.array_equal(got, want), (H, W, tau, s_c)


def test_hand_made_regions():
    H, W = 40, 40
    hyp = np.zeros((H, W, 4), np.int16)
    valid = np.zeros((H, W), np.uint8)
    # A: 10x10 block of one vector (100 < 150) with a similar outlier next to it
    hyp[2:12, 2:12] = (5, 5, 5, 5)
    valid[2:12, 2:12] = 1
    hyp[12, 5] = (6, 5, 4, 5)          # inconsistent, within 1 of the block
    # B: same block, the outlier next to it differs by 2 -> not extendable
    hyp[2:12, 20:30] = (5, 5, 5, 5)
    valid[2:12, 20:30] = 1
    hyp[12, 25] = (7, 5, 5, 5)
    # C: 13x13 block (169 >= 150) with a similar outlier -> kept
    hyp[20:33, 2:15] = (9, 9, 9, 9)
    valid[20:33, 2:15] = 1
    hyp[33, 5] = (9, 9, 9, 9)
    # D: a row whose vector increases by 1 per pixel (3..14, so never within 1
    # of the zero background) is one region (chained similarity) of 12 pixels;
    # a similar outlier at its end removes it all
    for k in range(12):
        hyp[36, 20 + k] = (3 + k, 0, 0, 0)
    valid[36, 20:32] = 1
    hyp[36, 32] = (14, 0, 0, 0)
    keep = oracle.region_filter(hyp, valid, 1, 150)
    assert keep[2:12, 2:12].sum() == 0
    assert keep[2:12, 20:30].sum() == 100
    assert keep[20:33, 2:15].sum() == 169
    assert keep[36, 20:32].sum() == 0
    # tau = 0: the increasing row falls apart into single pixels, none of which
    # has an identical outlier neighbour except the last one
    keep0 = oracle.region_filter(hyp, valid, 0, 150)
    assert keep0[36, 20:31].sum() == 11 and keep0[36, 31] == 0
    # "smaller than s_c": block A has exactly 100 pixels
    assert oracle.region_filter(hyp, valid, 1, 100)[2:12, 2:12].sum() == 100
    assert oracle.region_filter(hyp, valid, 1, 101)[2:12, 2:12].sum() == 0
    # s_c = 1: nothing is smaller than one pixel, so nothing is removed
    assert np.array_equal(oracle.region_filter(hyp, valid, 1, 1), valid)


def test_sparsify_matches_block_argmin():
    rng = np.random.default_rng(5)
    for H, W in ((9, 9), (10, 14), (1, 7), (7, 1), (2, 2), (31, 47)):
        keep = (rng.random((H, W)) < 0.4).astype(np.uint8)
        err = rng.integers(0, 3, (H, W)).astype(np.uint32)  # many ties
        err[rng.random((H, W)) < 0.1] = np.uint32(0xFFFFFFFF)
        got = oracle.sparsify(keep, err)
        assert got.shape == (-(-H // 3), -(-W // 3))
        assert np.array_equal(got, indep.sparsify_blocks(keep, err)), (H, W)


def test_sparsify_ties_and_empty_blocks():
    keep = np.zeros((3, 6), np.uint8)
    err = np.full((3, 6), 7, np.uint32)
    keep[0, 1] = keep[2, 0] = 1          # block 0: equal errors -> lower index (0, 1)
    got = oracle.sparsify(keep, err)
    assert got.tolist() == [[1, -1]]
    err[2, 0] = 6
    assert oracle.sparsify(keep, err).tolist() == [[12, -1]]
