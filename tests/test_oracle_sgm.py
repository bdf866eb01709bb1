"""Pins of the disparity fill by semi-global matching (Section 3.1, last
paragraph of "Consistency Check"; Hirschmueller 2008): census and Hamming
cost by NumPy bit operations, every path aggregation against an exhaustive
search over disparity sequences along the path, the zero-penalty closed
form, and the fill rule."""
import itertools

import numpy as np
import pytest

import oracle

DIRS = [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (1, -1), (-1, 1)]


def _census_np(g):
    H, W = g.shape
    pad = np.pad(g.astype(np.int32), 2, mode="edge")
    out = np.zeros((H, W), np.uint32)
    k = 0
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            if dx == 0 and dy == 0:
                continue
            nb = pad[2 + dy:2 + dy + H, 2 + dx:2 + dx + W]
            out |= (nb < g).astype(np.uint32) << np.uint32(k)
            k += 1
    return out


def test_grey_census_and_cost():
    rng = np.random.default_rng(1)
    img = rng.integers(0, 256, (9, 13, 3), dtype=np.uint8)
    g = oracle.grey(img)
    assert np.array_equal(g, ((img.astype(np.int32).sum(axis=2) + 1) // 3).astype(np.uint8))
    cl, cr = oracle.census(g), _census_np(g[::-1].copy())
    assert np.array_equal(cl, _census_np(g))
    D = 6
    cost = oracle.sgm_cost(cl, cr, D)
    H, W = g.shape
    for d in range(D):
        xs = np.clip(np.arange(W) - d, 0, W - 1)
        x = (cl ^ cr[:, xs]).view(np.uint8).reshape(H, W, 4)
        assert np.array_equal(cost[..., d], np.unpackbits(x, axis=-1).sum(axis=-1))


def _brute_path(cost, P1, P2, dx, dy, y, x):
    """min over disparity sequences along the path ending at (y, x) of the summed
    costs plus penalties (P1 for |change| = 1, P2 for larger), per end disparity."""
    H, W, D = cost.shape
    chain = []
    while 0 <= x < W and 0 <= y < H:
        chain.append((y, x))
        y, x = y - dy, x - dx
    chain = chain[::-1]
    best = np.full(D, np.iinfo(np.int64).max, np.int64)
    for seq in itertools.product(range(D), repeat=len(chain)):
        tot = sum(int(cost[py, px, d]) for (py, px), d in zip(chain, seq))
        for a, b in zip(seq[:-1], seq[1:]):
            tot += 0 if a == b else (P1 if abs(a - b) == 1 else P2)
        best[seq[-1]] = min(best[seq[-1]], tot)
    return best


@pytest.mark.parametrize("dxdy", DIRS)
def test_path_aggregation_is_the_path_minimum(dxdy):
    """L_r(p, .) is the minimal path cost up to a per-pixel constant (the
    subtracted minima), so both agree after removing their minimum."""
    rng = np.random.default_rng(3)
    H, W, D = 4, 5, 3
    cost = rng.integers(0, 25, (H, W, D)).astype(np.uint8)
    P1, P2 = 3, 9
    L = oracle.sgm_path(cost, P1, P2, *dxdy)
    for y in range(H):
        for x in range(W):
            b = _brute_path(cost, P1, P2, dxdy[0], dxdy[1], y, x)
            assert np.array_equal(L[y, x] - L[y, x].min(), b - b.min()), (dxdy, y, x)


def test_zero_penalties_reduce_to_winner_take_all():
    rng = np.random.default_rng(4)
    left = rng.integers(0, 256, (11, 17, 3), dtype=np.uint8)
    right = rng.integers(0, 256, (11, 17, 3), dtype=np.uint8)
    D = 7
    disp = oracle.sgm(left, right, D, 0, 0)
    cost = oracle.sgm_cost(oracle.census(oracle.grey(left)), oracle.census(oracle.grey(right)), D)
    assert np.array_equal(disp, cost.argmin(axis=-1).astype(np.int16))  # first minimum


def test_recovers_a_constant_disparity():
    rng = np.random.default_rng(5)
    H, W, d = 24, 48, 5
    left = rng.integers(0, 256, (H, W + d, 3), dtype=np.uint8)
    # right(x) = left(x + d): the left pixel x matches right pixel x - d
    right = left[:, d:]
    left = left[:, :W]
    disp = oracle.sgm(left, right, 12, 3, 24)
    assert (disp[:, d + 2:W - 2] == d).mean() > 0.98


def test_fill_rule():
    hyp = np.zeros((1, 6, 4), np.int16)
    hyp[0, :, 2] = [0, 1, 5, 3, 4, 4]
    valid = np.array([[1, 0, 0, 0, 0, 0]], np.uint8)
    disp = np.array([[9, 2, 0, 5, 4, 6]], np.int16)
    fill = oracle.disparity_fill(hyp, valid, disp, 1)
    # kept by the joint check; |1-2| <= 1; target x - d0 = 2 - 5 < 0; |3-5| > 1;
    # equal; |4-6| > 1
    assert fill[0].tolist() == [1, 1, 0, 0, 1, 0]
