"""Pins of the oracle's scale simulation and WHT features (Section 3.1) against
library routines, closed forms and invariants."""
import os

import numpy as np
import pytest

import oracle
from sff_inputs import make_scene, smoothed_noise, small_spec
from tests import indep

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Philox ----
def test_philox_known_answers():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(t, 16) for t in line.split()])
    assert len(rows) == 3
    for r in rows:
        out = oracle.philox4x32_10(r[0:4], r[4:6])
        assert [int(v) for v in out] == r[6:10]


@pytest.mark.parametrize("level,t", [(0, 0), (0, 5), (1, 2), (2, 0)])
def test_rs_offsets_cover_range_uniformly(level, t):
    n = 1 << level
    r0 = 32
    r = max(1, r0 >> t) * n
    big = 10_000
    centre = np.array([0, 0, 5000, 5000], np.int16)
    offs = []
    for it in range(40):
        for j in range(120):
            c = oracle.rs_candidate(7, level, 1, 3, j, 200, it, t, r0, big, big, centre)
            offs.append(c.astype(np.int64) - centre)
    offs = np.array(offs)
    assert offs.min() == -r and offs.max() == r or 2 * r + 1 > 200  # extremes reached
    assert np.all(np.abs(offs) <= r)
    # chi-square over 8 groups of consecutive integers, expected counts in
    # proportion to the number of integers in each group
    vals = np.arange(-r, r + 1)
    groups = np.array_split(vals, 8)
    for c in range(4):
        if 2 * r + 1 < 8 * 4:
            continue
        obs = np.array([np.isin(offs[:, c], g).sum() for g in groups])
        exp = np.array([len(g) for g in groups]) * len(offs) / (2 * r + 1)
        chi2 = ((obs - exp) ** 2 / exp).sum()
        assert chi2 < 30.0  # 7 dof, p ~ 1e-4


def test_rs_streams_are_distinct_and_clamped():
    centre = np.array([30, -30, 1, 60], np.int16)
    a = oracle.rs_candidate(1, 0, 1, 2, 3, 50, 0, 0, 32, 32, 64, centre)
    b = oracle.rs_candidate(1, 0, -1, 2, 3, 50, 0, 0, 32, 32, 64, centre)
    c = oracle.rs_candidate(2, 0, 1, 2, 3, 50, 0, 0, 32, 32, 64, centre)
    d = oracle.rs_candidate(1, 0, 1, 2, 3, 50, 1, 0, 32, 32, 64, centre)
    assert len({tuple(a), tuple(b), tuple(c), tuple(d)}) == 4
    for t in range(6):
        for it in range(20):
            h = oracle.rs_candidate(9, 0, 1, 1, 1, 8, it, t, 32, 32, 64, centre)
            assert -32 <= h[0] <= 32 and -32 <= h[1] <= 32
            assert 0 <= h[2] <= 64 and 0 <= h[3] <= 64


# -------------------------------------------------------------- Lanczos ----
@pytest.mark.parametrize("n", [2, 4, 8])
def test_lanczos_table_sums_and_symmetry(n):
    t = oracle.lanczos_q14(n)
    assert t.shape == (n, 6)
    assert np.all(t.sum(axis=1) == 16384)
    # phase p and n-1-p are mirror images about the pixel centre
    assert np.array_equal(t, t[::-1, ::-1])


@pytest.mark.parametrize("n", [2, 4])
def test_lanczos_table_matches_fp64_weights(n):
    t = oracle.lanczos_q14(n)
    for p in range(n):
        s = (p + 0.5) / n - 0.5
        f = s - np.floor(s)
        d = f + 2 - np.arange(6)
        w = np.sinc(d) * np.sinc(d / 3)
        w = w / w.sum() * 16384
        assert np.all(np.abs(t[p] - w) <= 3.0)


def test_smooth_identity_and_constants():
    rng = np.random.default_rng(0)
    img = rng.integers(0, 256, (13, 17, 3), dtype=np.uint8)
    assert np.array_equal(oracle.smooth(img, 1), img)
    for n in (2, 4, 8):
        const = np.full((21, 30, 2), 173, np.uint8)
        assert np.array_equal(oracle.smooth(const, n), const)


@pytest.mark.parametrize("n", [2, 4])
def test_smooth_mirror_symmetry(n):
    rng = np.random.default_rng(1)
    img = smoothed_noise(rng, 8 * n, 12 * n, 2, 1.0)
    out = oracle.smooth(img, n)
    flipped = oracle.smooth(img[:, ::-1].copy(), n)
    assert np.array_equal(flipped, out[:, ::-1])
    flipped = oracle.smooth(img[::-1].copy(), n)
    assert np.array_equal(flipped, out[::-1])


@pytest.mark.parametrize("n", [2, 4])
def test_smooth_against_fp64_lanczos(n):
    """Area mean then separable Lanczos-3 resampling in FP64 with np.sinc; the
    integer pipeline differs only by its two roundings and the Q14 weights."""
    rng = np.random.default_rng(2)
    H, W = 10 * n, 14 * n
    img = smoothed_noise(rng, H, W, 1, 1.2)
    A = img[:, :, 0].astype(np.float64).reshape(H // n, n, W // n, n).mean(axis=(1, 3))
    A = np.floor(A + 0.5)

    def resample(M, axis_len, out_len):
        x = np.arange(out_len)
        s = (x + 0.5) / n - 0.5
        base = np.floor(s).astype(int) - 2
        R = np.zeros((out_len, axis_len))
        for t in range(6):
            tap = base + t
            w = np.sinc(s - tap) * np.sinc((s - tap) / 3)
            np.add.at(R, (x, np.clip(tap, 0, axis_len - 1)), w)
        R /= R.sum(axis=1, keepdims=True)
        return R

    Rx = resample(None, W // n, W)
    Ry = resample(None, H // n, H)
    ref = Ry @ A @ Rx.T
    ref = np.clip(ref, 0, 255)
    out = oracle.smooth(img, n)[:, :, 0].astype(np.float64)
    diff = np.abs(out - ref)
    assert diff.max() <= 2.0
    assert diff.mean() < 0.5


# ------------------------------------------------------------------ WHT ----
def test_sequency_walsh_is_orthogonal():
    W8 = indep.sequency_walsh(8)
    assert np.array_equal(W8 @ W8.T, 8 * np.eye(8, dtype=np.int64))


@pytest.mark.parametrize("n", [1, 2, 4])
def test_wht_matches_scipy_hadamard(n):
    rng = np.random.default_rng(3)
    S = rng.integers(0, 256, (29, 37, 2), dtype=np.uint8)
    D = oracle.wht(S, n)
    pts = [(0, 0), (28, 36), (5, 33), (14, 2), (13, 18)] + \
          [tuple(p) for p in rng.integers(0, [29, 37], (20, 2))]
    for (y, x) in pts:
        for c in range(2):
            P = indep.patch(S, y, x, c, n)
            ref = indep.wht_block(P)
            assert np.array_equal(D[y, x, c].reshape(4, 4).astype(np.int64), ref)


def test_wht_inverse_gives_bin_sums_and_parseval():
    rng = np.random.default_rng(4)
    S = rng.integers(0, 256, (16, 16, 1), dtype=np.uint8)
    D = oracle.wht(S, 1).astype(np.int64)
    W4 = indep.sequency_walsh(4)
    B = indep.bin_sums(S, 1)
    for y in range(16):
        for x in range(16):
            c = D[y, x, 0].reshape(4, 4)
            # inverse 4x4 WHT: B = W4^T c W4 / 16
            assert np.array_equal(W4.T @ c @ W4, 16 * B[y, x, 0])
            assert (c ** 2).sum() == 16 * (B[y, x, 0] ** 2).sum()


def test_wht_constant_patch_and_range():
    S = np.full((9, 9, 1), 200, np.uint8)
    D = oracle.wht(S, 2)
    assert np.all(D[..., 0] == 64 * 200)
    assert np.all(D[..., 1:] == 0)
    chk = ((np.indices((20, 20)).sum(axis=0) % 2) * 255).astype(np.uint8)[..., None]
    D = oracle.wht(chk, 1).astype(np.int64)
    assert np.abs(D).max() <= 64 * 255
    full = oracle.wht(np.full((8, 8, 1), 255, np.uint8), 1)
    assert full[0, 0, 0, 0] == 16320


def test_features_level_composes_smooth_and_wht():
    sc = make_scene(small_spec(24, 40, 3, seed=11))
    for level in (0, 1, 2):
        n = 1 << level
        D = oracle.features(sc.l0, level)
        assert np.array_equal(D, oracle.wht(oracle.smooth(sc.l0, n), n))


@pytest.mark.parametrize("level", [0, 1, 2])
def test_descriptor_distance_is_16x_bin_distance(level):
    """Squared distance of two WHT descriptors (any two pixels, any two images,
    borders included) = 16 x squared distance of their 2x2-bin grids: the
    4-point sequency Walsh matrix is orthogonal with W W^T = 4 I per axis."""
    rng = np.random.default_rng(40 + level)
    n = 1 << level
    a = rng.integers(0, 256, (23, 31, 3), dtype=np.uint8)
    b = rng.integers(0, 256, (23, 31, 3), dtype=np.uint8)
    Da, Db = oracle.features(a, level).astype(np.int64), oracle.features(b, level).astype(np.int64)
    Ba = indep.bin_sums(oracle.smooth(a, n) if n > 1 else a, n)
    Bb = indep.bin_sums(oracle.smooth(b, n) if n > 1 else b, n)
    for _ in range(300):
        y0, x0, y1, x1 = rng.integers(0, 23), rng.integers(0, 31), rng.integers(0, 23), rng.integers(0, 31)
        d = ((Da[y0, x0] - Db[y1, x1]) ** 2).sum()
        assert d == 16 * ((Ba[y0, x0] - Bb[y1, x1]) ** 2).sum()
