"""Pins of the SIFT-PCA form of eq. (1) (Section 3.1, "Matching Cost"):
orientation conventions by ramps and by 90-degree rotation, the cell geometry
by a step edge, the normalisation on hand-made vectors, translation
equivariance, PCA against an SVD of the centred data (a different LAPACK
route) and a planted spectrum, and the cost against hand-built feature maps
(unsquared norms, clamping at the final coordinate, both directions) and a
pure translation scene (zero at the true vector)."""
import numpy as np
import pytest

from oracle import sift_pca as sp


def _img(g):
    return np.repeat(np.asarray(g, np.float64)[..., None], 3, axis=2).astype(np.uint8)


def test_ramps_fix_the_bin_convention():
    H, W = 12, 14
    ys, xs = np.indices((H, W))
    cases = [(2 * xs, 0, 4.0), (ys, 2, 2.0), (xs + ys, 1, 2 * np.sqrt(2)), (-xs, 4, 2.0),
             (-ys, 6, 2.0)]
    for g, b, m in cases:
        O = sp.orientation_energy(g.astype(np.float64))
        inner = O[:, 1:-1, 1:-1]
        assert np.allclose(inner[b], m), b
        assert np.allclose(np.delete(inner, b, axis=0), 0), b
    # between two bin centres: gx = 4, gy = 2 -> atan(1/2) = 26.57 degrees
    O = sp.orientation_energy((2 * xs + ys).astype(np.float64))[:, 5, 5]
    f = np.degrees(np.arctan2(2, 4)) / 45
    assert np.allclose(O[0], np.hypot(4, 2) * (1 - f)) and np.allclose(O[1], np.hypot(4, 2) * f)
    assert np.allclose(O[2:], 0)


def test_rotation_by_90_degrees_shifts_the_bins_by_two():
    rng = np.random.default_rng(3)
    g = rng.integers(0, 256, (9, 13)).astype(np.float64)
    O = sp.orientation_energy(g)
    Or = sp.orientation_energy(np.rot90(g))
    # (gx, gy) -> (gy, -gx): the orientation turns by -90 degrees, two bins
    want = np.stack([np.rot90(O[(b + 2) % 8]) for b in range(8)])
    assert np.allclose(Or, want, atol=1e-12)


def test_step_edge_fixes_the_cell_geometry():
    H, W, X0 = 30, 40, 20
    g = np.zeros((H, W))
    g[:, X0:] = 100
    d = sp.dense_sift(_img(g))
    # at x = X0 the edge columns X0 - 1 and X0 fall in cell columns 1 and 2
    v = d[15, X0].reshape(4, 4, 8)
    want = np.zeros((4, 4, 8))
    want[:, 1:3, 0] = 1 / np.sqrt(8)
    assert np.allclose(v, want)
    # at x = X0 + 6 only cell column 0 holds the edge column X0 (X0 - 1 is out)
    v = d[15, X0 + 6].reshape(4, 4, 8)
    want = np.zeros((4, 4, 8))
    want[:, 0, 0] = 0.5
    assert np.allclose(v, want)
    # far from the edge the descriptor is zero
    assert not d[15, 2].any() and not d[15, W - 8].any()


def test_ramp_descriptor_and_constant_image():
    H, W = 24, 26
    xs = np.indices((H, W))[1]
    d = sp.dense_sift(_img(3 * xs))
    v = d[12, 13].reshape(16, 8)
    # 16 equal cells -> 1/4 each, clamped to 0.2, renormalised to 1/4
    assert np.allclose(v[:, 0], 0.25) and np.allclose(v[:, 1:], 0)
    assert not sp.dense_sift(np.full((7, 9, 3), 77, np.uint8)).any()


def test_normalise_hand_made():
    v = np.zeros(128)
    v[:2] = (3, 4)
    out = sp.normalise(v)
    assert np.allclose(out[:2], 1 / np.sqrt(2)) and not out[2:].any()
    v = np.zeros(128)
    v[:50] = 1
    assert np.allclose(sp.normalise(v)[:50], 1 / np.sqrt(50))  # 0.141 < 0.2: untouched
    assert not sp.normalise(np.zeros(128)).any()
    rng = np.random.default_rng(0)
    out = sp.normalise(rng.random((20, 128)) ** 8)
    assert np.allclose(np.linalg.norm(out, axis=1), 1)


def test_translation_equivariance():
    rng = np.random.default_rng(5)
    big = rng.integers(0, 256, (40, 60, 3), dtype=np.uint8)
    a = sp.dense_sift(big[5:35, 5:55])
    b = sp.dense_sift(big[8:38, 2:52])      # shifted by (+3, -3)
    # interior pixels whose 12 x 12 support (+1 for the gradient) is inside both crops
    assert np.allclose(a[10:20, 13:40], b[7:17, 16:43])


def test_pca_against_svd_and_a_planted_spectrum():
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.standard_normal((128, 128)))
    sig = np.concatenate([[9.0, 5.0, 3.0], np.linspace(1.0, 0.1, 125)])
    F = rng.standard_normal((6000, 128)) * sig @ Q.T + rng.random(128)
    mean, cov, w, axes = sp.pca(F)
    Xc = F - F.mean(axis=0)
    _, s, Vt = np.linalg.svd(Xc, full_matrices=False)
    assert np.allclose(w, s[:3] ** 2 / len(F), rtol=1e-10)
    assert np.allclose(axes, sp.sign_fix(Vt[:3]), atol=1e-9)
    assert np.allclose(cov, np.cov(F.T, bias=True), atol=1e-12)
    # the planted axes, up to sampling error
    assert np.all(np.abs(np.sum(axes * sp.sign_fix(Q[:, :3].T), axis=1)) > 0.99)
    for r in range(3):
        k = np.argmax(np.abs(axes[r]))
        assert axes[r, k] > 0
    # centring: a constant added to every row changes the mean only
    m2, c2, w2, a2 = sp.pca(F + 5.0)
    assert np.allclose(m2, mean + 5) and np.allclose(c2, cov) and np.allclose(a2, axes)


def test_cost_uses_unsquared_norms_and_both_directions():
    H, W = 6, 7
    phi = np.zeros((4, H, W, 3))
    phi[1] = (3, 4, 0)     # l1
    phi[2] = (0, 0, 2)     # r0
    phi[3] = (1, 0, 0)     # r1
    hyp = np.zeros((H, W, 4), np.int16)
    assert np.allclose(sp.cost(phi, hyp, 1), 49 * (5 + 2 + 1))
    # inverse direction: R = r1, (T, S, X) = (r0, l1, l0)
    assert np.allclose(sp.cost(phi, hyp, -1), 49 * (np.hypot(1, 2) + np.hypot(2, 4) + 1))


def test_cost_clamps_the_final_coordinate():
    H, W = 5, 11
    phi = np.zeros((4, H, W, 3))
    phi[1, :, :, 0] = np.arange(W)          # T holds its column index
    hyp = np.zeros((H, W, 4), np.int16)
    hyp[..., 0] = 100                       # far to the right
    hyp[..., 2] = 3
    hyp[..., 3] = 3                          # S and X read l0 = r0 = r1 = 0 (zero)
    c = sp.cost(phi, hyp, 1)
    # every window pixel's temporal target clamps to column W - 1
    assert np.allclose(c, 49 * (W - 1))
    hyp[..., 0] = 0
    c = sp.cost(phi, hyp, 1)
    x = 0   # window columns -3..3 clamp to 0, 0, 0, 0, 1, 2, 3 at x = 0
    assert np.isclose(c[2, x], 7 * (0 + 0 + 0 + 0 + 1 + 2 + 3))


def test_cost_is_zero_at_the_true_vector_of_a_translation_scene():
    rng = np.random.default_rng(11)
    H, W, pad = 36, 48, 24
    big = rng.integers(0, 256, (H + 2 * pad, W + 2 * pad, 3), dtype=np.uint8)
    u, v, d0, d1 = 5, -2, 7, 4
    # view(p) = big(p + pad + shift): l0 at 0, l1 at -(u, v) so l1(p + (u, v)) = l0(p)
    def crop(dy, dx):
        return big[pad + dy:pad + dy + H, pad + dx:pad + dx + W]
    imgs = np.stack([crop(0, 0), crop(-v, -u), crop(0, d0), crop(-v, -(u - d1))])
    f = sp.sift_pca_features(imgs)
    hyp = np.zeros((H, W, 4), np.int16) + np.array([u, v, d0, d1], np.int16)
    c = sp.cost(f["phi"], hyp, 1)
    inner = c[12:H - 12, 20:W - 20]
    assert np.allclose(inner, 0, atol=1e-9)
    wrong = hyp.copy()
    wrong[..., 0] += 1
    assert np.all(sp.cost(f["phi"], wrong, 1)[12:H - 12, 20:W - 20] > 1e-3)
