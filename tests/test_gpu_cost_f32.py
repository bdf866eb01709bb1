"""GPU checks of the FP32 window cost (eq. (1) window form) and its backward
against the FP64 oracle and FP64 central finite differences.

Tolerances (FP32 against FP64): the forward sums 3 x 64 x C non-negative
terms in three nested partial sums (at most 3C + 16 sequential additions per
partial), so its relative error stays below ~(3C + 16) 2^-24 < 1e-5 for C = 32;
the test allows 2e-5.  A gradient entry sums about 192 signed terms (more at
clamped borders) with fused multiply-adds, so the error is bounded by
~192 2^-24 times the sum of the terms' magnitudes; the test allows
1e-4 |g| + 1e-4 mean|g|.
"""
import sys

import numpy as np
import pytest

from oracle import cost_f32 as ocf

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sff():
    import torch
    import paper_1710_10096_amd as m
    assert torch.cuda.is_available()
    return m


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _grad_close(g, ref):
    scale = np.abs(ref).mean()
    return np.abs(g - ref) <= 1e-4 * np.abs(ref) + 1e-4 * scale


def _random_case(seed, B, H, W, C, spread):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((B, 4, H, W, C)).astype(np.float32)
    hyp = np.empty((B, H, W, 4), np.int16)
    hyp[..., :2] = rng.integers(-spread, spread + 1, (B, H, W, 2))
    hyp[..., 2:] = rng.integers(0, spread + 1, (B, H, W, 2))
    g = rng.uniform(0.2, 2.0, (B, H, W)).astype(np.float32)
    return F, hyp, g


@pytest.mark.parametrize("s", [1, -1])
@pytest.mark.parametrize("C", [4, 8])
def test_small_forward_and_backward_match_fp64(sff, s, C):
    B, H, W = 2, 19, 27
    F, hyp, g = _random_case(10 + C + (s > 0), B, H, W, C, spread=9)
    _say("cost_f32 small", s, C)
    cost = sff.sff_cost_f32_fwd(_dev(F), _dev(hyp), s).cpu().numpy()
    grad = sff.sff_cost_f32_bwd(_dev(F), _dev(hyp), s, _dev(g)).cpu().numpy()
    for b in range(B):
        Fb = [F[b, m].astype(np.float64) for m in range(4)]
        ref = ocf.window_cost(Fb, hyp[b], s)
        assert np.allclose(cost[b], ref, rtol=2e-5, atol=0), b
        G = ocf.window_cost_grad(Fb, hyp[b], s, g[b])
        for m in range(4):
            assert _grad_close(grad[b, m], G[m]).all(), (b, m)
    again = sff.sff_cost_f32_bwd(_dev(F), _dev(hyp), s, _dev(g)).cpu().numpy()
    assert np.array_equal(again, grad)  # deterministic


@pytest.mark.parametrize("C", [4, 8, 16, 32, 64])
def test_gradient_kernels_identical(sff, C, monkeypatch):
    """The gradient kernels with C/4 lanes per entry (the default) against one
    lane per entry (SFF_COST_F32_EVAL=lane): every channel adds the same terms
    in the same order, so the gradients agree bit for bit; both against the
    FP64 oracle as above.  The forward in both forms against the oracle."""
    B, H, W = 2, 13, 41
    F, hyp, g = _random_case(100 + C, B, H, W, C, spread=7)
    _say("cost_f32 gradient kernels", C)
    monkeypatch.delenv("SFF_COST_F32_EVAL", raising=False)
    grad = sff.sff_cost_f32_bwd(_dev(F), _dev(hyp), -1, _dev(g)).cpu().numpy()
    monkeypatch.setenv("SFF_COST_F32_EVAL", "lane")
    lane = sff.sff_cost_f32_bwd(_dev(F), _dev(hyp), -1, _dev(g)).cpu().numpy()
    assert np.array_equal(grad, lane)
    Fb = [F[1, m].astype(np.float64) for m in range(4)]
    G = ocf.window_cost_grad(Fb, hyp[1], -1, g[1])
    for m in range(4):
        assert _grad_close(grad[1, m], G[m]).all(), m
    # forward: C/4 lanes per pixel (default; rounds differently from one lane
    # per pixel, same bound) and one lane per pixel, both against the oracle
    ref = ocf.window_cost(Fb, hyp[1], -1)
    c_lane = sff.sff_cost_f32_fwd(_dev(F), _dev(hyp), -1).cpu().numpy()
    monkeypatch.delenv("SFF_COST_F32_EVAL", raising=False)
    c_coop = sff.sff_cost_f32_fwd(_dev(F), _dev(hyp), -1).cpu().numpy()
    assert np.array_equal(c_coop, sff.sff_cost_f32_fwd(_dev(F), _dev(hyp), -1).cpu().numpy())
    for c in (c_coop, c_lane):
        assert np.allclose(c[1], ref, rtol=2e-5, atol=0)


def test_one_pixel_and_one_row_images(sff):
    for (H, W) in ((1, 1), (1, 9), (7, 1)):
        F, hyp, g = _random_case(H * 31 + W, 1, H, W, 4, spread=3)
        cost = sff.sff_cost_f32_fwd(_dev(F), _dev(hyp), 1).cpu().numpy()
        grad = sff.sff_cost_f32_bwd(_dev(F), _dev(hyp), 1, _dev(g)).cpu().numpy()
        Fb = [F[0, m].astype(np.float64) for m in range(4)]
        assert np.allclose(cost[0], ocf.window_cost(Fb, hyp[0], 1), rtol=2e-5)
        G = ocf.window_cost_grad(Fb, hyp[0], 1, g[0])
        for m in range(4):
            assert _grad_close(grad[0, m], G[m]).all(), (H, W, m)


def test_kitti_size_c32_against_finite_differences(sff):
    """Feature maps C = 32 ~ N(0, 1) at 1242 x 375 for the four views, vectors
    fixed to the oracle's forward level-0 field of the KITTI-like pair; loss =
    sum of per-pixel costs; 1000 random entries against FP64 central
    differences (eps 1e-3)."""
    import torch
    import oracle
    from sff_inputs import kitti_params, kitti_spec, make_scene
    sc = make_scene(kitti_spec())
    p = kitti_params()
    H, W = p["H"], p["W"]
    _say("oracle field for the fixed vectors")
    hyp = oracle.match_pair(sc.stack(), p, 2)["hyp"][0]
    rng = np.random.default_rng(4)
    F = rng.standard_normal((1, 4, H, W, 32)).astype(np.float32)
    feat = _dev(F).requires_grad_(True)
    hyp_t = _dev(hyp[None])
    _say("autograd forward/backward")
    cost = sff.MatchCost.apply(feat, hyp_t, 1)
    cost.sum().backward()
    grad = feat.grad.cpu().numpy()[0]
    cost = cost.detach().cpu().numpy()[0]
    torch.cuda.synchronize()
    Fb = [F[0, m].astype(np.float64) for m in range(4)]
    ones = np.ones((H, W))
    # forward on 2000 sampled pixels (borders included)
    ys = np.concatenate([rng.integers(0, H, 1990), [0, H - 1, 0, H - 1, 5]])
    xs = np.concatenate([rng.integers(0, W, 1990), [0, W - 1, W - 1, 0, 0]])
    ys, xs = ys[:2000], xs[:2000]
    ref = ocf.cost_px_at(Fb, hyp, 1, ys, xs)
    assert np.allclose(cost[ys, xs], ref, rtol=2e-5)
    _say("1000 finite differences")
    ent = [(int(rng.integers(4)), int(rng.integers(H)), int(rng.integers(W)), int(rng.integers(32)))
           for _ in range(1000)]
    fdh = ocf.FiniteDifferences(Fb, hyp, 1, ones)
    fd = np.array([fdh.grad_entry(*e, eps=1e-3) for e in ent])
    got = np.array([grad[m, y, x, c] for (m, y, x, c) in ent])
    scale = np.abs(fd).mean()
    assert (np.abs(got - fd) <= 1e-4 * np.abs(fd) + 1e-4 * scale).all()


def test_many_tiles_identical_to_one_lane(sff, monkeypatch):
    """C = 32 at 1 x 200 x 200 (7 tiles of 32 entries a row, 1400 per map,
    three target maps in one launch): the tiled gradient kernels against one
    lane per entry, bit for bit, twice (deterministic)."""
    F, hyp, g = _random_case(77, 1, 200, 200, 32, spread=12)
    _say("cost_f32 many tiles C=32 200x200")
    monkeypatch.delenv("SFF_COST_F32_EVAL", raising=False)
    grad = sff.sff_cost_f32_bwd(_dev(F), _dev(hyp), 1, _dev(g)).cpu().numpy()
    again = sff.sff_cost_f32_bwd(_dev(F), _dev(hyp), 1, _dev(g)).cpu().numpy()
    monkeypatch.setenv("SFF_COST_F32_EVAL", "lane")
    lane = sff.sff_cost_f32_bwd(_dev(F), _dev(hyp), 1, _dev(g)).cpu().numpy()
    assert np.array_equal(grad, again)
    assert np.array_equal(grad, lane)


def test_backward_on_one_stream_identical(sff, monkeypatch):
    """The backward with the reference map's gradient on the helper stream
    (default) against everything on the caller's stream (SFF_COST_F32_SPLIT=0):
    the maps' gradients are disjoint outputs of the same kernels, so the bits
    agree; two pairs, C = 32, several tiles a row."""
    F, hyp, g = _random_case(78, 2, 60, 200, 32, spread=12)
    _say("cost_f32 backward split vs one stream")
    monkeypatch.delenv("SFF_COST_F32_EVAL", raising=False)
    monkeypatch.delenv("SFF_COST_F32_SPLIT", raising=False)
    split = sff.sff_cost_f32_bwd(_dev(F), _dev(hyp), -1, _dev(g)).cpu().numpy()
    monkeypatch.setenv("SFF_COST_F32_SPLIT", "0")
    one = sff.sff_cost_f32_bwd(_dev(F), _dev(hyp), -1, _dev(g)).cpu().numpy()
    assert np.array_equal(split, one)
    Fb = [F[1, m].astype(np.float64) for m in range(4)]
    G = ocf.window_cost_grad(Fb, hyp[1], -1, g[1])
    for m in range(4):
        assert _grad_close(split[1, m], G[m]).all(), m


def test_crowded_centres_use_the_global_lists(sff, monkeypatch):
    """Vectors that send whole rows to one centre cell (u far to the left,
    clamped to column 0): the cells of the first tile of a row hold about
    8 x 300 pixels, more than a tile stages, so that tile reads the sorted
    lists from global memory; same bits as one lane per entry, and the FP64
    oracle's gradient."""
    B, H, W, C = 1, 12, 300, 8
    F, hyp, g = _random_case(5, B, H, W, C, spread=3)
    hyp[..., 0] = -1000
    _say("cost_f32 crowded centres")
    monkeypatch.delenv("SFF_COST_F32_EVAL", raising=False)
    grad = sff.sff_cost_f32_bwd(_dev(F), _dev(hyp), 1, _dev(g)).cpu().numpy()
    monkeypatch.setenv("SFF_COST_F32_EVAL", "lane")
    lane = sff.sff_cost_f32_bwd(_dev(F), _dev(hyp), 1, _dev(g)).cpu().numpy()
    assert np.array_equal(grad, lane)
    Fb = [F[0, m].astype(np.float64) for m in range(4)]
    G = ocf.window_cost_grad(Fb, hyp[0], 1, g[0])
    for m in range(4):
        assert _grad_close(grad[0, m], G[m]).all(), m
