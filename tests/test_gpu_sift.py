"""GPU parity of the SIFT-PCA form of eq. (1) (Section 3.1, "Matching Cost")
against the FP64 oracle.  Tolerances follow the arithmetic:

* descriptors (FP32 on the GPU): gradients are exact integers, the magnitude
  and the orientation weights carry a few ulp (sqrt, atan2), the 9-term cell
  sums and the two normalisations a few more, and the renormalisation after
  the clamp divides by a norm of at least 0.2 (5x): |d| <= 2e-5 per entry;
* covariance (FP64 sums of exact products of the FP32 entries): with delta the
  measured largest descriptor error and |f - mean| <= 1 per entry,
  |d cov| <= 2 delta + delta^2;
* axes: Davis-Kahan, sin(angle_k) <= ||d cov||_2 / gap_k (gap_k the distance
  of lambda_k to the rest of the oracle's spectrum), plus the iteration's
  residual 1e-12 lambda_1 / gap_k; compared up to sign (the sign rule itself is
  checked on the GPU output);
* phi: |d phi_k| <= ||d a_k|| ||f - mean|| + ||d f|| + ||d mean|| + FP32
  rounding of 128 terms;
* cost (147 unsquared 3-vector distances, FP32): |d C| <= 147 * 2 sqrt(3)
  max |d phi| + 150 u C; for the cost kernel alone (same FP32 features on both
  sides) 150 u C.
Inputs are seeded scenes and smoothed noise."""
import sys

import numpy as np
import pytest

import oracle
from oracle import sift_pca as sp
from sff_inputs import kitti_params, kitti_spec, make_scene, params_dict, small_spec
from sff_inputs.scenes import smoothed_noise

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
DESC_TOL = 2e-5


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sff():
    import torch
    import paper_1710_10096_amd as m
    assert torch.cuda.is_available()
    return m


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


SIFT_CASES = [  # H, W, C, nimg, sigma (0: raw noise)
    (7, 9, 3, 2, 1.5), (1, 30, 1, 1, 0), (30, 1, 2, 1, 0), (40, 57, 3, 3, 1.5), (33, 70, 4, 2, 0.8),
    (64, 64, 1, 1, 2.5),
]


@pytest.mark.parametrize("case", SIFT_CASES, ids=[str(c) for c in SIFT_CASES])
def test_dense_sift_parity(sff, case):
    import torch
    H, W, C, n, sig = case
    rng = np.random.default_rng(H * 100 + W + C)
    imgs = np.stack([smoothed_noise(rng, H, W, C, sig) if sig else
                     rng.integers(0, 256, (H, W, C), dtype=np.uint8) for _ in range(n)])
    p = params_dict(H, W, C, levels=1, iters=1)
    _say("dense sift", case)
    got = sff.sff_dense_sift(p, dev(imgs))
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.float64)
    for m in range(n):
        want = sp.dense_sift(imgs[m])
        err = np.abs(got[m] - want).max()
        assert err <= DESC_TOL, (case, m, err)
        norms = np.linalg.norm(got[m], axis=-1)
        assert np.all((np.abs(norms - 1) < 1e-5) | (norms == 0))


def _chain(sff, imgs, p):
    """GPU features of one pair against the oracle, each stage to its bound;
    returns (gpu outputs, oracle outputs, max |d phi|)."""
    import torch
    g = dev(imgs[None])
    out = sff.sff_sift_pca(p, g)
    sift = sff.sff_dense_sift(p, g[0])
    torch.cuda.synchronize()
    ref = sp.sift_pca_features(imgs)
    gs = sift.cpu().numpy().astype(np.float64)
    delta = np.abs(gs - ref["sift"]).max()
    assert delta <= DESC_TOL, delta
    mean, cov = out["mean"].cpu().numpy()[0], out["cov"].cpu().numpy()[0]
    assert np.abs(mean - ref["mean"]).max() <= delta + 1e-12
    dcov = cov - ref["cov"]
    assert np.abs(dcov).max() <= 2 * delta + delta ** 2 + 1e-12
    # axes: Davis-Kahan with the oracle's full spectrum
    lam = np.sort(np.linalg.eigvalsh(ref["cov"]))[::-1]
    dn = np.linalg.norm(dcov, 2) + 1e-12 * lam[0]
    axes, eig = out["axes"].cpu().numpy()[0], out["eigval"].cpu().numpy()[0]
    assert np.allclose(eig, ref["eigval"], rtol=0, atol=dn)
    signs = np.ones(3)
    da = np.zeros(3)
    for k in range(3):
        gap = min(abs(lam[k] - lam[j]) for j in range(len(lam)) if j != k)
        d_plus, d_minus = np.linalg.norm(axes[k] - ref["axes"][k]), np.linalg.norm(axes[k] + ref["axes"][k])
        signs[k] = 1.0 if d_plus <= d_minus else -1.0
        da[k] = min(d_plus, d_minus)
        assert da[k] <= 2 * dn / gap + 1e-9, (k, da[k], dn, gap)
        kmax = int(np.argmax(np.abs(axes[k])))
        assert axes[k, kmax] > 0                            # the sign rule
        assert abs(np.linalg.norm(axes[k]) - 1) < 1e-10
    # phi, per component, axis signs aligned
    phi = out["phi"].cpu().numpy()[0].astype(np.float64)
    assert not phi[..., 3].any()
    fm = np.linalg.norm(ref["sift"] - ref["mean"], axis=-1).max()
    for k in range(3):
        bound = da[k] * fm + 2 * np.sqrt(128) * delta + 200 * U32 * fm
        err = np.abs(signs[k] * phi[..., k] - ref["phi"][..., k]).max()
        assert err <= bound, (k, err, bound)
    dphi = np.abs(phi[..., :3] * signs - ref["phi"]).max()
    return out, ref, dphi


def test_sift_pca_chain_small_scene(sff):
    sc = make_scene(small_spec(48, 80, 3, seed=21))
    p = params_dict(48, 80, 3, levels=1, iters=1)
    _say("sift pca small scene")
    _chain(sff, sc.stack(), p)


def test_sift_pca_chain_batch_of_noise_pairs(sff):
    """Two pairs at once: the per-pair statistics are independent."""
    import torch
    rng = np.random.default_rng(8)
    H, W, C = 37, 51, 3
    imgs = np.stack([np.stack([smoothed_noise(rng, H, W, C, 1.2) for _ in range(4)]) for _ in range(2)])
    p = params_dict(H, W, C, levels=1, iters=1)
    _say("sift pca batch 2")
    out = sff.sff_sift_pca(p, dev(imgs))
    torch.cuda.synchronize()
    for b in range(2):
        ref = sp.sift_pca_features(imgs[b])
        one = sff.sff_sift_pca(p, dev(imgs[b][None]))
        torch.cuda.synchronize()
        for k in ("mean", "cov", "eigval", "axes", "phi"):
            assert torch.equal(out[k][b], one[k][0]), k       # same kernels, same order
        assert np.abs(out["cov"][b].cpu().numpy() - ref["cov"]).max() < 1e-4


def _cost_fp32_ref(phi32, hyp, s):
    return sp.cost(phi32.astype(np.float64)[..., :3], hyp, s)


def _sift_eval(monkeypatch, evaluator):
    """SFF_SIFT_EVAL=lane forces the per-lane SIFT cost and matching kernels; unset,
    the wave-shared ones run."""
    if evaluator == "lane":
        monkeypatch.setenv("SFF_SIFT_EVAL", "lane")
    else:
        monkeypatch.delenv("SFF_SIFT_EVAL", raising=False)


@pytest.mark.parametrize("evaluator", ["coop", "lane"])
@pytest.mark.parametrize("s", [1, -1])
def test_cost_kernel_on_oracle_features(sff, s, evaluator, monkeypatch):
    """The cost kernel alone: the oracle's phi rounded to FP32 feeds both sides;
    vectors random in range plus far out of the image."""
    import torch
    _sift_eval(monkeypatch, evaluator)
    sc = make_scene(small_spec(40, 64, 3, seed=5))
    imgs = sc.stack()
    ref = sp.sift_pca_features(imgs)
    phi32 = np.zeros((4, 40, 64, 4), np.float32)
    phi32[..., :3] = ref["phi"]
    rng = np.random.default_rng(6)
    hyp = np.stack([rng.integers(-20, 21, (40, 64)), rng.integers(-12, 13, (40, 64)),
                    rng.integers(0, 30, (40, 64)), rng.integers(0, 30, (40, 64))], axis=-1).astype(np.int16)
    hyp[::7, ::5, 0] = 300
    hyp[::9, ::4, 3] = -200
    p = params_dict(40, 64, 3, levels=1, iters=1)
    _say("cost kernel", s)
    c = sff.sff_cost_sift(p, dev(phi32[None]), dev(hyp[None]), s)
    torch.cuda.synchronize()
    want = _cost_fp32_ref(phi32, hyp, s)
    got = c.cpu().numpy()[0].astype(np.float64)
    assert np.all(np.abs(got - want) <= 150 * U32 * want + 1e-6)
    # the same FP32 operations in the same order as the oracle's matcher: equal bits
    assert np.array_equal(c.cpu().numpy()[0], oracle.cost_sift(phi32, hyp, s))
    # ground truth of the scene: lower cost than a shifted vector on average
    if s == 1:
        gt = sff.sff_cost_sift(p, dev(phi32[None]), dev(sc.gt_fwd[None]), 1).cpu().numpy()[0]
        shifted = sc.gt_fwd.copy()
        shifted[..., 0] += 3
        sh = sff.sff_cost_sift(p, dev(phi32[None]), dev(shifted[None]), 1).cpu().numpy()[0]
        assert gt.mean() < sh.mean()


def test_cost_chain_and_ragged_tiles(sff):
    """Features and cost from images on a size that is not a multiple of the
    16 x 16 tile, against the oracle chain within the propagated bound."""
    import torch
    sc = make_scene(small_spec(35, 50, 3, seed=9))
    imgs = sc.stack()
    p = params_dict(35, 50, 3, levels=1, iters=1)
    _say("cost chain 35x50")
    out, ref, dphi = _chain(sff, imgs, p)
    for s in (1, -1):
        hyp = sc.gt_fwd if s == 1 else sc.gt_inv
        c = sff.sff_cost_sift(p, out["phi"], dev(hyp[None]), s)
        torch.cuda.synchronize()
        want = sp.cost(ref["phi"], hyp, s)
        got = c.cpu().numpy()[0].astype(np.float64)
        bound = 147 * 2 * np.sqrt(3) * dphi + 150 * U32 * want + 1e-6
        assert np.all(np.abs(got - want) <= bound), s


def test_kitti_size_pair(sff):
    """The full KITTI-size pair in the launch configuration the bench times:
    every stage over all 1.86 M descriptors within its bound, and the cost at
    the ground-truth field on sampled pixels."""
    import torch
    sc = make_scene(kitti_spec())
    p = kitti_params()
    imgs = sc.stack()
    _say("sift pca kitti")
    out, ref, dphi = _chain(sff, imgs, p)
    cost = sff.sff_cost_sift(p, out["phi"], dev(sc.gt_fwd[None]), 1)
    torch.cuda.synchronize()
    rng = np.random.default_rng(12)
    ys, xs = rng.integers(0, p["H"], 3000), rng.integers(0, p["W"], 3000)
    want = np.array([_cost_at(ref["phi"], sc.gt_fwd, y, x) for y, x in zip(ys, xs)])
    got = cost.cpu().numpy()[0][ys, xs].astype(np.float64)
    assert np.all(np.abs(got - want) <= 147 * 2 * np.sqrt(3) * dphi + 150 * U32 * want + 1e-6)


def _cost_at(phi, hyp, y, x):
    """Eq. (1) at one pixel, forward direction, written out per window pixel."""
    _, H, W, _ = phi.shape
    u, v, d0, d1 = (int(c) for c in hyp[y, x])
    s = 0.0
    for wy in range(-3, 4):
        for wx in range(-3, 4):
            py, px = y + wy, x + wx
            r = phi[0, min(max(py, 0), H - 1), min(max(px, 0), W - 1)]
            for m, oy, ox in ((1, v, u), (2, 0, -d0), (3, v, u - d1)):
                t = phi[m, min(max(py + oy, 0), H - 1), min(max(px + ox, 0), W - 1)]
                s += float(np.sqrt(((r - t) ** 2).sum()))
    return s


def test_sift_sqrt_correctly_rounded(sff):
    """The cost's square root (sqrtf, on which the bit-exact SIFT-PCA cost and
    matching rely) against the host's IEEE float32 root, bit for bit: a stride
    through every non-negative finite float32 pattern (subnormals included),
    both sides of 2^-96 (where hipcc's sqrtf rescales its argument), the
    subnormal/normal edge, every float in [0.5, 0.5625) and the largest finite
    value."""
    import torch
    bits = np.arange(0, 0x7F800000, 997, dtype=np.uint32)
    edge = np.array([0, 1, 2, 3, 0x007FFFFF, 0x00800000, 0x00800001, 0x0F7FFFFF, 0x0F800000,
                     0x0F800001, 0x3F7FFFFF, 0x3F800000, 0x3F800001, 0x7F7FFFFF], np.uint32)
    dense = np.arange(0x3F000000, 0x3F000000 + (1 << 20), dtype=np.uint32)  # every float in [0.5, 0.5 + 2^-4)
    q = np.concatenate([bits, edge, dense]).view(np.float32)
    _say("sift sqrt", q.size)
    out = sff.sff_sift_sqrt(dev(q))
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    want = np.sqrt(q).view(np.uint32)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, [(hex(q.view(np.uint32)[i]), hex(got[i]), hex(want[i])) for i in bad[:8]]


# --------------------------------------------------------------------------
# Full-resolution matching with the SIFT-PCA cost: bit-exact against the
# oracle's FP32 matcher on the same features (the oracle's, rounded to FP32)
# and the same starting fields.

def _perturbed(rng, h, amount, fmax, dmax):
    out = h.astype(np.int32) + rng.integers(-amount, amount + 1, h.shape)
    out[..., :2] = np.clip(out[..., :2], -fmax, fmax)
    out[..., 2:] = np.clip(out[..., 2:], 0, dmax)
    return out.astype(np.int16)


MATCH_CASES = [  # H, W, iters, rs_samples, rs_r0, fmax, dmax, batch
    (40, 64, 3, 6, 8, 16, 16, 1), (23, 37, 2, 5, 4, 8, 12, 2), (1, 50, 2, 3, 4, 6, 6, 1),
    (50, 1, 2, 3, 4, 6, 6, 1), (33, 130, 2, 6, 16, 20, 16, 1),
]


@pytest.mark.parametrize("evaluator", ["coop", "lane"])
@pytest.mark.parametrize("case", MATCH_CASES, ids=[str(c) for c in MATCH_CASES])
def test_match_sift_parity(sff, case, evaluator, monkeypatch):
    import torch
    _sift_eval(monkeypatch, evaluator)
    H, W, iters, rs, r0, fmax, dmax, B = case
    rng = np.random.default_rng(H * 13 + W)
    phis, starts = [], []
    for b in range(B):
        sc = make_scene(small_spec(H, W, 3, seed=40 + b, flow_max=6, d_range=(0, 8)))
        phis.append(sp.sift_pca_features(sc.stack())["phi"])
        starts.append(np.stack([_perturbed(rng, sc.gt_fwd, 2, fmax, dmax),
                                _perturbed(rng, sc.gt_inv, 2, fmax, dmax)]))
    phi32 = np.zeros((B, 4, H, W, 4), np.float32)
    phi32[..., :3] = np.stack(phis)
    hyp0 = np.stack(starts, axis=1)                       # [2][B][H][W][4]
    seeds = np.array([17 + 5 * b for b in range(B)], np.int64)
    p = params_dict(H, W, 3, levels=1, iters=iters, rs_r0=r0, rs_samples=rs, fmax=fmax, dmax=dmax)
    _say("match sift", case, evaluator)
    hyp = dev(hyp0)
    cost = sff.sff_match_sift(p, dev(phi32), dev(seeds), hyp)
    torch.cuda.synchronize()
    hg, cg = hyp.cpu().numpy(), cost.cpu().numpy()
    for di, s in enumerate((1, -1)):
        for b in range(B):
            h, c = oracle.match_sift(phi32[b], hyp0[di, b], s, int(seeds[b]), iters, r0, rs, fmax, dmax)
            assert np.array_equal(hg[di, b], h), (case, s, b)
            assert np.array_equal(cg[di, b], c), (case, s, b)


@pytest.mark.parametrize("evaluator", ["coop", "lane"])
def test_match_sift_kitti_size(sff, evaluator, monkeypatch):
    """The KITTI-size pair: the oracle's features and its own WHT matching
    result as the start, two iterations, both fields, bit-exact."""
    import torch
    _sift_eval(monkeypatch, evaluator)
    sc = make_scene(kitti_spec())
    p = dict(kitti_params())
    p["iters"] = 2
    imgs = sc.stack()
    _say("match sift kitti: oracle features and start")
    phi32 = np.zeros((1, 4, p["H"], p["W"], 4), np.float32)
    phi32[0, ..., :3] = sp.sift_pca_features(imgs)["phi"]
    ref = oracle.match_pair(imgs, kitti_params(), 2)
    hyp0 = np.stack([ref["hyp"][0], ref["hyp"][1]])[:, None]
    hyp = dev(hyp0)
    _say("match sift kitti: gpu", evaluator)
    cost = sff.sff_match_sift(p, dev(phi32), dev(np.array([2], np.int64)), hyp)
    torch.cuda.synchronize()
    hg, cg = hyp.cpu().numpy(), cost.cpu().numpy()
    for di, s in enumerate((1, -1)):
        _say("match sift kitti: oracle", s)
        h, c = oracle.match_sift(phi32[0], hyp0[di, 0], s, 2, 2, p["rs_r0"], p["rs_samples"], p["fmax"],
                                 p["dmax"])
        assert np.array_equal(hg[di, 0], h), s
        assert np.array_equal(cg[di, 0], c), s


def test_pipeline_refine_sift(sff):
    """PairMatcher.refine_sift after a run: every pixel's cost is at most the
    SIFT-PCA cost of its starting vector, and the stored cost is the cost of
    the final field (same arithmetic as sff_cost_sift)."""
    import torch
    from sff_inputs import tiny_params, tiny_spec
    sc = make_scene(tiny_spec())
    p = tiny_params()
    imgs = dev(sc.stack()[None])
    seeds = dev(np.array([1], np.int64))
    _say("pipeline refine sift")
    m = sff.PairMatcher(p, 1)
    m.run(imgs, seeds)
    start = m.hyp[0].clone()
    feats = sff.sff_sift_pca(p, imgs)
    c0 = [sff.sff_cost_sift(p, feats["phi"], start[d], d_) for d, d_ in ((0, 1), (1, -1))]
    out = m.refine_sift(imgs, seeds)
    torch.cuda.synchronize()
    for d, d_ in ((0, 1), (1, -1)):
        c = out["cost"][d]
        assert torch.all(c <= c0[d])
        assert torch.equal(c, sff.sff_cost_sift(p, feats["phi"], out["hyp"][d], d_))
    assert out["valid"].sum().item() > 0
