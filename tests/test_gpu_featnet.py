"""GPU checks of the learned-descriptor helpers: level smoothing (bit-exact
against the oracle), quantisation of normalised features, and the triplet
loss with its gradient (FP32 against FP64 autograd on the same BF16 inputs)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import featnet as ofn
from sff_inputs import make_scene, small_spec, params_dict

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sff():
    import paper_1710_10096_amd as m
    assert torch.cuda.is_available()
    return m


def test_smooth_level_matches_oracle(sff):
    sc = make_scene(small_spec(45, 71, 3, 9))
    imgs = sc.stack()
    p = params_dict(45, 71, 3, levels=3, iters=1)
    for lv in range(3):
        _say("smooth level", lv)
        out = sff.sff_smooth_level(p, torch.from_numpy(imgs).cuda(), lv).cpu().numpy()
        for m in range(4):
            assert np.array_equal(out[m], oracle.smooth(imgs[m], 1 << lv))


def test_quantise_features(sff):
    rng = np.random.default_rng(1)
    f = ofn.bf16_round(rng.standard_normal((2, 7, 9, 32)) * rng.uniform(0.01, 10, (2, 7, 9, 1)))
    t = torch.from_numpy(f.astype(np.float32)).to(torch.bfloat16).cuda()
    d = sff.sff_quantise_features(t, 4096.0).cpu().numpy().reshape(2, 7, 9, 32).astype(np.int64)
    ref = np.rint(4096.0 * ofn.l2_normalise(f))
    assert np.abs(d - ref).max() <= 1
    assert (np.abs(d - ref) > 0).mean() < 0.01


def test_triplet_loss_and_gradient(sff):
    rng = np.random.default_rng(2)
    npx, T = 500, 3000
    f = ofn.bf16_round(rng.standard_normal((npx, 32)))
    trip = rng.integers(0, npx, (T, 3)).astype(np.int32)
    trip[:5, 1] = trip[:5, 0]                    # positive equal to anchor
    trip[5, 2] = npx + 3                          # invalid index: ignored
    margin = 0.5
    ft = torch.from_numpy(f.astype(np.float32)).to(torch.bfloat16).cuda()
    grad = torch.zeros((npx, 32), dtype=torch.float32, device="cuda")
    _say("triplet loss")
    loss = sff.sff_triplet_loss(ft, torch.from_numpy(trip).cuda(), margin, grad, weight=0.25)
    loss = loss.cpu().numpy()
    valid = (trip < npx).all(axis=1)
    fn = ofn.l2_normalise(f)
    ref = np.zeros(T)
    ref[valid] = ofn.triplet_loss(fn[trip[valid, 0]], fn[trip[valid, 1]], fn[trip[valid, 2]], margin)
    assert np.allclose(loss, ref, rtol=1e-5, atol=1e-6)
    # FP64 autograd of 0.25 * sum(loss) through the normalisation
    x = torch.from_numpy(f).requires_grad_(True)
    xn = x / x.norm(dim=1, keepdim=True)
    tv = torch.from_numpy(trip[valid].astype(np.int64))
    a, p, n = xn[tv[:, 0]], xn[tv[:, 1]], xn[tv[:, 2]]
    l = torch.clamp(margin + ((a - p) ** 2).sum(1) - ((a - n) ** 2).sum(1), min=0)
    (0.25 * l.sum()).backward()
    g = grad.cpu().numpy()
    gr = x.grad.numpy()
    assert np.allclose(g, gr, rtol=1e-4, atol=1e-5 * np.abs(gr).max())
    out = sff.sff_take_grad_bf16(grad)
    assert float(grad.abs().max()) == 0.0
    assert np.array_equal(out.to(torch.float32).cpu().numpy(), ofn.bf16_round(g).astype(np.float32))
