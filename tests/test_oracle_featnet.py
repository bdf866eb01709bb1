"""Pins of the FP64 learned-feature oracle: convolution against torch's
float64 conv2d (an independent library implementation) and its gradients
against autograd and finite differences; bfloat16 rounding against torch."""
import numpy as np
import pytest
import torch

from oracle import featnet as ofn


def _torch_conv(x, w, b, dil):
    xt = torch.from_numpy(x).permute(0, 3, 1, 2)
    wt = torch.from_numpy(w).permute(0, 3, 1, 2)
    y = torch.nn.functional.conv2d(xt, wt, torch.from_numpy(b), padding=dil, dilation=dil)
    return y.permute(0, 2, 3, 1).numpy()


@pytest.mark.parametrize("dil", [1, 2, 4])
@pytest.mark.parametrize("cin,cout", [(3, 32), (32, 32), (5, 7)])
def test_conv_matches_torch_float64(dil, cin, cout):
    rng = np.random.default_rng(dil * 100 + cin)
    x = rng.standard_normal((2, 11, 13, cin))
    w = rng.standard_normal((cout, 3, 3, cin))
    b = rng.standard_normal(cout)
    y = ofn.conv3x3(x, w, b, dil)
    assert np.allclose(y, _torch_conv(x, w, b, dil), rtol=1e-12, atol=1e-12)
    assert np.array_equal(ofn.conv3x3(x, w, b, dil, relu=True), np.maximum(y, 0))


@pytest.mark.parametrize("dil", [1, 3])
def test_conv_gradients_match_autograd(dil):
    rng = np.random.default_rng(7 + dil)
    x = rng.standard_normal((1, 9, 10, 4))
    w = rng.standard_normal((6, 3, 3, 4))
    b = rng.standard_normal(6)
    gy = rng.standard_normal((1, 9, 10, 6))
    xt = torch.from_numpy(x).permute(0, 3, 1, 2).requires_grad_(True)
    wt = torch.from_numpy(w).permute(0, 3, 1, 2).detach().requires_grad_(True)
    bt = torch.from_numpy(b).requires_grad_(True)
    yt = torch.nn.functional.conv2d(xt, wt, bt, padding=dil, dilation=dil)
    (yt * torch.from_numpy(gy).permute(0, 3, 1, 2)).sum().backward()
    dx = ofn.conv3x3_dgrad(gy, w, dil)
    dw, db = ofn.conv3x3_wgrad(x, gy, dil)
    assert np.allclose(dx, xt.grad.permute(0, 2, 3, 1).numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(dw, wt.grad.permute(0, 2, 3, 1).numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(db, bt.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_conv_gradient_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 6, 7, 2))
    w = rng.standard_normal((3, 3, 3, 2))
    b = rng.standard_normal(3)
    gy = rng.standard_normal((1, 6, 7, 3))
    L = lambda xx, ww: (ofn.conv3x3(xx, ww, b, 2) * gy).sum()
    dx = ofn.conv3x3_dgrad(gy, w, 2)
    dw, _ = ofn.conv3x3_wgrad(x, gy, 2)
    e = 1e-6
    for idx in [(0, 0, 0, 0), (0, 5, 6, 1), (0, 2, 3, 0)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += e
        xm[idx] -= e
        assert abs((L(xp, w) - L(xm, w)) / (2 * e) - dx[idx]) < 1e-6
    for idx in [(0, 0, 0, 0), (2, 2, 2, 1), (1, 1, 0, 1)]:
        wp, wm = w.copy(), w.copy()
        wp[idx] += e
        wm[idx] -= e
        assert abs((L(x, wp) - L(x, wm)) / (2 * e) - dw[idx]) < 1e-6


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(5)
    a = np.concatenate([rng.standard_normal(10000) * 10 ** rng.uniform(-3, 3, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0]]).astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ofn.bf16_round(a), ref)


def test_triplet_loss_closed_forms():
    a = np.array([[1.0, 0.0]])
    p = np.array([[1.0, 0.0]])
    n = np.array([[0.0, 1.0]])
    assert ofn.triplet_loss(a, p, n, 0.5)[0] == 0.0       # |a-p|^2 = 0, |a-n|^2 = 2
    assert ofn.triplet_loss(a, n, p, 0.5)[0] == 2.5       # swapped: 0.5 + 2 - 0
    f = np.array([[3.0, 4.0]])
    assert np.allclose(ofn.l2_normalise(f), [[0.6, 0.8]])
