"""GPU checks of the BF16 MFMA 3x3 convolutions against the FP64 oracle on the
same BF16-rounded inputs.

Tolerances: outputs and input gradients are FP32 sums of at most 288 products
rounded once to BF16.  The FP32 sum is within 288 2^-24 (< 2e-5) of the sum of
the terms' magnitudes S from the exact value, and rounding to BF16 adds at most
one unit in the last place (at most 2^-7 |y|), so the test allows
2^-7 |y| + 2e-5 S.  Weight gradients are FP32 sums over every pixel in per-block
partials; the bound is ~(1024 + number of blocks) 2^-24 times the sum of the
terms' magnitudes; the test allows 2e-4 of that sum.
"""
import sys

import numpy as np
import pytest

from oracle import featnet as ofn

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sff():
    import torch
    import paper_1710_10096_amd as m
    assert torch.cuda.is_available()
    return m


def _bf(a):
    import torch
    return torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).cuda()


def _np(t):
    import torch
    return t.to(torch.float32).cpu().numpy().astype(np.float64)


def _within_bf16_ulp(got, ref, abs_sum):
    # one BF16 unit in the last place: 2^-7 of the binade [2^e, 2^(e+1)) of the value
    big = np.maximum(np.abs(got), np.abs(ref))
    return np.abs(got - ref) <= big * 2.0 ** -7 + 2e-5 * abs_sum + 1e-30


CASES = [(1, 9, 70, 3, 1), (2, 17, 131, 32, 1), (1, 23, 64, 32, 2), (1, 30, 97, 32, 4),
         (1, 5, 6, 32, 16), (1, 1, 1, 3, 1),
         # several 256-pixel tiles of the 32-channel kernel with ragged tails
         (1, 7, 300, 32, 1), (2, 6, 530, 32, 3), (1, 40, 270, 32, 16)]


@pytest.mark.parametrize("case", CASES, ids=[str(c) for c in CASES])
def test_conv_forward_and_gradients(sff, case):
    import torch
    n, H, W, cin, dil = case
    rng = np.random.default_rng(H * 1000 + W + cin + dil)
    x = ofn.bf16_round(rng.standard_normal((n, H, W, cin)))
    w = ofn.bf16_round(rng.standard_normal((32, 3, 3, cin)) / np.sqrt(9 * cin))
    b = rng.standard_normal(32).astype(np.float32).astype(np.float64)
    _say("conv", case)
    for relu in (False, True):
        y = sff.sff_conv3x3_bf16_fwd(_bf(x), _bf(w), torch.from_numpy(b.astype(np.float32)).cuda(),
                                     dil, relu)
        ref = ofn.bf16_round(ofn.conv3x3(x, w, b, dil, relu))
        S = ofn.conv3x3(np.abs(x), np.abs(w), np.abs(b), dil)
        assert _within_bf16_ulp(_np(y), ref, S).all(), relu
    # gradients with a ReLU mask from a layer output
    relu_out = ofn.bf16_round(np.maximum(rng.standard_normal((n, H, W, 32)), 0))
    dy = ofn.bf16_round(rng.standard_normal((n, H, W, 32)))
    dz = dy * (relu_out > 0)
    dw, db = sff.sff_conv3x3_bf16_wgrad(_bf(x), _bf(dy), dil, _bf(relu_out))
    rdw, rdb = ofn.conv3x3_wgrad(x, dz, dil)
    adw, adb = ofn.conv3x3_wgrad(np.abs(x), np.abs(dz), dil)
    assert (np.abs(dw.cpu().numpy() - rdw) <= 2e-4 * adw + 1e-6).all()
    assert (np.abs(db.cpu().numpy() - rdb) <= 2e-4 * adb + 1e-6).all()
    if cin == 32:
        dx = sff.sff_conv3x3_bf16_dgrad(_bf(dy), _bf(w), dil, _bf(relu_out))
        rdx = ofn.bf16_round(ofn.conv3x3_dgrad(dz, w, dil))
        S = ofn.conv3x3_dgrad(np.abs(dz), np.abs(w), dil)
        assert _within_bf16_ulp(_np(dx), rdx, S).all()
        dx2 = sff.sff_conv3x3_bf16_dgrad(_bf(dz), _bf(w), dil, None)
        assert np.array_equal(_np(dx2), _np(dx))
    dw2, _ = sff.sff_conv3x3_bf16_wgrad(_bf(x), _bf(dy), dil, _bf(relu_out))
    assert np.array_equal(dw2.cpu().numpy(), dw.cpu().numpy())  # deterministic


CASES32 = [(2, 17, 131, 32, 1), (1, 7, 300, 32, 1), (2, 6, 530, 32, 3), (1, 40, 270, 32, 16)]


@pytest.mark.parametrize("case", CASES32, ids=[str(c) for c in CASES32])
def test_conv32_kernel_same_as_im2col(sff, case, monkeypatch):
    """The 32-channel kernels with 16-byte staging (the default for 16-byte
    aligned tensors: forward and input gradient without an im2col tile, weight
    gradient with vector-loaded transposed tiles) against the element-wise
    kernels (SFF_CONV_IM2COL=1) and against the same tensors at a 2-byte offset
    (which take the element-wise kernels): the same MFMAs on the same values,
    so forward, input and weight gradients agree bit for bit."""
    import torch
    n, H, W, cin, dil = case
    rng = np.random.default_rng(7 * H + W + dil)
    x = ofn.bf16_round(rng.standard_normal((n, H, W, 32)))
    w = ofn.bf16_round(rng.standard_normal((32, 3, 3, 32)) / np.sqrt(288))
    b = torch.from_numpy(rng.standard_normal(32).astype(np.float32)).cuda()
    relu_out = ofn.bf16_round(np.maximum(rng.standard_normal((n, H, W, 32)), 0))
    dy = ofn.bf16_round(rng.standard_normal((n, H, W, 32)))

    def offset(a):  # the same values at a 2-byte offset (contiguous, not 16-byte aligned)
        t = _bf(a).reshape(-1)
        buf = torch.empty(t.numel() + 8, dtype=torch.bfloat16, device="cuda")
        v = buf[1:1 + t.numel()]
        v.copy_(t)
        return v.view(a.shape)

    _say("conv32 vs im2col", case)
    monkeypatch.delenv("SFF_CONV_IM2COL", raising=False)
    y = sff.sff_conv3x3_bf16_fwd(_bf(x), _bf(w), b, dil, True)
    dx = sff.sff_conv3x3_bf16_dgrad(_bf(dy), _bf(w), dil, _bf(relu_out))
    y_off = sff.sff_conv3x3_bf16_fwd(offset(x), _bf(w), b, dil, True)
    dx_off = sff.sff_conv3x3_bf16_dgrad(offset(dy), _bf(w), dil, offset(relu_out))
    dw, db = sff.sff_conv3x3_bf16_wgrad(_bf(x), _bf(dy), dil, _bf(relu_out))
    dw_off, db_off = sff.sff_conv3x3_bf16_wgrad(offset(x), offset(dy), dil, offset(relu_out))
    monkeypatch.setenv("SFF_CONV_IM2COL", "1")
    y_ref = sff.sff_conv3x3_bf16_fwd(_bf(x), _bf(w), b, dil, True)
    dx_ref = sff.sff_conv3x3_bf16_dgrad(_bf(dy), _bf(w), dil, _bf(relu_out))
    dw_ref, db_ref = sff.sff_conv3x3_bf16_wgrad(_bf(x), _bf(dy), dil, _bf(relu_out))
    torch.cuda.synchronize()
    for got in (y, y_off):
        assert torch.equal(got.view(torch.int16), y_ref.view(torch.int16))
    for got in (dx, dx_off):
        assert torch.equal(got.view(torch.int16), dx_ref.view(torch.int16))
    for got, ref in ((dw, dw_ref), (dw_off, dw_ref), (db, db_ref), (db_off, db_ref)):
        assert torch.equal(got, ref)


@pytest.mark.parametrize("case", [(2, 9, 70, 1), (1, 7, 300, 1), (1, 12, 530, 4), (1, 40, 270, 16), (1, 1, 1, 1)],
                         ids=str)
def test_first_layer_kernel_same_as_im2col(sff, case, monkeypatch):
    """The 3-channel first layer read from staged input rows (the default)
    against the im2col kernel (SFF_CONV_IM2COL=1): the same MFMA operands, so
    the same bits; and against the FP64 oracle."""
    import torch
    n, H, W, dil = case
    rng = np.random.default_rng(H + 3 * W + dil)
    x = ofn.bf16_round(rng.standard_normal((n, H, W, 3)))
    w = ofn.bf16_round(rng.standard_normal((32, 3, 3, 3)) / np.sqrt(27))
    b = rng.standard_normal(32).astype(np.float32)
    bt = torch.from_numpy(b).cuda()
    _say("first layer vs im2col", case)
    monkeypatch.delenv("SFF_CONV_IM2COL", raising=False)
    y = sff.sff_conv3x3_bf16_fwd(_bf(x), _bf(w), bt, dil, True)
    monkeypatch.setenv("SFF_CONV_IM2COL", "1")
    y_ref = sff.sff_conv3x3_bf16_fwd(_bf(x), _bf(w), bt, dil, True)
    torch.cuda.synchronize()
    assert torch.equal(y.view(torch.int16), y_ref.view(torch.int16))
    ref = ofn.bf16_round(ofn.conv3x3(x, w, b.astype(np.float64), dil, True))
    S = ofn.conv3x3(np.abs(x), np.abs(w), np.abs(b.astype(np.float64)), dil)
    assert _within_bf16_ulp(_np(y), ref, S).all()


FUSED_CASES = [(1, 1, 1), (2, 9, 70), (1, 8, 64), (1, 17, 131), (3, 23, 200), (1, 40, 270),
               # exact tiles of 24 x 26 outputs, one pixel past them, several of each
               (1, 24, 26), (2, 25, 27), (1, 49, 79), (1, 72, 52)]


@pytest.mark.parametrize("case", FUSED_CASES, ids=[str(c) for c in FUSED_CASES])
def test_fused_network_forward_same_as_layers(sff, case):
    """The four layers in one launch (activations on chip, tiles of 24 x 26
    outputs, ragged edges) against the four per-layer calls, bit for bit;
    the last layer against the FP64 oracle on the per-layer path's layer-3
    output."""
    import torch
    n, H, W = case
    rng = np.random.default_rng(H * 7 + W + n)
    x = ofn.bf16_round(rng.standard_normal((n, H, W, 3)) * 2.0)
    ws, bs = [], []
    for cin in (3, 32, 32, 32):
        ws.append(ofn.bf16_round(rng.standard_normal((32, 3, 3, cin)) / np.sqrt(9 * cin)))
        bs.append(rng.standard_normal(32).astype(np.float32).astype(np.float64) * 0.1)
    wt = [_bf(w) for w in ws]
    bt = [torch.from_numpy(b.astype(np.float32)).cuda() for b in bs]
    _say("fused network", case)
    y = sff.sff_featnet_fwd_bf16(_bf(x), wt, bt)
    h = _bf(x)
    acts = []
    for l in range(4):
        h = sff.sff_conv3x3_bf16_fwd(h, wt[l], bt[l], 1, l < 3)
        acts.append(h)
    assert np.array_equal(_np(y), _np(h))
    x3 = _np(acts[2])
    ref = ofn.bf16_round(ofn.conv3x3(x3, ws[3], bs[3], 1, False))
    S = ofn.conv3x3(np.abs(x3), np.abs(ws[3]), np.abs(bs[3]), 1)
    assert _within_bf16_ulp(_np(y), ref, S).all()
