"""FP64 oracle of the learned-feature extractor -- TEST INFRASTRUCTURE.

The learned path replaces the WHT descriptors (Section 3.1, "Initialization",
features for the matching cost) with the output of a small convolutional
network: four 3x3 convolutions 3 -> 32 -> 32 -> 32 -> 32, ReLU after the first
three, each with zero padding and dilation d (d = n = 2^k at pyramid level k,
so the receptive field grows with the level as the stride-n WHT patch does).
Tensors are NHWC; weights [Cout][3][3][Cin] (tap (ky, kx) at offset
((ky - 1) d, (kx - 1) d)).

Everything here is float64 and written from the definitions:
  y[p, o] = b[o] + sum_{ky, kx, i} w[o, ky, kx, i] x[p + ((ky-1)d, (kx-1)d), i]
(x = 0 outside the image); the input gradient is the sum of w times the output
gradient over every output pixel that read the input pixel; the weight
gradient is the sum over pixels of output gradient times input.

Descriptors are the per-pixel L2-normalised network outputs; the triplet loss
of a (anchor, positive, negative) triple of descriptors is
max(0, margin + |a - p|^2 - |a - n|^2).
"""
from __future__ import annotations

import numpy as np


def bf16_round(a):
    """Round float arrays to the nearest bfloat16 (ties to even), as float64."""
    x = np.asarray(a, np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _shifted(x, dy, dx):
    """x[p + (dy, dx)] with zeros outside; x: [N][H][W][C]."""
    N, H, W, C = x.shape
    out = np.zeros_like(x)
    ys0, ys1 = max(0, -dy), min(H, H - dy)
    xs0, xs1 = max(0, -dx), min(W, W - dx)
    if ys0 < ys1 and xs0 < xs1:
        out[:, ys0:ys1, xs0:xs1] = x[:, ys0 + dy:ys1 + dy, xs0 + dx:xs1 + dx]
    return out


def conv3x3(x, w, b, dil=1, relu=False):
    """y = conv(x, w) + b (then ReLU); float64."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    y = np.zeros(x.shape[:3] + (w.shape[0],), np.float64) + np.asarray(b, np.float64)
    for ky in range(3):
        for kx in range(3):
            xs = _shifted(x, (ky - 1) * dil, (kx - 1) * dil)
            y += np.einsum("nhwi,oi->nhwo", xs, w[:, ky, kx, :])
    return np.maximum(y, 0) if relu else y


def conv3x3_dgrad(dy, w, dil=1):
    """dL/dx given dL/dy (pre-activation): each output pixel p read input pixel
    p + (ky-1, kx-1) d with weight w[:, ky, kx, :]."""
    dy = np.asarray(dy, np.float64)
    w = np.asarray(w, np.float64)
    dx = np.zeros(dy.shape[:3] + (w.shape[3],), np.float64)
    for ky in range(3):
        for kx in range(3):
            contrib = np.einsum("nhwo,oi->nhwi", dy, w[:, ky, kx, :])
            dx += _shifted(contrib, -(ky - 1) * dil, -(kx - 1) * dil)
    return dx


def conv3x3_wgrad(x, dy, dil=1):
    """dL/dw [Cout][3][3][Cin] and dL/db [Cout] given dL/dy (pre-activation)."""
    x = np.asarray(x, np.float64)
    dy = np.asarray(dy, np.float64)
    dw = np.zeros((dy.shape[3], 3, 3, x.shape[3]), np.float64)
    for ky in range(3):
        for kx in range(3):
            xs = _shifted(x, (ky - 1) * dil, (kx - 1) * dil)
            dw[:, ky, kx, :] = np.einsum("nhwo,nhwi->oi", dy, xs)
    return dw, dy.sum(axis=(0, 1, 2))


def l2_normalise(f, eps=1e-12):
    n = np.sqrt((np.asarray(f, np.float64) ** 2).sum(axis=-1, keepdims=True))
    return f / np.maximum(n, eps)


def triplet_loss(a, p, n, margin):
    """Per-triple hinge loss on descriptors a, p, n [T][C] (already normalised)."""
    dp = ((a - p) ** 2).sum(axis=-1)
    dn = ((a - n) ** 2).sum(axis=-1)
    return np.maximum(0.0, margin + dp - dn)
