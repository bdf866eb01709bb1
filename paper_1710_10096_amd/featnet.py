"""Learned descriptors for the matching cost, trained on the plain method's
consistent matches.

The WHT features of Section 3.1 are replaced by a 4-layer 3x3 convolutional
network (3 -> 32 -> 32 -> 32 -> 32, ReLU after the first three) whose 32
output channels, L2-normalised per pixel and rounded to int16, form a C = 2
descriptor map for the unchanged exact integer matcher (init, propagation,
random search, consistency).  At pyramid level k the network runs with
dilation n = 2^k on the level's smoothed image, so its receptive field (8n + 1
pixels) spans the stride-n 8x8 patch the WHT path samples.

All convolutions, their gradients, the loss and the descriptor quantisation
are libsff kernels; torch supplies device memory, random sampling of triples
and the Adam update of the FP32 master weights.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import api
from ._native import SffParams
from .pipeline import PairMatcher

CH = 32
LAYERS = ((3, CH), (CH, CH), (CH, CH), (CH, CH))


class FeatNet:
    def __init__(self, seed: int = 0, device="cuda", lr: float = 1e-3):
        g = torch.Generator(device="cpu").manual_seed(seed)
        self.params = []
        for cin, cout in LAYERS:
            w = torch.randn((cout, 3, 3, cin), generator=g) * math.sqrt(2.0 / (9 * cin))
            b = torch.zeros(cout)
            self.params += [w.to(device), b.to(device)]
        for t in self.params:
            t.requires_grad_(False)
        self.opt = torch.optim.Adam(self.params, lr=lr)
        self.device = torch.device(device)

    def weights_bf16(self):
        return [self.params[2 * l].to(torch.bfloat16).contiguous() for l in range(4)]

    def forward(self, x: torch.Tensor, dil: int = 1, keep: bool = False, wb=None):
        """x bf16 [n][H][W][3] -> bf16 [n][H][W][32] (and the activations).
        Without `keep`, at dilation 1, the four layers run as one launch with the
        activations on chip (same bits as the per-layer calls)."""
        wb = wb if wb is not None else self.weights_bf16()
        if not keep and dil == 1:
            return api.sff_featnet_fwd_bf16(x, wb, [self.params[2 * l + 1] for l in range(4)])
        acts = [x]
        h = x
        for l in range(4):
            h = api.sff_conv3x3_bf16_fwd(h, wb[l], self.params[2 * l + 1], dil, relu=l < 3)
            acts.append(h)
        return (h, acts) if keep else h

    def backward(self, acts, dout: torch.Tensor, dil: int = 1, wb=None):
        """Gradients (dw, db) of every layer given dL/d(output) in bf16."""
        wb = wb if wb is not None else self.weights_bf16()
        grads = [None] * 8
        g = dout
        for l in range(3, -1, -1):
            relu_out = acts[l + 1] if l < 3 else None
            dw, db = api.sff_conv3x3_bf16_wgrad(acts[l], g, dil, relu_out)
            grads[2 * l], grads[2 * l + 1] = dw, db
            if l > 0:
                g = api.sff_conv3x3_bf16_dgrad(g, wb[l], dil, relu_out)
        return grads

    def step(self, grads):
        for t, gr in zip(self.params, grads):
            t.grad = gr
        self.opt.step()
        self.opt.zero_grad(set_to_none=True)

    def state(self):
        return [t.detach().cpu().clone() for t in self.params]


def images_bf16(imgs_u8: torch.Tensor) -> torch.Tensor:
    """uint8 [n][H][W][3] -> bf16 in [0, 1]."""
    return (imgs_u8.to(torch.float32) / 255.0).to(torch.bfloat16).contiguous()


class TripletPool:
    """Positive correspondences of one training pair: consistent forward
    matches of the WHT matcher give, for an anchor pixel in I_l^0, its
    temporal (I_l^1), stereo (I_r^0) and cross (I_r^1) partners."""

    def __init__(self, hyp_fwd: np.ndarray, valid: np.ndarray):
        H, W = valid.shape
        ys, xs = np.nonzero(valid)
        u, v, d0, d1 = (hyp_fwd[ys, xs, k].astype(np.int64) for k in range(4))
        self.H, self.W = H, W
        self.anchor = ys * W + xs
        self.pos = np.stack([(ys + v) * W + (xs + u),            # view 1 (l1)
                             ys * W + (xs - d0),                  # view 2 (r0)
                             (ys + v) * W + (xs + u - d1)], 1)    # view 3 (r1)
        self.pos_xy = np.stack([np.stack([xs + u, ys + v], 1), np.stack([xs - d0, ys], 1),
                                np.stack([xs + u - d1, ys + v], 1)], 1)

    def sample(self, rng: np.random.Generator, T: int) -> np.ndarray:
        """T triples of pixel indices into the stacked maps [4][H][W]."""
        HW = self.H * self.W
        i = rng.integers(0, len(self.anchor), T)
        view = rng.integers(0, 3, T)
        pxy = self.pos_xy[i, view]
        # negative: the positive shifted by 3..16 px in a random direction, inside the image
        r = rng.integers(3, 17, T)
        ang = rng.uniform(0, 2 * np.pi, T)
        nx = np.clip(pxy[:, 0] + np.rint(r * np.cos(ang)).astype(np.int64), 0, self.W - 1)
        ny = np.clip(pxy[:, 1] + np.rint(r * np.sin(ang)).astype(np.int64), 0, self.H - 1)
        a = self.anchor[i]
        p = (view + 1) * HW + self.pos[i, view]
        n = (view + 1) * HW + ny * self.W + nx
        return np.stack([a, p, n], 1).astype(np.int32)


def train(net: FeatNet, scenes, params: dict, seeds, steps: int = 2000, triples: int = 4096,
          margin: float = 0.5, seed: int = 0, log=None):
    """Train on consistent WHT matches of the given pairs (cycled), returns the
    mean loss of the last 100 steps."""
    dev = net.device
    p = params
    pools, inputs = [], []
    for sc, sd in zip(scenes, seeds):
        m = PairMatcher(p, 1, dev)
        out = m.run(torch.from_numpy(sc.stack()[None]).to(dev),
                    torch.tensor([sd], dtype=torch.int64, device=dev))
        pools.append(TripletPool(out["hyp"][0, 0].cpu().numpy(), out["valid"][0].cpu().numpy() > 0))
        inputs.append(images_bf16(torch.from_numpy(sc.stack()).to(dev)))
        del m
    rng = np.random.default_rng(seed)
    H, W = p["H"], p["W"]
    grad = torch.zeros((4 * H * W, CH), dtype=torch.float32, device=dev)
    hist = []
    for it in range(steps):
        k = it % len(pools)
        wb = net.weights_bf16()
        out, acts = net.forward(inputs[k], 1, keep=True, wb=wb)
        trip = torch.from_numpy(pools[k].sample(rng, triples)).to(dev)
        loss = api.sff_triplet_loss(out, trip, margin, grad, weight=1.0 / triples)
        dout = api.sff_take_grad_bf16(grad).view(4, H, W, CH)
        net.step(net.backward(acts, dout, 1, wb=wb))
        hist.append(loss.mean())
        if log is not None and (it % 200 == 0 or it == steps - 1):
            log(f"step {it} loss {float(torch.stack(hist[-50:]).mean()):.4f}")
    return float(torch.stack(hist[-100:]).mean())


class LearnedMatcher:
    """The matching stage with learned descriptors: per level, the smoothed
    views go through the network (dilation 2^k), are normalised and quantised
    to int16, and feed sff_init_nn / sff_match_level (C = 2); then the
    consistency check."""

    SCALE = 4096.0

    def __init__(self, net: FeatNet, params: dict, batch: int = 1):
        self.net = net
        pc = dict(params)
        pc["C"] = 2
        self.pimg = SffParams.from_dict(params)
        self.inner = PairMatcher(pc, batch, net.device, maps="desc")
        self.batch = batch
        ws = max(api.sff_wht_workspace_bytes(self.pimg, 4 * batch, k) for k in range(self.pimg.levels))
        self.ws_img = torch.empty(max(ws, 256), dtype=torch.uint8, device=net.device)
        self.smoothed = torch.empty((4 * batch, self.pimg.H, self.pimg.W, self.pimg.C),
                                    dtype=torch.uint8, device=net.device)

    def run(self, imgs: torch.Tensor, seeds: torch.Tensor) -> dict:
        p, m, B = self.pimg, self.inner, self.batch
        flat = imgs.view(4 * B, p.H, p.W, p.C)
        desc = m.desc.view(4 * B, p.H, p.W, 2, 16)
        wb = self.net.weights_bf16()
        top = p.levels - 1
        for k in range(top, -1, -1):
            sm = api.sff_smooth_level(p, flat, k, self.smoothed, self.ws_img)
            feat = self.net.forward(images_bf16(sm), 1 << k, wb=wb)
            api.sff_quantise_features(feat, self.SCALE, desc)
            if k == top:
                api.sff_init_nn(m.p, m.desc, api.DIR_BOTH, m.hyp[k], m.cost[k], m.ws)
                api.sff_match_level(m.p, m.desc, api.DIR_BOTH, k, seeds, m.hyp[k], m.cost[k])
            else:
                api.sff_match_level(m.p, m.desc, api.DIR_BOTH, k, seeds, m.hyp[k], m.cost[k],
                                    m.hyp[k + 1])
        api.sff_consistency(m.p, m.hyp[0][0], m.hyp[0][1], m.valid, m.err)
        return dict(hyp=m.hyp[0], cost=m.cost[0], valid=m.valid, err=m.err)


def match_quality(hyp_fwd: np.ndarray, valid: np.ndarray, gt: np.ndarray, gt_ok: np.ndarray):
    """Consistent-match fraction and endpoint errors of consistent matches
    where the ground truth is defined: flow EPE |(u, v) - gt| and mean
    absolute disparity errors."""
    v = valid.astype(bool)
    sel = v & gt_ok
    d = hyp_fwd.astype(np.float64) - gt.astype(np.float64)
    epe = np.sqrt(d[..., 0] ** 2 + d[..., 1] ** 2)
    return dict(consistent_frac=float(v.mean()),
                flow_epe=float(epe[sel].mean()) if sel.any() else float("nan"),
                d0_err=float(np.abs(d[..., 2])[sel].mean()) if sel.any() else float("nan"),
                d1_err=float(np.abs(d[..., 3])[sel].mean()) if sel.any() else float("nan"),
                outliers_3px=float((epe[sel] > 3).mean()) if sel.any() else float("nan"))
