"""Seeded synthetic stereo-pair scenes (input generator only).

This module produces the four images of two rectified stereo pairs
(I_l^0, I_l^1, I_r^0, I_r^1) together with the integer ground-truth scene flow
(u, v, d0, d1) of the left reference view and of the right view at t1.  It holds
none of the matching method's arithmetic: no descriptors, costs, search or
checks live here.  Both the CPU oracle and the GPU path read its output.

Scene model (problem statement of Section 3: two rectified stereo pairs at t0
and t1, scene flow u = (u, v, d0, d1) per reference pixel):

* texture: uniform noise, Gaussian-smoothed per channel, min-max stretched to
  0..255 and rounded;
* geometry: Voronoi segments of random sites, each with an integer-rounded
  planar disparity d0 = a + b x + c y, an integer translation (u, v) and a
  disparity change d1 = d0 + delta; optionally one compact foreground
  occluder with the largest disparity and its own motion;
* rendering: forward splatting of I_l^0 pixels to I_l^1 at p + (u, v), to
  I_r^0 at p - (d0, 0) and to I_r^1 at p + (u - d1, v), with a z-buffer in
  which the larger disparity (nearer surface) wins, ties to the smaller source
  index; holes filled with fresh smoothed noise;
* optional salt noise: each pixel of each image independently set to 255 in all
  channels with a given probability.

Every array is produced from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.ndimage import gaussian_filter


@dataclass(frozen=True)
class SceneSpec:
    """Parameters of one synthetic scene-flow pair."""

    H: int
    W: int
    C: int
    seed: int
    n_segments: tuple = (3, 3)        # inclusive range of Voronoi segments
    d_range: tuple = (5, 30)          # disparity range [lo, hi] in px
    flow_max: int = 20                # |u|, |v| <= flow_max
    delta_max: int = 0                # |d1 - d0| <= delta_max per segment
    slope_max: float = 0.02           # planar disparity slope bound (px/px)
    occluder: bool = False            # one compact foreground segment
    occluder_scale: float = 1.0       # size multiplier of the occluder ellipse
    flow_max_v: int | None = None     # |v| bound if different from flow_max
    flow_power: float = 1.0           # |u| = flow_max * r^power, r ~ U(0, 1): > 1 favours small motions
    salt: float = 0.0                 # per-pixel salt probability per image
    sigma: float = 1.5                # Gaussian smoothing of the texture


@dataclass
class Scene:
    """Four uint8 images [H][W][C] plus integer ground truth."""

    spec: SceneSpec
    l0: np.ndarray
    l1: np.ndarray
    r0: np.ndarray
    r1: np.ndarray
    gt_fwd: np.ndarray                 # int16 [H][W][4] (u, v, d0, d1) at l0
    gt_inv: np.ndarray                 # int16 [H][W][4] at r1 (valid where inv_mask)
    inv_mask: np.ndarray               # bool [H][W]: r1 pixel received a splat
    vis_T: np.ndarray                  # bool [H][W]: l0 pixel visible in l1
    vis_S: np.ndarray                  # bool [H][W]: visible in r0
    vis_X: np.ndarray                  # bool [H][W]: visible in r1
    labels: np.ndarray = field(repr=False, default=None)  # segment id per l0 pixel

    def images(self):
        """(l0, l1, r0, r1) in the canonical order."""
        return self.l0, self.l1, self.r0, self.r1

    def stack(self):
        """uint8 [4][H][W][C] in the canonical order (l0, l1, r0, r1)."""
        return np.stack(self.images(), axis=0)


def smoothed_noise(rng: np.random.Generator, H: int, W: int, C: int,
                   sigma: float) -> np.ndarray:
    """Uniform noise, Gaussian-smoothed per channel (replicated border),
    min-max stretched per channel to 0..255 and rounded to uint8."""
    out = np.empty((H, W, C), dtype=np.uint8)
    for c in range(C):
        a = rng.uniform(0.0, 1.0, size=(H, W))
        a = gaussian_filter(a, sigma=sigma, mode="nearest")
        lo, hi = float(a.min()), float(a.max())
        a = (a - lo) * (255.0 / max(hi - lo, 1e-12))
        out[:, :, c] = np.clip(np.rint(a), 0, 255).astype(np.uint8)
    return out


def _motion(rng, F, Fv, power):
    if power == 1.0:
        return int(rng.integers(-F, F + 1)), int(rng.integers(-Fv, Fv + 1))
    r = rng.uniform(0.0, 1.0, 2) ** power * rng.choice([-1.0, 1.0], 2)
    return int(np.rint(F * r[0])), int(np.rint(Fv * r[1]))


def _segments(rng, spec: SceneSpec):
    H, W = spec.H, spec.W
    nseg = int(rng.integers(spec.n_segments[0], spec.n_segments[1] + 1))
    sites = np.stack([rng.uniform(0, H, nseg), rng.uniform(0, W, nseg)], axis=1)
    yy, xx = np.mgrid[0:H, 0:W]
    d2 = (yy[None] - sites[:, 0, None, None]) ** 2 + (xx[None] - sites[:, 1, None, None]) ** 2
    labels = np.argmin(d2, axis=0).astype(np.int32)
    dlo, dhi = spec.d_range
    F = spec.flow_max
    Fv = spec.flow_max if spec.flow_max_v is None else spec.flow_max_v
    d0 = np.zeros((H, W), np.int64)
    d1 = np.zeros((H, W), np.int64)
    u = np.zeros((H, W), np.int64)
    v = np.zeros((H, W), np.int64)
    for s in range(nseg):
        m = labels == s
        dc = rng.uniform(dlo, dhi)
        bx, by = rng.uniform(-spec.slope_max, spec.slope_max, 2) * (dhi - dlo) / 8.0
        plane = dc + bx * (xx - sites[s, 1]) / 8.0 + by * (yy - sites[s, 0]) / 8.0
        dd = np.clip(np.rint(plane), dlo, dhi).astype(np.int64)
        delta = int(rng.integers(-spec.delta_max, spec.delta_max + 1)) if spec.delta_max else 0
        us, vs = _motion(rng, F, Fv, spec.flow_power)
        d0[m] = dd[m]
        d1[m] = np.clip(dd[m] + delta, dlo, dhi)
        u[m] = us
        v[m] = vs
    if spec.occluder:
        cy, cx = rng.uniform(0.25 * H, 0.75 * H), rng.uniform(0.2 * W, 0.8 * W)
        ry = rng.uniform(0.12, 0.22) * H * spec.occluder_scale
        rx = rng.uniform(0.06, 0.12) * W * spec.occluder_scale
        m = ((yy - cy) / ry) ** 2 + ((xx - cx) / rx) ** 2 <= 1.0
        labels = labels.copy()
        labels[m] = nseg
        d0[m] = dhi
        delta = int(rng.integers(-spec.delta_max, 1)) if spec.delta_max else 0
        d1[m] = np.clip(dhi + delta, dlo, dhi)
        u[m], v[m] = _motion(rng, F, Fv, spec.flow_power)
    return labels, u, v, d0, d1


def _splat(src: np.ndarray, tx: np.ndarray, ty: np.ndarray, depth: np.ndarray,
           fill: np.ndarray):
    """Forward-splat every source pixel to (ty, tx); larger depth wins, ties to
    the smaller source index.  Returns (image, winner mask over source pixels,
    winner source index per target or -1)."""
    H, W, C = src.shape
    n = H * W
    inb = (tx >= 0) & (tx < W) & (ty >= 0) & (ty < H)
    sidx = np.arange(n, dtype=np.int64)
    t = (ty * W + tx).ravel()
    keep = inb.ravel()
    s_in = sidx[keep]
    t_in = t[keep]
    d_in = depth.ravel()[keep]
    # primary key: target; then larger depth first; then smaller source index
    order = np.lexsort((s_in, -d_in, t_in))
    t_sorted = t_in[order]
    first = np.ones(t_sorted.shape, bool)
    first[1:] = t_sorted[1:] != t_sorted[:-1]
    win_t = t_sorted[first]
    win_s = s_in[order][first]
    out = fill.reshape(n, C).copy()
    out[win_t] = src.reshape(n, C)[win_s]
    owner = np.full(n, -1, np.int64)
    owner[win_t] = win_s
    wmask = np.zeros(n, bool)
    wmask[win_s] = True
    return out.reshape(H, W, C), wmask.reshape(H, W), owner.reshape(H, W)


def make_scene(spec: SceneSpec) -> Scene:
    """Render one scene-flow pair from ``spec`` (deterministic in spec.seed)."""
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    H, W, C = spec.H, spec.W, spec.C
    l0 = smoothed_noise(rng, H, W, C, spec.sigma)
    labels, u, v, d0, d1 = _segments(rng, spec)
    yy, xx = np.mgrid[0:H, 0:W]
    fills = [smoothed_noise(rng, H, W, C, spec.sigma) for _ in range(3)]
    l1, vis_T, _ = _splat(l0, xx + u, yy + v, d1, fills[0])
    r0, vis_S, _ = _splat(l0, xx - d0, yy, d0, fills[1])
    r1, vis_X, owner = _splat(l0, xx + u - d1, yy + v, d1, fills[2])
    gt_fwd = np.stack([u, v, d0, d1], axis=-1).astype(np.int16)
    inv_mask = owner >= 0
    gt_inv = np.zeros((H, W, 4), np.int16)
    o = owner[inv_mask]
    gt_inv[inv_mask, 0] = (d1.ravel()[o] - d0.ravel()[o] - u.ravel()[o])
    gt_inv[inv_mask, 1] = -v.ravel()[o]
    gt_inv[inv_mask, 2] = d1.ravel()[o]
    gt_inv[inv_mask, 3] = d0.ravel()[o]
    imgs = [l0, l1, r0, r1]
    if spec.salt > 0:
        for im in imgs:
            m = rng.random((H, W)) < spec.salt
            im[m] = 255
    return Scene(spec, imgs[0], imgs[1], imgs[2], imgs[3], gt_fwd, gt_inv, inv_mask,
                 vis_T, vis_S, vis_X, labels)
