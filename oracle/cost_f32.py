"""FP64 oracle of the differentiable window form of the matching cost --
TEST INFRASTRUCTURE.

Eq. (1) of SceneFlowFields (Section 3.1) sums, over the three correspondences
(temporal (x + u, y + v), stereo (x - s d0, y), cross (x + u - s d1, y + v)),
the distances of per-pixel features over a window around the pixel.  With
real-valued feature maps F (C channels per pixel) and squared distances, the
per-pixel cost at fixed vectors h is

    cost(p) = sum_corr sum_{w in {-3..4}^2} sum_c
              (F_R(clamp(p + w), c) - F_corr(clamp(t_corr(p) + w), c))^2,

    t_corr(p) = clamp(p + o_corr(h_p)),

with replicated borders (clamp) as in Section 3.1, and the loss L = sum_p
g_p cost(p) for upstream weights g.  Its gradient follows from the chain rule:
each term with difference delta adds 2 g_p delta to the reference entry and
subtracts it from the target entry.  This module computes both in float64 by
those definitions, plus a central finite difference of L for single entries.

Maps are given in the canonical order (l0, l1, r0, r1); direction s = +1 uses
(R, T, S, X) = (l0, l1, r0, r1), s = -1 uses (r1, r0, l1, l0).
"""
from __future__ import annotations

import numpy as np

WIN = np.arange(-3, 5)  # window offsets, the 8x8 patch of the descriptors


def view_index(s: int):
    """Canonical map index of (R, T, S, X) for direction s."""
    return (0, 1, 2, 3) if s > 0 else (3, 2, 1, 0)


def _targets(hyp, s, ys, xs, H, W):
    u = hyp[ys, xs, 0].astype(np.int64)
    v = hyp[ys, xs, 1].astype(np.int64)
    d0 = hyp[ys, xs, 2].astype(np.int64)
    d1 = hyp[ys, xs, 3].astype(np.int64)
    ty = np.clip(ys + v, 0, H - 1)
    return [(ty, np.clip(xs + u, 0, W - 1)),
            (ys, np.clip(xs - s * d0, 0, W - 1)),
            (ty, np.clip(xs + u - s * d1, 0, W - 1))]


def cost_px_at(F, hyp, s, ys, xs):
    """cost(p) for the pixels (ys, xs); F: 4 maps [H][W][C] (float64)."""
    R = view_index(s)
    H, W, _ = F[0].shape
    ys = np.asarray(ys, np.int64)
    xs = np.asarray(xs, np.int64)
    tg = _targets(hyp, s, ys, xs, H, W)
    out = np.zeros(ys.shape, np.float64)
    for dy in WIN:
        ry = np.clip(ys + dy, 0, H - 1)
        for dx in WIN:
            rx = np.clip(xs + dx, 0, W - 1)
            a = F[R[0]][ry, rx]
            for k, (ty, tx) in enumerate(tg):
                b = F[R[k + 1]][np.clip(ty + dy, 0, H - 1), np.clip(tx + dx, 0, W - 1)]
                out += ((a - b) ** 2).sum(axis=-1)
    return out


def window_cost(F, hyp, s):
    """cost(p) for every pixel, [H][W] float64."""
    H, W, _ = F[0].shape
    yy, xx = np.indices((H, W))
    out = np.empty((H, W), np.float64)
    rows = max(1, 200_000 // W)
    for y0 in range(0, H, rows):
        sl = slice(y0, min(H, y0 + rows))
        out[sl] = cost_px_at(F, hyp, s, yy[sl], xx[sl])
    return out


def window_cost_grad(F, hyp, s, g):
    """dL/dF for L = sum_p g_p cost(p): four maps [H][W][C] float64 in the
    canonical order, accumulated term by term (np.add.at)."""
    R = view_index(s)
    H, W, C = F[0].shape
    G = [np.zeros((H, W, C), np.float64) for _ in range(4)]
    yy, xx = np.indices((H, W))
    ys, xs = yy.ravel(), xx.ravel()
    gg = np.asarray(g, np.float64).ravel()[:, None]
    tg = _targets(hyp, s, ys, xs, H, W)
    for dy in WIN:
        ry = np.clip(ys + dy, 0, H - 1)
        for dx in WIN:
            rx = np.clip(xs + dx, 0, W - 1)
            a = F[R[0]][ry, rx]
            for k, (ty, tx) in enumerate(tg):
                by = np.clip(ty + dy, 0, H - 1)
                bx = np.clip(tx + dx, 0, W - 1)
                d = 2.0 * gg * (a - F[R[k + 1]][by, bx])
                np.add.at(G[R[0]], (ry, rx), d)
                np.add.at(G[R[k + 1]], (by, bx), -d)
    return G


def affected_pixels(hyp, s, m, y, x, H, W):
    """Pixels whose cost involves entry (map m, y, x): reference windows
    containing (y, x) and target windows containing it (with clamping)."""
    R = view_index(s)
    yy, xx = np.indices((H, W))
    ys, xs = yy.ravel(), xx.ravel()
    hit = np.zeros(ys.shape, bool)
    if R[0] == m:
        hit |= (np.abs(np.clip(ys[:, None] + WIN, 0, H - 1) - y).min(axis=1) == 0) & \
               (np.abs(np.clip(xs[:, None] + WIN, 0, W - 1) - x).min(axis=1) == 0)
    tg = _targets(hyp, s, ys, xs, H, W)
    for k, (ty, tx) in enumerate(tg):
        if R[k + 1] != m:
            continue
        hit |= (np.abs(np.clip(ty[:, None] + WIN, 0, H - 1) - y).min(axis=1) == 0) & \
               (np.abs(np.clip(tx[:, None] + WIN, 0, W - 1) - x).min(axis=1) == 0)
    return ys[hit], xs[hit]


def _preimage(q, w, n):
    """All p in [0, n) with clamp(p + w) == q.  With |w| <= 4 they lie within
    8 of q (a border q also collects the clamped positions beyond it)."""
    p = np.arange(max(0, q - 8), min(n, q + 9))
    return p[np.clip(p + w, 0, n - 1) == q]


class FiniteDifferences:
    """Central differences of L for many single entries at one (F, hyp, g):
    pixels whose cost involves an entry are found by enumerating the window
    preimages of the entry, through per-correspondence buckets of pixels by
    target centre (built once with a stable argsort)."""

    def __init__(self, F, hyp, s, g):
        self.F, self.hyp, self.s, self.g = F, hyp, s, np.asarray(g, np.float64)
        H, W, _ = F[0].shape
        self.H, self.W = H, W
        yy, xx = np.indices((H, W))
        self.ys, self.xs = yy.ravel(), xx.ravel()
        self.buckets = []
        for ty, tx in _targets(hyp, s, self.ys, self.xs, H, W):
            key = ty * W + tx
            order = np.argsort(key, kind="stable")
            self.buckets.append((key[order], order))

    def affected(self, m, y, x):
        R = view_index(self.s)
        H, W = self.H, self.W
        # window positions w whose preimage contains a given pixel/centre cell
        cells = set()
        for wy in WIN:
            for wx in WIN:
                cy, cx = _preimage(y, wy, H), _preimage(x, wx, W)
                cells.update(int(a) * W + int(b) for a in cy for b in cx)
        cells = np.array(sorted(cells), np.int64)
        picked = []
        if R[0] == m:
            picked.append(cells)
        for k in range(3):
            if R[k + 1] != m:
                continue
            keys, order = self.buckets[k]
            lo = np.searchsorted(keys, cells)
            hi = np.searchsorted(keys, cells + 1)
            for a, b in zip(lo, hi):
                picked.append(order[a:b])
        if not picked:
            return np.zeros(0, np.int64), np.zeros(0, np.int64)
        idx = np.unique(np.concatenate(picked))
        return self.ys[idx], self.xs[idx]

    def grad_entry(self, m, y, x, c, eps=1e-3):
        ys, xs = self.affected(m, y, x)
        if len(ys) == 0:
            return 0.0
        gw = self.g[ys, xs]
        Fm = self.F[m]
        old = Fm[y, x, c]
        try:  # perturb in place, restore afterwards
            Fm[y, x, c] = old + eps
            lp = (gw * cost_px_at(self.F, self.hyp, self.s, ys, xs)).sum()
            Fm[y, x, c] = old - eps
            lm = (gw * cost_px_at(self.F, self.hyp, self.s, ys, xs)).sum()
        finally:
            Fm[y, x, c] = old
        return (lp - lm) / (2 * eps)


def fd_grad_entry(F, hyp, s, g, m, y, x, c, eps=1e-3):
    """Central finite difference of L w.r.t. F[m][y, x, c] (float64).  L is
    quadratic in F, so the central difference is exact up to rounding."""
    H, W, _ = F[0].shape
    ys, xs = affected_pixels(hyp, s, m, y, x, H, W)
    gw = np.asarray(g, np.float64)[ys, xs]
    Fp = [f if i != m else f.copy() for i, f in enumerate(F)]
    old = F[m][y, x, c]
    Fp[m][y, x, c] = old + eps
    lp = (gw * cost_px_at(Fp, hyp, s, ys, xs)).sum()
    Fp[m][y, x, c] = old - eps
    lm = (gw * cost_px_at(Fp, hyp, s, ys, xs)).sum()
    return (lp - lm) / (2 * eps)
