"""Independent NumPy routes used to pin the oracle (test code only).

Nothing here re-types the oracle's loops.  The WHT is taken from
``scipy.linalg.hadamard`` reordered to sequency order.  Descriptor distances go
through Parseval: the four lowest-sequency length-8 Walsh functions are constant
on pixel pairs and equal the length-4 sequency-ordered Walsh functions, so the
4x4 coefficient block of a patch is W4 B W4^T with B the 4x4 matrix of 2x2-bin
sums, and since W4 W4^T = 4 I the squared distance of two 16-coefficient
descriptors is 16 times the squared distance of their bin sums.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import hadamard


def sequency_walsh(N: int) -> np.ndarray:
    """Rows of the Sylvester Hadamard matrix sorted by number of sign changes."""
    Hm = hadamard(N)
    changes = (np.diff(Hm, axis=1) != 0).sum(axis=1)
    return Hm[np.argsort(changes, kind="stable")].astype(np.int64)


def patch_indices(H, W, y, x, n):
    ys = np.clip(y + n * (np.arange(8) - 3), 0, H - 1)
    xs = np.clip(x + n * (np.arange(8) - 3), 0, W - 1)
    return ys, xs


def patch(img, y, x, c, n):
    H, W = img.shape[:2]
    ys, xs = patch_indices(H, W, y, x, n)
    return img[np.ix_(ys, xs)][:, :, c].astype(np.int64)


def wht_block(P: np.ndarray) -> np.ndarray:
    """4x4 lowest-sequency block of the full 8x8 2-D WHT (a rows, b columns)."""
    W8 = sequency_walsh(8)
    return (W8 @ P @ W8.T)[:4, :4]


def bin_sums(img, n):
    """B[y][x][c][4][4]: 2x2-bin sums of the stride-n 8x8 patch at every pixel."""
    img = np.asarray(img)
    H, W, C = img.shape
    ys = np.clip(np.arange(H)[:, None] + n * (np.arange(8)[None, :] - 3), 0, H - 1)  # H x 8
    xs = np.clip(np.arange(W)[:, None] + n * (np.arange(8)[None, :] - 3), 0, W - 1)  # W x 8
    P = img.astype(np.int64)[ys[:, None, :, None], xs[None, :, None, :], :]  # H W 8 8 C
    P = np.moveaxis(P, -1, 2)  # H W C 8 8
    B = P.reshape(H, W, C, 4, 2, 4, 2).sum(axis=(4, 6))
    return B


def views(imgs, s):
    l0, l1, r0, r1 = imgs
    return (l0, l1, r0, r1) if s > 0 else (r1, r0, l1, l0)


def targets(x, y, h, s):
    u, v, d0, d1 = (int(t) for t in h)
    return [(x + u, y + v), (x - s * d0, y), (x + u - s * d1, y + v)]


def cost_parseval(Bs, s, x, y, h):
    """Eq. (1) cost via bin sums.  Bs: per-view bin-sum maps in (l0, l1, r0, r1)."""
    R, T, S, X = views(Bs, s)
    H, W = R.shape[:2]
    total = 0
    for img, (tx, ty) in zip((T, S, X), targets(x, y, h, s)):
        tx = min(max(tx, 0), W - 1)
        ty = min(max(ty, 0), H - 1)
        total += 16 * int(((R[y, x] - img[ty, tx]) ** 2).sum())
    return total


def ssd_maps(Bq, Bmap):
    """16 * sum (Bq - Bmap[y][x])^2 for every pixel of Bmap."""
    return 16 * ((Bmap - Bq[None, None]) ** 2).sum(axis=(2, 3, 4))


def brute_init(Bs, s, level, fmax, dmax):
    """Exhaustive exact nearest neighbours per view (Section 3.1 initialisation
    read as exact search), lowest linear target index on ties."""
    n = 1 << level
    R, T, S, X = views(Bs, s)
    H, W = R.shape[:2]
    Hk, Wk = (H + n - 1) // n, (W + n - 1) // n
    hyp = np.zeros((Hk, Wk, 4), np.int64)
    cst = np.zeros((Hk, Wk), np.int64)
    gy = np.arange(0, H, n)
    gx = np.arange(0, W, n)
    for i in range(Hk):
        for j in range(Wk):
            x, y = n * j, n * i
            q = R[y, x]
            # temporal: grid targets within the box
            cy = gy[np.abs(gy - y) <= fmax]
            cx = gx[np.abs(gx - x) <= fmax]
            e = 16 * ((T[np.ix_(cy, cx)] - q) ** 2).sum(axis=(2, 3, 4))
            lin = cy[:, None] * W + cx[None, :]
            k = np.lexsort((lin.ravel(), e.ravel()))[0]
            ty, tx = cy[k // len(cx)], cx[k % len(cx)]
            u, v = tx - x, ty - y
            # stereo, same row
            d = s * (x - gx)
            cand = gx[(d >= 0) & (d <= dmax)]
            e = 16 * ((S[y, cand] - q) ** 2).sum(axis=(1, 2, 3))
            tx0 = cand[np.lexsort((cand, e))[0]]
            d0 = s * (x - tx0)
            # cross, row y + v
            d = s * (x + u - gx)
            cand = gx[(d >= 0) & (d <= dmax)]
            e = 16 * ((X[y + v, cand] - q) ** 2).sum(axis=(1, 2, 3))
            tx1 = cand[np.lexsort((cand, e))[0]]
            d1 = s * (x + u - tx1)
            hyp[i, j] = (u, v, d0, d1)
            cst[i, j] = cost_parseval(Bs, s, x, y, hyp[i, j])
    return hyp, cst


def exhaustive_min(Bs, s, level, fmax, dmax):
    """Minimum of eq. (1) over every integer hypothesis in the search bounds,
    per grid pixel (tiny images only)."""
    n = 1 << level
    R, T, S, X = views(Bs, s)
    H, W = R.shape[:2]
    Hk, Wk = (H + n - 1) // n, (W + n - 1) // n
    out = np.zeros((Hk, Wk), np.int64)
    uu = np.arange(-fmax, fmax + 1)
    dd = np.arange(0, dmax + 1)
    for i in range(Hk):
        for j in range(Wk):
            x, y = n * j, n * i
            q = R[y, x]
            ty = np.clip(y + uu, 0, H - 1)
            tx = np.clip(x + uu, 0, W - 1)
            eT = 16 * ((T[np.ix_(ty, tx)] - q) ** 2).sum(axis=(2, 3, 4))  # [v][u]
            sx = np.clip(x - s * dd, 0, W - 1)
            eS = 16 * ((S[y, sx] - q) ** 2).sum(axis=(1, 2, 3))  # [d0]
            best = None
            for vi, v in enumerate(uu):
                yy = min(max(y + v, 0), H - 1)
                # cross: x + u - s d1 for every (u, d1)
                xx = np.clip(x + uu[:, None] - s * dd[None, :], 0, W - 1)
                eX = 16 * ((X[yy][xx] - q) ** 2).sum(axis=(2, 3, 4))  # [u][d1]
                tot = (eT[vi][:, None] + eX).min() + eS.min()
                best = tot if best is None else min(best, tot)
            out[i, j] = best
    return out


def region_filter_union_find(hyp, valid, tau, s_c):
    """Region filter by union-find over the similarity edges (a different
    algorithm from the oracle's breadth-first growing): edges join
    4-neighbours that are both valid with every vector component within tau;
    a component is dropped when it has fewer than s_c pixels and an invalid
    4-neighbour of one of its pixels is within tau of that pixel's vector."""
    H, W = valid.shape
    parent = np.arange(H * W)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    h = hyp.reshape(H * W, 4).astype(np.int64)
    v = valid.reshape(-1).astype(bool)
    sim = lambda p, q: bool(np.all(np.abs(h[p] - h[q]) <= tau))
    for y in range(H):
        for x in range(W):
            p = y * W + x
            for q in ([p + 1] if x + 1 < W else []) + ([p + W] if y + 1 < H else []):
                if v[p] and v[q] and sim(p, q):
                    a, b = find(p), find(q)
                    if a != b:
                        parent[max(a, b)] = min(a, b)
    root = np.array([find(p) for p in range(H * W)])
    size = np.bincount(root[v], minlength=H * W)
    flagged = np.zeros(H * W, bool)
    for y in range(H):
        for x in range(W):
            p = y * W + x
            if v[p]:
                continue
            for yn, xn in ((y, x - 1), (y, x + 1), (y - 1, x), (y + 1, x)):
                if 0 <= yn < H and 0 <= xn < W:
                    q = yn * W + xn
                    if v[q] and sim(p, q):
                        flagged[root[q]] = True
    drop = flagged[root] & (size[root] < s_c)
    return (v & ~drop).reshape(H, W).astype(np.uint8)


def sparsify_blocks(keep, err):
    """Per 3x3 block: argmin over (err, raster index) of the kept pixels, by a
    padded reshape and a lexicographic key; -1 for empty blocks."""
    H, W = keep.shape
    Hb, Wb = -(-H // 3), -(-W // 3)
    idx = np.full((Hb * 3, Wb * 3), -1, np.int64)
    idx[:H, :W] = np.arange(H * W).reshape(H, W)
    e = np.full((Hb * 3, Wb * 3), np.iinfo(np.int64).max, np.int64)
    k = np.zeros((Hb * 3, Wb * 3), bool)
    k[:H, :W] = keep.astype(bool)
    e[:H, :W] = err.astype(np.int64)
    key = np.where(k, e * (H * W + 1) + idx, np.iinfo(np.int64).max)
    blocks = key.reshape(Hb, 3, Wb, 3).transpose(0, 2, 1, 3).reshape(Hb, Wb, 9)
    m = blocks.min(axis=2)
    out = np.where(m == np.iinfo(np.int64).max, -1, m % (H * W + 1))
    return out.astype(np.int32)


def brute_init_leaves(Bs, s, level, fmax, dmax, leaves):
    """Initialisation with `leaves` temporal leaves by brute force: the whole
    temporal box sorted by (distance, linear index) with lexsort, each of the
    first `leaves` targets paired with the exhaustive cross argmin of its row,
    the combination with the smallest T + S + X distance (first on ties)."""
    n = 1 << level
    R, T, S, X = views(Bs, s)
    H, W = R.shape[:2]
    Hk, Wk = (H + n - 1) // n, (W + n - 1) // n
    hyp = np.zeros((Hk, Wk, 4), np.int64)
    joint = np.zeros((Hk, Wk), np.int64)
    gy = np.arange(0, H, n)
    gx = np.arange(0, W, n)

    def row_argmin(img_row, q, tx_of_d):
        d = np.arange(0, dmax + 1, n)
        tx = tx_of_d(d)
        ok = (tx >= 0) & (tx < W)
        d, tx = d[ok], tx[ok]
        e = 16 * ((img_row[tx] - q) ** 2).sum(axis=(1, 2, 3))
        k = np.lexsort((tx, e))[0]
        return d[k], e[k]

    for i in range(Hk):
        for j in range(Wk):
            x, y = n * j, n * i
            q = R[y, x]
            cy = gy[np.abs(gy - y) <= fmax]
            cx = gx[np.abs(gx - x) <= fmax]
            e = 16 * ((T[np.ix_(cy, cx)] - q) ** 2).sum(axis=(2, 3, 4))
            lin = cy[:, None] * W + cx[None, :]
            order = np.lexsort((lin.ravel(), e.ravel()))[:leaves]
            d0, eS = row_argmin(S[y], q, lambda d: x - s * d)
            best = None
            for k in order:
                ty, tx = cy[k // len(cx)], cx[k % len(cx)]
                u, v = tx - x, ty - y
                d1, eX = row_argmin(X[y + v], q, lambda d: x + u - s * d)
                tot = e.ravel()[k] + eS + eX
                if best is None or tot < best[0]:
                    best = (tot, (u, v, d0, d1))
            joint[i, j] = best[0]
            hyp[i, j] = best[1]
    return hyp, joint
