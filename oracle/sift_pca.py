"""FP64 oracle of the paper's own matching cost -- TEST INFRASTRUCTURE (only
the tests, the smoke check and the bench's CPU baseline use it).

SceneFlowFields, Section 3.1, "Matching Cost", eq. (1): the cost of a scene
flow vector at pixel p sums, over a 7 x 7 window around p and over the three
correspondences (temporal, stereo, cross), the Euclidean distance between the
first three principal components of the SIFT flow features of the reference
pixel and of its correspondence; the principal axes are those of the SIFT
features of all four images together; images are padded by replicating the
boundary pixel.

The paper gives no SIFT parameters.  The readings, following the dense SIFT
of SIFT flow (Liu et al., TPAMI 2011) and Lowe's descriptor (IJCV 2004):

* grey = channel mean;
* gradient by central differences with clamped neighbours; magnitude
  m = |(gx, gy)|, orientation atan2(gy, gx) with y pointing down;
* 8 orientation bins of 45 degrees, bin b centred at b * 45 degrees, each
  pixel's magnitude split linearly between the two nearest bin centres;
* 4 x 4 cells of 3 x 3 pixels, window rows and columns -6 .. +5 around the
  pixel, each pixel counted in its own cell only (flat window), pixels outside
  the image replaced by the clamped pixel;
* the 128 values (cell-major: index (4 i + j) * 8 + b for cell row i, cell
  column j, bin b) normalised to unit length, clamped at 0.2 and normalised
  again; an all-zero vector stays zero;
* PCA per pair: mean and covariance (1/N, N = 4 H W) over all descriptors of
  the four images, the three eigenvectors of largest eigenvalue, each signed so
  that its component of largest magnitude is positive (the first on ties);
  phi = axes (f - mean);
* cost(p) = sum over w in {-3..3}^2 and the three correspondences of
  || phi_R(clamp(p + w)) - phi_corr(clamp(p + w + o_corr)) ||_2, with
  o_T = (u, v), o_S = (-s d0, 0), o_X = (u - s d1, v): every lookup is clamped
  at the final coordinate (the padded image), distances are not squared.

Direction s = +1 uses the views (l0, l1, r0, r1) as (R, T, S, X), s = -1 uses
(r1, r0, l1, l0), as in the rest of the matcher.
"""
from __future__ import annotations

import numpy as np

NBINS = 8
CELL = 3           # pixels per cell side
NCELL = 4          # cells per descriptor side
DESC = NCELL * NCELL * NBINS
HALF = NCELL * CELL // 2   # 6: the window spans -6 .. +5
CLAMP = 0.2
WIN = np.arange(-3, 4)     # the 7 x 7 cost window


def view_index(s: int):
    """Canonical image index of (R, T, S, X) for direction s."""
    return (0, 1, 2, 3) if s > 0 else (3, 2, 1, 0)


def grey(img: np.ndarray) -> np.ndarray:
    """Channel mean of a [H][W][C] uint8 image, float64."""
    return img.astype(np.float64).mean(axis=2)


def orientation_energy(g: np.ndarray) -> np.ndarray:
    """Per-pixel orientation histogram [8][H][W]: the gradient magnitude split
    between the two bins whose centres enclose the gradient's orientation."""
    gp = np.pad(g, 1, mode="edge")
    gx = gp[1:-1, 2:] - gp[1:-1, :-2]
    gy = gp[2:, 1:-1] - gp[:-2, 1:-1]
    m = np.hypot(gx, gy)
    pos = np.mod(np.arctan2(gy, gx) / (2 * np.pi / NBINS), NBINS)
    lo = np.floor(pos)
    frac = pos - lo
    b0 = lo.astype(np.int64) % NBINS
    b1 = (b0 + 1) % NBINS
    H, W = g.shape
    O = np.zeros((NBINS, H, W))
    ii, jj = np.indices((H, W))
    np.add.at(O, (b0, ii, jj), m * (1 - frac))
    np.add.at(O, (b1, ii, jj), m * frac)
    return O


def cell_sums(O: np.ndarray) -> np.ndarray:
    """C[b][Y + 6][X + 6] = sum of O[b] over the 3 x 3 cell with top-left
    corner (Y, X), coordinates clamped, for Y in -6 .. H + 2, X in -6 .. W + 2."""
    _, H, W = O.shape
    Op = np.pad(O, ((0, 0), (HALF, HALF - 1), (HALF, HALF - 1)), mode="edge")
    He, We = H + 2 * HALF - CELL, W + 2 * HALF - CELL
    Cs = np.zeros((NBINS, He, We))
    for a in range(CELL):
        for c in range(CELL):
            Cs += Op[:, a:a + He, c:c + We]
    return Cs


def normalise(v: np.ndarray) -> np.ndarray:
    """Unit length, clamp at 0.2, unit length again, along the last axis."""
    v = np.asarray(v, dtype=np.float64)
    n = np.linalg.norm(v, axis=-1, keepdims=True)
    v = np.divide(v, n, out=np.zeros_like(v), where=n > 0)
    v = np.minimum(v, CLAMP)
    n = np.linalg.norm(v, axis=-1, keepdims=True)
    return np.divide(v, n, out=np.zeros_like(v), where=n > 0)


def dense_sift(img: np.ndarray) -> np.ndarray:
    """Dense SIFT [H][W][128] of a [H][W][C] uint8 image."""
    g = grey(img)
    H, W = g.shape
    Cs = cell_sums(orientation_energy(g))
    v = np.zeros((H, W, DESC))
    for i in range(NCELL):
        for j in range(NCELL):
            k = (i * NCELL + j) * NBINS
            v[:, :, k:k + NBINS] = Cs[:, CELL * i:CELL * i + H, CELL * j:CELL * j + W].transpose(1, 2, 0)
    return normalise(v)


def sign_fix(axes: np.ndarray) -> np.ndarray:
    """Each row signed so that its component of largest magnitude is positive."""
    axes = np.array(axes, dtype=np.float64)
    for r in range(axes.shape[0]):
        k = int(np.argmax(np.abs(axes[r])))
        if axes[r, k] < 0:
            axes[r] = -axes[r]
    return axes


def pca(feats: np.ndarray, ncomp: int = 3):
    """Mean, covariance (1/N), the ncomp largest eigenvalues and their axes
    [ncomp][D] of the rows of feats [N][D]."""
    F = np.asarray(feats, dtype=np.float64).reshape(-1, feats.shape[-1])
    mean = F.mean(axis=0)
    Xc = F - mean
    cov = Xc.T @ Xc / F.shape[0]
    w, V = np.linalg.eigh(cov)
    order = np.argsort(-w, kind="stable")[:ncomp]
    return mean, cov, w[order], sign_fix(V[:, order].T)


def sift_pca_features(imgs: np.ndarray):
    """imgs [4][H][W][C] uint8 (l0, l1, r0, r1) -> dict with the SIFT features
    [4][H][W][128], mean [128], cov [128][128], eigval [3], axes [3][128] and
    phi [4][H][W][3]."""
    sift = np.stack([dense_sift(im) for im in imgs])
    mean, cov, eigval, axes = pca(sift)
    phi = (sift - mean) @ axes.T
    return {"sift": sift, "mean": mean, "cov": cov, "eigval": eigval, "axes": axes, "phi": phi}


def cost(phi: np.ndarray, hyp: np.ndarray, s: int = 1) -> np.ndarray:
    """Eq. (1) per pixel: phi [4][H][W][k] (canonical views), hyp [H][W][4]
    (u, v, d0, d1) -> float64 [H][W]."""
    _, H, W, _ = phi.shape
    R, T, S, X = (phi[i] for i in view_index(s))
    u, v = hyp[..., 0].astype(np.int64), hyp[..., 1].astype(np.int64)
    d0, d1 = hyp[..., 2].astype(np.int64), hyp[..., 3].astype(np.int64)
    ys, xs = np.indices((H, W))
    offs = ((T, u, v), (S, -s * d0, np.zeros_like(d0)), (X, u - s * d1, v))
    out = np.zeros((H, W))
    for wy in WIN:
        for wx in WIN:
            py, px = ys + wy, xs + wx
            ref = R[np.clip(py, 0, H - 1), np.clip(px, 0, W - 1)]
            for img, ox, oy in offs:
                tgt = img[np.clip(py + oy, 0, H - 1), np.clip(px + ox, 0, W - 1)]
                out += np.sqrt(((ref - tgt) ** 2).sum(axis=-1))
    return out
