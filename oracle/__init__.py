"""CPU oracle of the sparse scene-flow matching stage (SceneFlowFields,
arXiv 1710.10096, Section 3.1) -- TEST INFRASTRUCTURE.

A plain C implementation (``sff_oracle.c``) of what the GPU path computes,
wrapped for NumPy arrays.  Only the tests, the smoke check and the bench's
CPU-baseline leg use it; the GPU library never imports, links or calls it, and
it shares no code with that library.

Each wrapper names the passage its C function follows:

* ``philox4x32_10``  -- Philox4x32-10 counter-based generator (Salmon et al.,
  SC'11), used for the random search.
* ``lanczos_q14``, ``smooth`` -- scale simulation, Section 3.1
  "Multi-Scale Propagation" (area downsampling, Lanczos upsampling).
* ``wht``, ``features`` -- WHT feature vectors, Section 3.1 "Initialization".
* ``cost`` -- matching cost, eq. (1).
* ``init_nn`` -- initialisation by nearest neighbours, Section 3.1.
* ``match_level`` -- propagation and random search, Section 3.1.
* ``consistency`` -- consistency check, Section 3.1 and tau_c of Section 5.
* ``region_filter`` -- region filter, Section 3.1 (second step of the
  consistency check) and s_c of Section 5.
* ``sparsify`` -- best match per 3x3 block, Section 3.2 "Sparsification".
* ``grey``, ``census``, ``sgm_cost``, ``sgm_path``, ``sgm``,
  ``disparity_fill`` -- the disparity fill by semi-global matching, Section 3.1
  (last paragraph of "Consistency Check").
* ``match_pair`` -- the whole stage for one pair, Section 3 overview
  (``schedule="scan"``: the paper's sequential four-corner propagation,
  ``match_level_scan``, CPU only, to measure the red-black schedule).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB, build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i32 = ctypes.c_int
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_lanczos_q14.argtypes = [i32, P]
        L.orc_smooth.argtypes = [P, i32, i32, i32, i32, P]
        L.orc_wht.argtypes = [P, i32, i32, i32, i32, P]
        L.orc_features.argtypes = [P, i32, i32, i32, i32, P]
        L.orc_cost.argtypes = [P, P, P, P, i32, i32, i32, i32, i32, i32, P]
        L.orc_cost.restype = ctypes.c_uint32
        L.orc_init_nn.argtypes = [P, P, P, P] + [i32] * 8 + [P, P]
        L.orc_init_nn_leaves.argtypes = [P] * 4 + [i32] * 9 + [P, P]
        L.orc_cost_sift.argtypes = [P, i32, i32, i32, P, P]
        L.orc_match_sift.argtypes = ([P, i32, i32, i32, ctypes.c_uint64] + [i32] * 7 + [P, P])
        L.orc_match_level.argtypes = ([P, P, P, P] + [i32] * 5 + [ctypes.c_uint64]
                                      + [i32] * 5 + [P, i32, i32, P, P])
        L.orc_consistency.argtypes = [P, P, i32, i32, i32, P, P]
        L.orc_grey.argtypes = [P, i32, i32, i32, P]
        L.orc_census.argtypes = [P, i32, i32, P]
        L.orc_sgm_cost.argtypes = [P, P, i32, i32, i32, P]
        L.orc_sgm_path.argtypes = [P, i32, i32, i32, i32, i32, i32, i32, P]
        L.orc_sgm.argtypes = [P, P, i32, i32, i32, i32, i32, i32, P]
        L.orc_disparity_fill.argtypes = [P, P, P, i32, i32, i32, P]
        L.orc_region_filter.argtypes = [P, P, i32, i32, i32, i32, P]
        L.orc_sparsify.argtypes = [P, P, i32, i32, P]
        L.orc_match_pair.argtypes = ([P] + [i32] * 10 + [ctypes.c_uint64, i32] + [P] * 4)
        L.orc_match_pair_schedule.argtypes = ([P] + [i32] * 10 + [ctypes.c_uint64, i32, i32, i32]
                                              + [P] * 4)
        L.orc_match_level_scan.argtypes = ([P] * 4 + [i32] * 5 + [ctypes.c_uint64] + [i32] * 5
                                           + [P, i32, P, P])
        L.orc_max_threads.restype = i32
        L.orc_rs_candidate.argtypes = ([ctypes.c_uint64] + [i32] * 10 + [P, P])
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def max_threads() -> int:
    return int(lib().orc_max_threads())


def philox4x32_10(ctr, key) -> np.ndarray:
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def rs_candidate(seed: int, level: int, s: int, i: int, j: int, Wk: int, it: int, t: int,
                 rs_r0: int, fmax: int, dmax: int, centre) -> np.ndarray:
    """Random-search sample t of grid pixel (i, j) in iteration it (Section 3.1)."""
    c = _c(centre, np.int16)
    out = np.zeros(4, np.int16)
    lib().orc_rs_candidate(seed, level, s, i, j, Wk, it, t, rs_r0, fmax, dmax, _p(c), _p(out))
    return out


def lanczos_q14(n: int) -> np.ndarray:
    t = np.zeros((n, 6), np.int32)
    lib().orc_lanczos_q14(n, _p(t))
    return t


def smooth(img: np.ndarray, n: int) -> np.ndarray:
    img = _c(img, np.uint8)
    H, W, C = img.shape
    out = np.zeros_like(img)
    assert lib().orc_smooth(_p(img), H, W, C, n, _p(out)) == 0
    return out


def wht(S: np.ndarray, n: int) -> np.ndarray:
    S = _c(S, np.uint8)
    H, W, C = S.shape
    out = np.zeros((H, W, C, 16), np.int16)
    assert lib().orc_wht(_p(S), H, W, C, n, _p(out)) == 0
    return out


def features(img: np.ndarray, level: int) -> np.ndarray:
    img = _c(img, np.uint8)
    H, W, C = img.shape
    out = np.zeros((H, W, C, 16), np.int16)
    assert lib().orc_features(_p(img), H, W, C, level, _p(out)) == 0
    return out


def _descs(descs):
    ds = [_c(d, np.int16) for d in descs]
    H, W, C, _ = ds[0].shape
    return ds, H, W, C


def cost(descs, s: int, x: int, y: int, h) -> int:
    ds, H, W, C = _descs(descs)
    hh = _c(h, np.int16)
    return int(lib().orc_cost(*[_p(d) for d in ds], H, W, C, s, x, y, _p(hh)))


def grid_shape(H: int, W: int, level: int):
    n = 1 << level
    return (H + n - 1) // n, (W + n - 1) // n


def init_nn(descs, level: int, s: int, fmax: int, dmax: int, nthreads: int = 0,
            leaves: int = 1):
    """Exact-NN initialisation; ``leaves`` > 1 keeps that many temporal leaves
    and picks the cheapest combination by eq. (1)."""
    ds, H, W, C = _descs(descs)
    Hk, Wk = grid_shape(H, W, level)
    hyp = np.zeros((Hk, Wk, 4), np.int16)
    cst = np.zeros((Hk, Wk), np.uint32)
    if leaves == 1:
        assert lib().orc_init_nn(*[_p(d) for d in ds], H, W, C, level, s, fmax, dmax, nthreads,
                                 _p(hyp), _p(cst)) == 0
    else:
        assert lib().orc_init_nn_leaves(*[_p(d) for d in ds], H, W, C, level, s, fmax, dmax,
                                        leaves, nthreads, _p(hyp), _p(cst)) == 0
    return hyp, cst


def match_level(descs, level: int, s: int, seed: int, iters: int, rs_r0: int, rs_samples: int,
                fmax: int, dmax: int, hyp, cost=None, hyp_coarse=None, order: int = 0,
                nthreads: int = 0):
    """Run one level.  With ``hyp_coarse`` the level starts from the hand-off of
    the coarser field (``hyp``/``cost`` are then outputs only); otherwise it
    starts from ``hyp``/``cost``.  Returns new (hyp, cost) arrays."""
    ds, H, W, C = _descs(descs)
    Hk, Wk = grid_shape(H, W, level)
    h = np.array(hyp, dtype=np.int16, copy=True, order="C") if hyp is not None else \
        np.zeros((Hk, Wk, 4), np.int16)
    c = np.array(cost, dtype=np.uint32, copy=True, order="C") if cost is not None else \
        np.zeros((Hk, Wk), np.uint32)
    assert h.shape == (Hk, Wk, 4) and c.shape == (Hk, Wk)
    hc = None
    if hyp_coarse is not None:
        hc = _c(hyp_coarse, np.int16)
        assert hc.shape[:2] == grid_shape(H, W, level + 1)
    assert lib().orc_match_level(*[_p(d) for d in ds], H, W, C, level, s, seed, iters, rs_r0,
                                 rs_samples, fmax, dmax,
                                 _p(hc) if hc is not None else None, order, nthreads,
                                 _p(h), _p(c)) == 0
    return h, c


def consistency(hyp_fwd, hyp_inv, tau: int):
    hf = _c(hyp_fwd, np.int16)
    hi = _c(hyp_inv, np.int16)
    H, W, _ = hf.shape
    valid = np.zeros((H, W), np.uint8)
    err = np.zeros((H, W), np.uint32)
    assert lib().orc_consistency(_p(hf), _p(hi), H, W, tau, _p(valid), _p(err)) == 0
    return valid, err


def grey(img):
    """Rounded channel mean, uint8 [H][W] (disparity fill reading)."""
    im = _c(img, np.uint8)
    H, W, C = im.shape
    out = np.zeros((H, W), np.uint8)
    assert lib().orc_grey(_p(im), H, W, C, _p(out)) == 0
    return out


def census(grey_img):
    """5x5 census words uint32 [H][W]."""
    g = _c(grey_img, np.uint8)
    H, W = g.shape
    out = np.zeros((H, W), np.uint32)
    assert lib().orc_census(_p(g), H, W, _p(out)) == 0
    return out


def sgm_cost(cl, cr, D: int):
    """Hamming cost volume uint8 [H][W][D]."""
    a, b = _c(cl, np.uint32), _c(cr, np.uint32)
    H, W = a.shape
    out = np.zeros((H, W, D), np.uint8)
    assert lib().orc_sgm_cost(_p(a), _p(b), H, W, D, _p(out)) == 0
    return out


def sgm_path(cost, P1: int, P2: int, dx: int, dy: int):
    """Aggregated cost int32 [H][W][D] along one path direction."""
    c = _c(cost, np.uint8)
    H, W, D = c.shape
    out = np.zeros((H, W, D), np.int32)
    assert lib().orc_sgm_path(_p(c), H, W, D, P1, P2, dx, dy, _p(out)) == 0
    return out


def sgm(left, right, D: int, P1: int, P2: int):
    """SGM disparity int16 [H][W] of a rectified pair (Section 3.1, last
    paragraph of "Consistency Check"; Hirschmueller 2008)."""
    l, r = _c(left, np.uint8), _c(right, np.uint8)
    H, W, C = l.shape
    out = np.zeros((H, W), np.int16)
    assert lib().orc_sgm(_p(l), _p(r), H, W, C, D, P1, P2, _p(out)) == 0
    return out


def disparity_fill(hyp_fwd, valid, disp, tau: int):
    """1 where the joint check kept the match or its d0 agrees with the SGM
    disparity within tau."""
    hf, va, dp = _c(hyp_fwd, np.int16), _c(valid, np.uint8), _c(disp, np.int16)
    H, W, _ = hf.shape
    out = np.zeros((H, W), np.uint8)
    assert lib().orc_disparity_fill(_p(hf), _p(va), _p(dp), H, W, tau, _p(out)) == 0
    return out


def region_filter(hyp_fwd, valid, tau: int, s_c: int):
    """Region filter (Section 3.1, "Consistency Check", second step): keep
    uint8 [H][W] from the forward field [H][W][4] and the consistency mask."""
    hf = _c(hyp_fwd, np.int16)
    va = _c(valid, np.uint8)
    H, W, _ = hf.shape
    keep = np.zeros((H, W), np.uint8)
    assert lib().orc_region_filter(_p(hf), _p(va), H, W, tau, s_c, _p(keep)) == 0
    return keep


def sparsify(keep, err):
    """Sparsification (Section 3.2): per non-overlapping 3x3 block the index
    y*W + x of the surviving match with the lowest error (ties: lowest index),
    or -1; int32 [ceil(H/3)][ceil(W/3)]."""
    kp = _c(keep, np.uint8)
    er = _c(err, np.uint32)
    H, W = kp.shape
    seeds = np.zeros(((H + 2) // 3, (W + 2) // 3), np.int32)
    assert lib().orc_sparsify(_p(kp), _p(er), H, W, _p(seeds)) == 0
    return seeds


def match_level_scan(descs, level: int, s: int, seed: int, iters: int, rs_r0: int,
                     rs_samples: int, fmax: int, dmax: int, hyp0, cost0, hyp_coarse=None,
                     nthreads: int = 0):
    """One level with the paper's sequential four-corner schedule (CPU only)."""
    D = [_c(d, np.int16) for d in descs]
    H, W, C, _ = D[0].shape
    n = 1 << level
    Hk, Wk = -(-H // n), -(-W // n)
    hyp = np.zeros((Hk, Wk, 4), np.int16) if hyp0 is None else _c(hyp0, np.int16).copy()
    cost = np.zeros((Hk, Wk), np.uint32) if cost0 is None else _c(cost0, np.uint32).copy()
    hc = None if hyp_coarse is None else _c(hyp_coarse, np.int16)
    assert lib().orc_match_level_scan(*[_p(d) for d in D], H, W, C, level, s, seed, iters, rs_r0,
                                      rs_samples, fmax, dmax, None if hc is None else _p(hc),
                                      nthreads, _p(hyp), _p(cost)) == 0
    return hyp, cost


def match_pair(imgs, params: dict, seed: int, nthreads: int = 0, schedule: str = "red-black",
               leaves: int = 1):
    """Whole stage on one pair.  imgs: uint8 [4][H][W][C] (l0, l1, r0, r1).
    Returns dict with hyp [2][H][W][4] (forward, inverse), cost [2][H][W],
    valid [H][W], err [H][W]."""
    im = _c(imgs, np.uint8)
    _, H, W, C = im.shape
    hyp = np.zeros((2, H, W, 4), np.int16)
    cst = np.zeros((2, H, W), np.uint32)
    valid = np.zeros((H, W), np.uint8)
    err = np.zeros((H, W), np.uint32)
    p = params
    scan = {"red-black": 0, "scan": 1}[schedule]
    assert lib().orc_match_pair_schedule(_p(im), H, W, C, p["levels"], p["iters"], p["rs_r0"],
                                         p["rs_samples"], p["fmax"], p["dmax"], p["tau"], seed,
                                         nthreads, scan, leaves, _p(hyp), _p(cst), _p(valid),
                                         _p(err)) == 0
    return dict(hyp=hyp, cost=cst, valid=valid, err=err)


def cost_sift(phi, hyp, s: int = 1):
    """Eq. (1) with SIFT-PCA features phi [4][H][W][3 or 4] (rounded to float32),
    FP32 as the oracle's matcher computes it: float32 [H][W]."""
    ph = _phi4(phi)
    _, H, W, _ = ph.shape
    h = _c(hyp, np.int16)
    out = np.zeros((H, W), np.float32)
    assert lib().orc_cost_sift(_p(ph), H, W, s, _p(h), _p(out)) == 0
    return out


def match_sift(phi, hyp, s: int, seed: int, iters: int, rs_r0: int, rs_samples: int, fmax: int,
               dmax: int, order: int = 0, nthreads: int = 0):
    """Full-resolution propagation and random search with the SIFT-PCA cost
    from the field hyp [H][W][4]; returns (hyp, cost float32)."""
    ph = _phi4(phi)
    _, H, W, _ = ph.shape
    h = np.array(hyp, dtype=np.int16, copy=True, order="C")
    c = np.zeros((H, W), np.float32)
    assert lib().orc_match_sift(_p(ph), H, W, s, seed, iters, rs_r0, rs_samples, fmax, dmax, order,
                                nthreads, _p(h), _p(c)) == 0
    return h, c


def _phi4(phi):
    ph = np.asarray(phi)
    out = np.zeros(ph.shape[:3] + (4,), np.float32)
    out[..., :3] = ph[..., :3]
    return np.ascontiguousarray(out)
