"""Thin Python binding of libsff: the C entry points under the same names,
taking torch tensors that live on the GPU.  Argument marshalling only -- every
step of the matching stage runs in the HIP kernels behind the C ABI.

dtype conventions: uint32 arrays of the ABI (cost, err) are carried in
``torch.int32`` tensors with the same bits; uint64 seeds in ``torch.int64``.
"""
from __future__ import annotations

import ctypes

import torch

from ._native import SffParams, lib

DIR_FORWARD, DIR_INVERSE, DIR_BOTH = 1, -1, 0


class SffError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = int(code)
        msg = lib().sff_status_string(self.code).decode()
        super().__init__(f"{where}: {msg} (status {self.code})")


def _check(code: int, where: str):
    if code != 0:
        raise SffError(code, where)


def _params(p) -> SffParams:
    return p if isinstance(p, SffParams) else SffParams.from_dict(p)


def _ptr(t: torch.Tensor | None, dtype=None, name: str = "tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def grid_shape(p, level: int):
    p = _params(p)
    n = 1 << level
    return (p.H + n - 1) // n, (p.W + n - 1) // n


def sff_version() -> int:
    return int(lib().sff_version())


def sff_lanczos_q14(n: int):
    """Host helper: Q14 Lanczos-3 weights [n][6] as nested lists."""
    buf = (ctypes.c_int32 * (n * 6))()
    _check(lib().sff_lanczos_q14(n, ctypes.cast(buf, ctypes.c_void_p)), "sff_lanczos_q14")
    return [[buf[p * 6 + t] for t in range(6)] for p in range(n)]


def desc_channels(C: int) -> int:
    """Channels of a stored descriptor record (records are padded to 32, 64
    or 128 bytes): 1, 2, 4, 4 for C = 1..4."""
    cp = int(lib().sff_desc_channels(int(C)))
    if cp == 0:
        raise ValueError(f"C must be 1..4, got {C}")
    return cp


def _check_shape(t: torch.Tensor, shape, name: str):
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


def sff_wht_workspace_bytes(p, nimg: int, level: int) -> int:
    pp = _params(p)
    return int(lib().sff_wht_workspace_bytes(ctypes.byref(pp), nimg, level))


def sff_bin_bytes(p, level: int) -> int:
    """Bytes of one image's WHT bin-sum planes at ``level``."""
    return int(lib().sff_bin_bytes(ctypes.byref(_params(p)), level))


def sff_wht_features(p, img: torch.Tensor, level: int, desc: torch.Tensor | None = None,
                     workspace: torch.Tensor | None = None, stream=None, *, bins=None,
                     want_desc: bool = True) -> torch.Tensor:
    """img uint8 [n][H][W][C] -> desc int16 [n][H][W][Cp][16] at ``level``
    (Cp = desc_channels(C); channels C..Cp-1 are left as they are, zero for a
    descriptor tensor allocated here).  ``bins``, if given (uint8 or int16
    tensor of n * sff_bin_bytes bytes), also receives the bin-sum planes; with
    want_desc=False only the planes are computed and they are returned."""
    pp = _params(p)
    nimg = img.shape[0]
    if tuple(img.shape[1:]) != (pp.H, pp.W, pp.C):
        raise ValueError("img shape does not match params")
    shape = (nimg, pp.H, pp.W, desc_channels(pp.C), 16)
    if want_desc:
        if desc is None:
            desc = torch.zeros(shape, dtype=torch.int16, device=img.device)
        _check_shape(desc, shape, "desc")
    else:
        desc = None
        if bins is None:
            bins = torch.empty(nimg * sff_bin_bytes(pp, level), dtype=torch.uint8, device=img.device)
    if bins is not None:
        if not bins.is_contiguous() or bins.numel() * bins.element_size() < nimg * sff_bin_bytes(pp, level):
            raise ValueError("bins too small or not contiguous")
    need = sff_wht_workspace_bytes(pp, nimg, level)
    if workspace is None and need > 0:
        workspace = torch.empty(need, dtype=torch.uint8, device=img.device)
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(lib().sff_wht_features(ctypes.byref(pp), nimg, level, _ptr(img, torch.uint8, "img"),
                                  _ptr(desc, torch.int16, "desc"), _ptr(bins, None, "bins"),
                                  _ptr(workspace, None, "ws"), ws_bytes, _stream(stream)),
           "sff_wht_features")
    return desc if want_desc else bins


def _field(p, batch, ndir, level, device, hyp=None, cost=None):
    Hk, Wk = grid_shape(p, level)
    if hyp is None:
        hyp = torch.empty((ndir, batch, Hk, Wk, 4), dtype=torch.int16, device=device)
    if cost is None:
        cost = torch.empty((ndir, batch, Hk, Wk), dtype=torch.int32, device=device)
    _check_shape(hyp, (ndir, batch, Hk, Wk, 4), "hyp")
    _check_shape(cost, (ndir, batch, Hk, Wk), "cost")
    return hyp, cost


def _check_pair_desc(pp, desc: torch.Tensor):
    _check_shape(desc, (desc.shape[0], 4, pp.H, pp.W, desc_channels(pp.C), 16), "desc")


def sff_init_workspace_bytes(p, batch: int) -> int:
    pp = _params(p)
    return int(lib().sff_init_workspace_bytes(ctypes.byref(pp), batch))


def sff_init_nn(p, desc: torch.Tensor, dir: int = DIR_BOTH, hyp=None, cost=None,
                workspace: torch.Tensor | None = None, stream=None, leaves: int = 1):
    """desc int16 [batch][4][H][W][Cp][16] at the coarsest level -> (hyp, cost).
    ``leaves`` (1, 2, 4): temporal leaves whose combinations are compared."""
    pp = _params(p)
    _check_pair_desc(pp, desc)
    batch = desc.shape[0]
    ndir = 2 if dir == DIR_BOTH else 1
    hyp, cost = _field(pp, batch, ndir, pp.levels - 1, desc.device, hyp, cost)
    if workspace is None:
        workspace = torch.empty(sff_init_workspace_bytes(pp, batch), dtype=torch.uint8,
                                device=desc.device)
    ws_bytes = workspace.numel() * workspace.element_size()
    _check(lib().sff_init_nn_leaves(ctypes.byref(pp), batch, dir, int(leaves),
                                    _ptr(desc, torch.int16, "desc"), _ptr(hyp, torch.int16, "hyp"),
                                    _ptr(cost, torch.int32, "cost"),
                                    _ptr(workspace, None, "workspace"), ws_bytes, _stream(stream)),
           "sff_init_nn")
    return hyp, cost


def sff_init_bins_workspace_bytes(p, batch: int) -> int:
    return int(lib().sff_init_bins_workspace_bytes(ctypes.byref(_params(p)), batch))


def sff_init_nn_bins(p, bins: torch.Tensor, batch: int, dir: int = DIR_BOTH, hyp=None, cost=None,
                     workspace=None, stream=None, leaves: int = 1):
    """Exact-NN initialisation at the coarsest level from its bin-sum planes
    (``bins``: the 4 views of ``batch`` pairs); same results as sff_init_nn on
    the level's descriptors."""
    pp = _params(p)
    top = pp.levels - 1
    if not bins.is_contiguous() or bins.numel() * bins.element_size() < 4 * batch * sff_bin_bytes(pp, top):
        raise ValueError("bins too small or not contiguous")
    ndir = 2 if dir == DIR_BOTH else 1
    hyp, cost = _field(pp, batch, ndir, top, bins.device, hyp, cost)
    need = sff_init_bins_workspace_bytes(pp, batch)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=bins.device)
    ws_bytes = workspace.numel() * workspace.element_size()
    _check(lib().sff_init_nn_bins(ctypes.byref(pp), batch, dir, int(leaves), _ptr(bins, None, "bins"),
                                  _ptr(hyp, torch.int16, "hyp"), _ptr(cost, torch.int32, "cost"),
                                  _ptr(workspace, None, "ws"), ws_bytes, _stream(stream)),
           "sff_init_nn_bins")
    return hyp, cost


def sff_match_level(p, desc: torch.Tensor, dir: int, level: int, seeds: torch.Tensor,
                    hyp: torch.Tensor | None = None, cost: torch.Tensor | None = None,
                    hyp_coarse: torch.Tensor | None = None, stream=None):
    """One level of propagation + random search, in place on (hyp, cost);
    desc int16 [batch][4][H][W][Cp][16] at ``level``."""
    pp = _params(p)
    _check_pair_desc(pp, desc)
    batch = desc.shape[0]
    if seeds.numel() != batch:
        raise ValueError("seeds must hold one value per pair")
    if hyp_coarse is not None:
        Hc, Wc = grid_shape(pp, level + 1)
        _check_shape(hyp_coarse, (2 if dir == DIR_BOTH else 1, batch, Hc, Wc, 4), "hyp_coarse")
    ndir = 2 if dir == DIR_BOTH else 1
    if hyp_coarse is None and (hyp is None or cost is None):
        raise ValueError("without hyp_coarse the starting field (hyp, cost) is required")
    hyp, cost = _field(pp, batch, ndir, level, desc.device, hyp, cost)
    _check(lib().sff_match_level(ctypes.byref(pp), batch, dir, level,
                                 _ptr(desc, torch.int16, "desc"),
                                 _ptr(seeds, torch.int64, "seeds"),
                                 _ptr(hyp_coarse, torch.int16, "hyp_coarse"),
                                 _ptr(hyp, torch.int16, "hyp"), _ptr(cost, torch.int32, "cost"),
                                 _stream(stream)), "sff_match_level")
    return hyp, cost


def sff_match_level_bins(p, bins: torch.Tensor, dir: int, level: int, seeds: torch.Tensor,
                         hyp: torch.Tensor | None = None, cost: torch.Tensor | None = None,
                         hyp_coarse: torch.Tensor | None = None, stream=None):
    """One level of propagation + random search with the WHT descriptor
    distances taken from the bin-sum planes, in place on (hyp, cost); bins
    holds the level's planes of the 4 views of ``seeds.numel()`` pairs."""
    pp = _params(p)
    batch = seeds.numel()
    if not bins.is_contiguous() or bins.numel() * bins.element_size() < 4 * batch * sff_bin_bytes(pp, level):
        raise ValueError("bins too small or not contiguous")
    if hyp_coarse is not None:
        Hc, Wc = grid_shape(pp, level + 1)
        _check_shape(hyp_coarse, (2 if dir == DIR_BOTH else 1, batch, Hc, Wc, 4), "hyp_coarse")
    ndir = 2 if dir == DIR_BOTH else 1
    if hyp_coarse is None and (hyp is None or cost is None):
        raise ValueError("without hyp_coarse the starting field (hyp, cost) is required")
    hyp, cost = _field(pp, batch, ndir, level, bins.device, hyp, cost)
    _check(lib().sff_match_level_bins(ctypes.byref(pp), batch, dir, level, _ptr(bins, None, "bins"),
                                      _ptr(seeds, torch.int64, "seeds"),
                                      _ptr(hyp_coarse, torch.int16, "hyp_coarse"),
                                      _ptr(hyp, torch.int16, "hyp"), _ptr(cost, torch.int32, "cost"),
                                      _stream(stream)), "sff_match_level_bins")
    return hyp, cost


def sff_consistency(p, hyp_fwd: torch.Tensor, hyp_inv: torch.Tensor, valid=None, err=None,
                    stream=None):
    """Level-0 fields [batch][H][W][4] -> (valid uint8 [batch][H][W], err int32-bits)."""
    pp = _params(p)
    batch = hyp_fwd.shape[0]
    if valid is None:
        valid = torch.empty((batch, pp.H, pp.W), dtype=torch.uint8, device=hyp_fwd.device)
    if err is None:
        err = torch.empty((batch, pp.H, pp.W), dtype=torch.int32, device=hyp_fwd.device)
    _check(lib().sff_consistency(ctypes.byref(pp), batch, _ptr(hyp_fwd, torch.int16, "hyp_fwd"),
                                 _ptr(hyp_inv, torch.int16, "hyp_inv"),
                                 _ptr(valid, torch.uint8, "valid"), _ptr(err, torch.int32, "err"),
                                 _stream(stream)), "sff_consistency")
    return valid, err


def sff_region_workspace_bytes(p, batch: int) -> int:
    pp = _params(p)
    return int(lib().sff_region_workspace_bytes(ctypes.byref(pp), batch))


def sff_region_filter(p, hyp_fwd: torch.Tensor, valid: torch.Tensor, s_c: int = 150, keep=None,
                      workspace=None, stream=None) -> torch.Tensor:
    """Region filter: level-0 forward field [batch][H][W][4] and consistency
    mask [batch][H][W] -> keep uint8 [batch][H][W] (tau of the params is the
    vector similarity threshold, s_c the minimal region size)."""
    pp = _params(p)
    batch = hyp_fwd.shape[0]
    _check_shape(hyp_fwd, (batch, pp.H, pp.W, 4), "hyp_fwd")
    _check_shape(valid, (batch, pp.H, pp.W), "valid")
    if keep is None:
        keep = torch.empty((batch, pp.H, pp.W), dtype=torch.uint8, device=hyp_fwd.device)
    _check_shape(keep, (batch, pp.H, pp.W), "keep")
    if workspace is None:
        workspace = torch.empty(sff_region_workspace_bytes(pp, batch), dtype=torch.uint8,
                                device=hyp_fwd.device)
    ws_bytes = workspace.numel() * workspace.element_size()
    _check(lib().sff_region_filter(ctypes.byref(pp), batch, int(s_c),
                                   _ptr(hyp_fwd, torch.int16, "hyp_fwd"),
                                   _ptr(valid, torch.uint8, "valid"), _ptr(keep, torch.uint8, "keep"),
                                   _ptr(workspace, None, "workspace"), ws_bytes, _stream(stream)),
           "sff_region_filter")
    return keep


def sff_sparsify(p, keep: torch.Tensor, err: torch.Tensor, seeds=None, stream=None) -> torch.Tensor:
    """Best match per 3x3 block: keep uint8 and err (uint32 bits in int32)
    [batch][H][W] -> seeds int32 [batch][ceil(H/3)][ceil(W/3)] (index or -1)."""
    pp = _params(p)
    batch = keep.shape[0]
    _check_shape(keep, (batch, pp.H, pp.W), "keep")
    _check_shape(err, (batch, pp.H, pp.W), "err")
    shape = (batch, (pp.H + 2) // 3, (pp.W + 2) // 3)
    if seeds is None:
        seeds = torch.empty(shape, dtype=torch.int32, device=keep.device)
    _check_shape(seeds, shape, "seeds")
    _check(lib().sff_sparsify(ctypes.byref(pp), batch, _ptr(keep, torch.uint8, "keep"),
                              _ptr(err, torch.int32, "err"), _ptr(seeds, torch.int32, "seeds"),
                              _stream(stream)), "sff_sparsify")
    return seeds


SGM_P1, SGM_P2 = 3, 24  # census 5x5 (costs 0..24)


def sff_sgm_workspace_bytes(p, batch: int) -> int:
    pp = _params(p)
    return int(lib().sff_sgm_workspace_bytes(ctypes.byref(pp), batch))


def sff_sgm_disparity(p, left: torch.Tensor, right: torch.Tensor, P1: int = SGM_P1,
                      P2: int = SGM_P2, disp=None, workspace=None, stream=None) -> torch.Tensor:
    """SGM disparity of rectified pairs: left/right uint8 views [batch][H][W][C]
    (may be strided along the batch, e.g. imgs[:, 0] and imgs[:, 2] of a
    [batch][4][H][W][C] tensor) -> int16 [batch][H][W] in 0..dmax."""
    pp = _params(p)
    batch = left.shape[0]
    for t, nm in ((left, "left"), (right, "right")):
        _check_shape(t, (batch, pp.H, pp.W, pp.C), nm)
        if not t.is_cuda or t.dtype != torch.uint8 or not t[0].is_contiguous():
            raise ValueError(f"{nm} must be GPU uint8 with contiguous images")
    if left.stride(0) != right.stride(0):
        raise ValueError("left and right must have the same batch stride")
    if disp is None:
        disp = torch.empty((batch, pp.H, pp.W), dtype=torch.int16, device=left.device)
    _check_shape(disp, (batch, pp.H, pp.W), "disp")
    if workspace is None:
        workspace = torch.empty(sff_sgm_workspace_bytes(pp, batch), dtype=torch.uint8,
                                device=left.device)
    ws_bytes = workspace.numel() * workspace.element_size()
    _check(lib().sff_sgm_disparity(ctypes.byref(pp), batch, ctypes.c_void_p(left.data_ptr()),
                                   ctypes.c_void_p(right.data_ptr()), left.stride(0), int(P1),
                                   int(P2), _ptr(disp, torch.int16, "disp"),
                                   _ptr(workspace, None, "workspace"), ws_bytes, _stream(stream)),
           "sff_sgm_disparity")
    return disp


def sff_disparity_fill(p, hyp_fwd: torch.Tensor, valid: torch.Tensor, disp: torch.Tensor,
                       fill=None, stream=None) -> torch.Tensor:
    """1 where the joint check kept the match or its d0 agrees with the SGM
    disparity within tau: uint8 [batch][H][W]."""
    pp = _params(p)
    batch = hyp_fwd.shape[0]
    _check_shape(hyp_fwd, (batch, pp.H, pp.W, 4), "hyp_fwd")
    _check_shape(valid, (batch, pp.H, pp.W), "valid")
    _check_shape(disp, (batch, pp.H, pp.W), "disp")
    if fill is None:
        fill = torch.empty((batch, pp.H, pp.W), dtype=torch.uint8, device=hyp_fwd.device)
    _check_shape(fill, (batch, pp.H, pp.W), "fill")
    _check(lib().sff_disparity_fill(ctypes.byref(pp), batch, _ptr(hyp_fwd, torch.int16, "hyp_fwd"),
                                    _ptr(valid, torch.uint8, "valid"), _ptr(disp, torch.int16, "disp"),
                                    _ptr(fill, torch.uint8, "fill"), _stream(stream)),
           "sff_disparity_fill")
    return fill


def sff_sift_workspace_bytes(p, nimg: int) -> int:
    pp = _params(p)
    return int(lib().sff_sift_workspace_bytes(ctypes.byref(pp), nimg))


def sff_dense_sift(p, img: torch.Tensor, sift=None, workspace=None, stream=None) -> torch.Tensor:
    """Dense SIFT of uint8 images [nimg][H][W][C] -> float32 [nimg][H][W][128]."""
    pp = _params(p)
    nimg = img.shape[0]
    _check_shape(img, (nimg, pp.H, pp.W, pp.C), "img")
    if sift is None:
        sift = torch.empty((nimg, pp.H, pp.W, 128), dtype=torch.float32, device=img.device)
    _check_shape(sift, (nimg, pp.H, pp.W, 128), "sift")
    if workspace is None:
        workspace = torch.empty(sff_sift_workspace_bytes(pp, nimg), dtype=torch.uint8, device=img.device)
    ws_bytes = workspace.numel() * workspace.element_size()
    _check(lib().sff_dense_sift(ctypes.byref(pp), nimg, _ptr(img, torch.uint8, "img"),
                                _ptr(sift, torch.float32, "sift"), _ptr(workspace, None, "workspace"),
                                ws_bytes, _stream(stream)), "sff_dense_sift")
    return sift


def sff_sift_pca(p, imgs: torch.Tensor, out=None, workspace=None, stream=None) -> dict:
    """SIFT-PCA features of eq. (1) for pairs imgs uint8 [batch][4][H][W][C]:
    dict of mean [batch][128], cov [batch][128][128], eigval [batch][3],
    axes [batch][3][128] (float64) and phi float32 [batch][4][H][W][4]."""
    pp = _params(p)
    batch = imgs.shape[0]
    _check_shape(imgs, (batch, 4, pp.H, pp.W, pp.C), "imgs")
    dev = imgs.device
    if out is None:
        f64 = dict(dtype=torch.float64, device=dev)
        out = {"mean": torch.empty((batch, 128), **f64), "cov": torch.empty((batch, 128, 128), **f64),
               "eigval": torch.empty((batch, 3), **f64), "axes": torch.empty((batch, 3, 128), **f64),
               "phi": torch.empty((batch, 4, pp.H, pp.W, 4), dtype=torch.float32, device=dev)}
    for k, shp in (("mean", (batch, 128)), ("cov", (batch, 128, 128)), ("eigval", (batch, 3)),
                   ("axes", (batch, 3, 128)), ("phi", (batch, 4, pp.H, pp.W, 4))):
        _check_shape(out[k], shp, k)
    if workspace is None:
        workspace = torch.empty(sff_sift_workspace_bytes(pp, 4 * batch), dtype=torch.uint8, device=dev)
    ws_bytes = workspace.numel() * workspace.element_size()
    _check(lib().sff_sift_pca(ctypes.byref(pp), batch, _ptr(imgs, torch.uint8, "imgs"),
                              _ptr(out["mean"], torch.float64, "mean"), _ptr(out["cov"], torch.float64, "cov"),
                              _ptr(out["eigval"], torch.float64, "eigval"),
                              _ptr(out["axes"], torch.float64, "axes"), _ptr(out["phi"], torch.float32, "phi"),
                              _ptr(workspace, None, "workspace"), ws_bytes, _stream(stream)), "sff_sift_pca")
    return out


def sff_cost_sift(p, phi: torch.Tensor, hyp: torch.Tensor, dir: int = DIR_FORWARD, cost=None,
                  stream=None) -> torch.Tensor:
    """Eq. (1) with SIFT-PCA features: phi float32 [batch][4][H][W][4], hyp int16
    [batch][H][W][4] -> float32 [batch][H][W]."""
    pp = _params(p)
    batch = phi.shape[0]
    _check_shape(phi, (batch, 4, pp.H, pp.W, 4), "phi")
    _check_shape(hyp, (batch, pp.H, pp.W, 4), "hyp")
    if cost is None:
        cost = torch.empty((batch, pp.H, pp.W), dtype=torch.float32, device=phi.device)
    _check_shape(cost, (batch, pp.H, pp.W), "cost")
    _check(lib().sff_cost_sift(ctypes.byref(pp), batch, int(dir), _ptr(phi, torch.float32, "phi"),
                               _ptr(hyp, torch.int16, "hyp"), _ptr(cost, torch.float32, "cost"),
                               _stream(stream)), "sff_cost_sift")
    return cost


def sff_match_sift(p, phi: torch.Tensor, seeds: torch.Tensor, hyp: torch.Tensor, dir: int = DIR_BOTH,
                   iters: int | None = None, cost=None, stream=None) -> torch.Tensor:
    """Full-resolution propagation and random search with the SIFT-PCA cost of
    eq. (1), in place on hyp int16 [ndir][batch][H][W][4] (the starting field);
    returns cost float32 [ndir][batch][H][W]."""
    pp = _params(p)
    batch = phi.shape[0]
    ndir = 2 if dir == DIR_BOTH else 1
    _check_shape(phi, (batch, 4, pp.H, pp.W, 4), "phi")
    _check_shape(hyp, (ndir, batch, pp.H, pp.W, 4), "hyp")
    _check_shape(seeds, (batch,), "seeds")
    if cost is None:
        cost = torch.empty((ndir, batch, pp.H, pp.W), dtype=torch.float32, device=phi.device)
    _check_shape(cost, (ndir, batch, pp.H, pp.W), "cost")
    it = pp.iters if iters is None else int(iters)
    _check(lib().sff_match_sift(ctypes.byref(pp), batch, int(dir), _ptr(phi, torch.float32, "phi"),
                                _ptr(seeds, torch.int64, "seeds"), it, _ptr(hyp, torch.int16, "hyp"),
                                _ptr(cost, torch.float32, "cost"), _stream(stream)), "sff_match_sift")
    return cost


def sff_sift_sqrt(x: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """The SIFT-PCA cost's correctly rounded square root of every element of
    x (float32, finite, >= 0, contiguous on the device)."""
    n = x.numel()
    if out is None:
        out = torch.empty_like(x)
    _check_shape(out, tuple(x.shape), "out")
    _check(lib().sff_sift_sqrt(_ptr(x, torch.float32, "x"), _ptr(out, torch.float32, "out"), n, _stream(stream)),
           "sff_sift_sqrt")
    return out


def sff_cost_f32_fwd(feat: torch.Tensor, hyp: torch.Tensor, dir: int, cost=None, stream=None):
    """feat float32 [batch][4][H][W][cf], hyp int16 [batch][H][W][4] -> cost [batch][H][W]."""
    B, four, H, W, cf = feat.shape
    if four != 4 or tuple(hyp.shape) != (B, H, W, 4):
        raise ValueError("feat must be [batch][4][H][W][cf] and hyp [batch][H][W][4]")
    if cost is None:
        cost = torch.empty((B, H, W), dtype=torch.float32, device=feat.device)
    _check(lib().sff_cost_f32_fwd(B, H, W, cf, dir, _ptr(feat, torch.float32, "feat"),
                                  _ptr(hyp, torch.int16, "hyp"), _ptr(cost, torch.float32, "cost"),
                                  _stream(stream)), "sff_cost_f32_fwd")
    return cost


def sff_cost_f32_bwd_workspace_bytes(batch: int, H: int, W: int) -> int:
    return int(lib().sff_cost_f32_bwd_workspace_bytes(batch, H, W))


def sff_cost_f32_bwd(feat: torch.Tensor, hyp: torch.Tensor, dir: int, grad_cost: torch.Tensor,
                     grad_feat=None, workspace=None, stream=None):
    """Gradient of sum(grad_cost * cost) w.r.t. feat (all four maps)."""
    B, four, H, W, cf = feat.shape
    if grad_feat is None:
        grad_feat = torch.empty_like(feat)
    if workspace is None:
        workspace = torch.empty(sff_cost_f32_bwd_workspace_bytes(B, H, W), dtype=torch.uint8,
                                device=feat.device)
    ws_bytes = workspace.numel() * workspace.element_size()
    _check(lib().sff_cost_f32_bwd(B, H, W, cf, dir, _ptr(feat, torch.float32, "feat"),
                                  _ptr(hyp, torch.int16, "hyp"),
                                  _ptr(grad_cost, torch.float32, "grad_cost"),
                                  _ptr(grad_feat, torch.float32, "grad_feat"),
                                  _ptr(workspace, None, "workspace"), ws_bytes, _stream(stream)),
           "sff_cost_f32_bwd")
    return grad_feat


class MatchCost(torch.autograd.Function):
    """Per-pixel window cost of eq. (1) at fixed vectors, differentiable with
    respect to the four FP32 feature maps (forward and backward are libsff
    kernels)."""

    @staticmethod
    def forward(ctx, feat: torch.Tensor, hyp: torch.Tensor, dir: int = DIR_FORWARD):
        feat = feat.contiguous()
        ctx.save_for_backward(feat, hyp)
        ctx.dir = dir
        return sff_cost_f32_fwd(feat, hyp, dir)

    @staticmethod
    def backward(ctx, grad_cost):
        feat, hyp = ctx.saved_tensors
        g = sff_cost_f32_bwd(feat, hyp, ctx.dir, grad_cost.contiguous().float())
        return g, None, None


def sff_conv3x3_bf16_fwd(x: torch.Tensor, w: torch.Tensor, bias: torch.Tensor | None, dil: int = 1,
                         relu: bool = False, y=None, stream=None):
    """x bf16 [n][H][W][cin], w bf16 [cout][3][3][cin], bias f32 [cout] -> y bf16."""
    n, H, W, cin = x.shape
    cout = w.shape[0]
    if y is None:
        y = torch.empty((n, H, W, cout), dtype=torch.bfloat16, device=x.device)
    _check(lib().sff_conv3x3_bf16_fwd(n, H, W, cin, cout, dil, int(bool(relu)),
                                      _ptr(x, torch.bfloat16, "x"), _ptr(w, torch.bfloat16, "w"),
                                      _ptr(bias, torch.float32, "bias"),
                                      _ptr(y, torch.bfloat16, "y"), _stream(stream)),
           "sff_conv3x3_bf16_fwd")
    return y


def sff_featnet_fwd_bf16(x: torch.Tensor, ws, bs, dil: int = 1, y=None, stream=None):
    """The four-layer network in one launch: x bf16 [n][H][W][3], ws four bf16
    weight tensors ([32][3][3][3], then [32][3][3][32]), bs four f32 biases (or
    None) -> y bf16 [n][H][W][32]."""
    n, H, W, cin = x.shape
    if cin != 3 or len(ws) != 4 or len(bs) != 4:
        raise ValueError("x must have 3 channels; four weights and four biases")
    if y is None:
        y = torch.empty((n, H, W, 32), dtype=torch.bfloat16, device=x.device)
    args = []
    for w, b in zip(ws, bs):
        args += [_ptr(w, torch.bfloat16, "w"), _ptr(b, torch.float32, "bias")]
    _check(lib().sff_featnet_fwd_bf16(n, H, W, dil, _ptr(x, torch.bfloat16, "x"), *args,
                                      _ptr(y, torch.bfloat16, "y"), _stream(stream)),
           "sff_featnet_fwd_bf16")
    return y


def _conv_ws(n, H, W, cin, cout, device, workspace):
    if workspace is not None:
        return workspace
    nb = int(lib().sff_conv3x3_bf16_bwd_workspace_bytes(n, H, W, cin, cout))
    return torch.empty(max(nb, 256), dtype=torch.uint8, device=device)


def sff_conv3x3_bf16_dgrad(dy: torch.Tensor, w: torch.Tensor, dil: int = 1,
                           relu_out: torch.Tensor | None = None, dx=None, workspace=None,
                           stream=None):
    n, H, W, cout = dy.shape
    cin = w.shape[3]
    if dx is None:
        dx = torch.empty((n, H, W, cin), dtype=torch.bfloat16, device=dy.device)
    ws = _conv_ws(n, H, W, cin, cout, dy.device, workspace)
    _check(lib().sff_conv3x3_bf16_dgrad(n, H, W, cin, cout, dil, _ptr(dy, torch.bfloat16, "dy"),
                                        _ptr(relu_out, torch.bfloat16, "relu_out"),
                                        _ptr(w, torch.bfloat16, "w"), _ptr(dx, torch.bfloat16, "dx"),
                                        _ptr(ws, None, "ws"), ws.numel(), _stream(stream)),
           "sff_conv3x3_bf16_dgrad")
    return dx


def sff_conv3x3_bf16_wgrad(x: torch.Tensor, dy: torch.Tensor, dil: int = 1,
                           relu_out: torch.Tensor | None = None, dw=None, db=None, workspace=None,
                           stream=None):
    n, H, W, cin = x.shape
    cout = dy.shape[3]
    if dw is None:
        dw = torch.empty((cout, 3, 3, cin), dtype=torch.float32, device=x.device)
    if db is None:
        db = torch.empty((cout,), dtype=torch.float32, device=x.device)
    ws = _conv_ws(n, H, W, cin, cout, x.device, workspace)
    _check(lib().sff_conv3x3_bf16_wgrad(n, H, W, cin, cout, dil, _ptr(x, torch.bfloat16, "x"),
                                        _ptr(dy, torch.bfloat16, "dy"),
                                        _ptr(relu_out, torch.bfloat16, "relu_out"),
                                        _ptr(dw, torch.float32, "dw"), _ptr(db, torch.float32, "db"),
                                        _ptr(ws, None, "ws"), ws.numel(), _stream(stream)),
           "sff_conv3x3_bf16_wgrad")
    return dw, db


def sff_smooth_level(p, img: torch.Tensor, level: int, out=None, workspace=None, stream=None):
    """The level-k smoothed images, uint8 [n][H][W][C]."""
    pp = _params(p)
    nimg = img.shape[0]
    if out is None:
        out = torch.empty_like(img)
    need = sff_wht_workspace_bytes(pp, nimg, level)
    if workspace is None and need > 0:
        workspace = torch.empty(need, dtype=torch.uint8, device=img.device)
    ws_bytes = 0 if workspace is None else workspace.numel()
    _check(lib().sff_smooth_level(ctypes.byref(pp), nimg, level, _ptr(img, torch.uint8, "img"),
                                  _ptr(out, torch.uint8, "out"), _ptr(workspace, None, "ws"),
                                  ws_bytes, _stream(stream)), "sff_smooth_level")
    return out


def sff_quantise_features(feat: torch.Tensor, scale: float = 4096.0, desc=None, stream=None):
    """bf16 [n][H][W][32] -> int16 descriptors [n][H][W][2][16] (C = 2 records)."""
    n, H, W, F = feat.shape
    if F != 32:
        raise ValueError("features must have 32 channels")
    if desc is None:
        desc = torch.empty((n, H, W, 2, 16), dtype=torch.int16, device=feat.device)
    _check(lib().sff_quantise_features(n, H, W, _ptr(feat, torch.bfloat16, "feat"), float(scale),
                                       _ptr(desc, torch.int16, "desc"), _stream(stream)),
           "sff_quantise_features")
    return desc


def sff_triplet_loss(feat: torch.Tensor, triplets: torch.Tensor, margin: float, grad: torch.Tensor,
                     weight: float = 1.0, loss=None, stream=None):
    """feat bf16 [..][32] (pixels flattened), triplets int32 [T][3] -> loss [T]; adds
    weight * dloss/dfeat into grad (float32, same pixel count)."""
    npx = feat.numel() // 32
    T = triplets.shape[0]
    if loss is None:
        loss = torch.empty((T,), dtype=torch.float32, device=feat.device)
    _check(lib().sff_triplet_loss(npx, _ptr(feat, torch.bfloat16, "feat"), T,
                                  _ptr(triplets, torch.int32, "triplets"), float(margin),
                                  float(weight), _ptr(loss, torch.float32, "loss"),
                                  _ptr(grad, torch.float32, "grad"), _stream(stream)),
           "sff_triplet_loss")
    return loss


def sff_take_grad_bf16(grad: torch.Tensor, out=None, stream=None):
    if out is None:
        out = torch.empty(grad.shape, dtype=torch.bfloat16, device=grad.device)
    _check(lib().sff_take_grad_bf16(grad.numel(), _ptr(grad, torch.float32, "grad"),
                                    _ptr(out, torch.bfloat16, "out"), _stream(stream)),
           "sff_take_grad_bf16")
    return out


def sff_probe_copy(src: torch.Tensor, dst: torch.Tensor, stream=None):
    nb = src.numel() * src.element_size()
    _check(lib().sff_probe_copy(_ptr(src), _ptr(dst), nb, _stream(stream)), "sff_probe_copy")


def sff_probe_gather(buf: torch.Tensor, record_bytes: int, threads: int, per_thread: int,
                     out: torch.Tensor, seed: int = 1, coop: bool = False, stream=None):
    nb = buf.numel() * buf.element_size()
    _check(lib().sff_probe_gather(_ptr(buf), nb, record_bytes, threads, per_thread, seed,
                                  int(bool(coop)),
                                  _ptr(out, torch.int32, "out"), _stream(stream)),
           "sff_probe_gather")
