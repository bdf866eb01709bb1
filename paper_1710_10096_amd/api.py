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


def sff_wht_workspace_bytes(p, nimg: int, level: int) -> int:
    pp = _params(p)
    return int(lib().sff_wht_workspace_bytes(ctypes.byref(pp), nimg, level))


def sff_wht_features(p, img: torch.Tensor, level: int, desc: torch.Tensor | None = None,
                     workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """img uint8 [n][H][W][C] -> desc int16 [n][H][W][C][16] at ``level``."""
    pp = _params(p)
    nimg = img.shape[0]
    if tuple(img.shape[1:]) != (pp.H, pp.W, pp.C):
        raise ValueError("img shape does not match params")
    if desc is None:
        desc = torch.empty((nimg, pp.H, pp.W, pp.C, 16), dtype=torch.int16, device=img.device)
    need = sff_wht_workspace_bytes(pp, nimg, level)
    if workspace is None and need > 0:
        workspace = torch.empty(need, dtype=torch.uint8, device=img.device)
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(lib().sff_wht_features(ctypes.byref(pp), nimg, level, _ptr(img, torch.uint8, "img"),
                                  _ptr(desc, torch.int16, "desc"), _ptr(workspace, None, "ws"),
                                  ws_bytes, _stream(stream)), "sff_wht_features")
    return desc


def _field(p, batch, ndir, level, device, hyp=None, cost=None):
    Hk, Wk = grid_shape(p, level)
    if hyp is None:
        hyp = torch.empty((ndir, batch, Hk, Wk, 4), dtype=torch.int16, device=device)
    if cost is None:
        cost = torch.empty((ndir, batch, Hk, Wk), dtype=torch.int32, device=device)
    return hyp, cost


def sff_init_workspace_bytes(p, batch: int) -> int:
    pp = _params(p)
    return int(lib().sff_init_workspace_bytes(ctypes.byref(pp), batch))


def sff_init_nn(p, desc: torch.Tensor, dir: int = DIR_BOTH, hyp=None, cost=None,
                workspace: torch.Tensor | None = None, stream=None):
    """desc int16 [batch][4][H][W][C][16] at the coarsest level -> (hyp, cost)."""
    pp = _params(p)
    batch = desc.shape[0]
    ndir = 2 if dir == DIR_BOTH else 1
    hyp, cost = _field(pp, batch, ndir, pp.levels - 1, desc.device, hyp, cost)
    if workspace is None:
        workspace = torch.empty(sff_init_workspace_bytes(pp, batch), dtype=torch.uint8,
                                device=desc.device)
    ws_bytes = workspace.numel() * workspace.element_size()
    _check(lib().sff_init_nn(ctypes.byref(pp), batch, dir, _ptr(desc, torch.int16, "desc"),
                             _ptr(hyp, torch.int16, "hyp"), _ptr(cost, torch.int32, "cost"),
                             _ptr(workspace, None, "workspace"), ws_bytes, _stream(stream)),
           "sff_init_nn")
    return hyp, cost


def sff_match_level(p, desc: torch.Tensor, dir: int, level: int, seeds: torch.Tensor,
                    hyp: torch.Tensor | None = None, cost: torch.Tensor | None = None,
                    hyp_coarse: torch.Tensor | None = None, stream=None):
    """One level of propagation + random search, in place on (hyp, cost)."""
    pp = _params(p)
    batch = desc.shape[0]
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
