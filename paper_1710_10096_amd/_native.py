"""ctypes loader for libsff.so (built in-tree by ``build.py``).

There is no fallback: if the HIP library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsff.so")


class SffParams(ctypes.Structure):
    """Mirror of ``sff_params`` in include/sff.h."""

    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("C", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("rs_r0", ctypes.c_int32), ("rs_samples", ctypes.c_int32),
                ("fmax", ctypes.c_int32), ("dmax", ctypes.c_int32), ("tau", ctypes.c_int32)]

    @classmethod
    def from_dict(cls, d: dict) -> "SffParams":
        return cls(**{k: int(d[k]) for k, _ in cls._fields_})

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


EXPORTS = ("sff_status_string", "sff_version", "sff_desc_channels", "sff_lanczos_q14", "sff_wht_workspace_bytes",
           "sff_wht_features", "sff_wht_scratch_bytes", "sff_wht_features_noalloc", "sff_bin_bytes", "sff_match_level_bins",
           "sff_init_workspace_bytes", "sff_init_nn", "sff_init_bins_workspace_bytes", "sff_init_nn_bins", "sff_init_nn_leaves", "sff_match_level",
           "sff_consistency", "sff_region_workspace_bytes", "sff_region_filter", "sff_sparsify",
           "sff_sgm_workspace_bytes", "sff_sgm_disparity", "sff_disparity_fill",
           "sff_sift_workspace_bytes", "sff_dense_sift", "sff_sift_pca", "sff_cost_sift",
           "sff_match_sift", "sff_sift_sqrt",
           "sff_cost_f32_fwd", "sff_cost_f32_bwd_workspace_bytes",
           "sff_cost_f32_bwd", "sff_conv3x3_bf16_fwd", "sff_featnet_fwd_bf16",
           "sff_conv3x3_bf16_bwd_workspace_bytes",
           "sff_conv3x3_bf16_dgrad", "sff_conv3x3_bf16_wgrad", "sff_smooth_level",
           "sff_quantise_features", "sff_triplet_loss", "sff_take_grad_bf16", "sff_probe_copy",
           "sff_probe_gather")

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1710_10096_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32 = ctypes.c_int32
    PP = ctypes.POINTER(SffParams)
    L.sff_status_string.argtypes = [i32]
    L.sff_status_string.restype = ctypes.c_char_p
    L.sff_version.argtypes = []
    L.sff_version.restype = i32
    L.sff_desc_channels.argtypes = [i32]
    L.sff_desc_channels.restype = i32
    L.sff_lanczos_q14.argtypes = [i32, P]
    L.sff_lanczos_q14.restype = i32
    L.sff_wht_workspace_bytes.argtypes = [PP, i32, i32]
    L.sff_wht_workspace_bytes.restype = ctypes.c_size_t
    L.sff_wht_features.argtypes = [PP, i32, i32, P, P, P, P, ctypes.c_size_t, P]
    L.sff_wht_features.restype = i32
    L.sff_wht_scratch_bytes.argtypes = []
    L.sff_wht_scratch_bytes.restype = ctypes.c_size_t
    L.sff_wht_features_noalloc.argtypes = [PP, i32, i32, P, P, P, P]
    L.sff_wht_features_noalloc.restype = i32
    L.sff_bin_bytes.argtypes = [PP, i32]
    L.sff_bin_bytes.restype = ctypes.c_size_t
    L.sff_match_level_bins.argtypes = [PP, i32, i32, i32, P, P, P, P, P, P]
    L.sff_match_level_bins.restype = i32
    L.sff_init_workspace_bytes.argtypes = [PP, i32]
    L.sff_init_workspace_bytes.restype = ctypes.c_size_t
    L.sff_init_nn.argtypes = [PP, i32, i32, P, P, P, P, ctypes.c_size_t, P]
    L.sff_init_nn.restype = i32
    L.sff_init_bins_workspace_bytes.argtypes = [PP, i32]
    L.sff_init_bins_workspace_bytes.restype = ctypes.c_size_t
    L.sff_init_nn_bins.argtypes = [PP, i32, i32, i32, P, P, P, P, ctypes.c_size_t, P]
    L.sff_init_nn_bins.restype = i32
    L.sff_init_nn_leaves.argtypes = [PP, i32, i32, i32, P, P, P, P, ctypes.c_size_t, P]
    L.sff_init_nn_leaves.restype = i32
    L.sff_match_level.argtypes = [PP, i32, i32, i32, P, P, P, P, P, P]
    L.sff_match_level.restype = i32
    L.sff_consistency.argtypes = [PP, i32, P, P, P, P, P]
    L.sff_consistency.restype = i32
    L.sff_region_workspace_bytes.argtypes = [PP, i32]
    L.sff_region_workspace_bytes.restype = ctypes.c_size_t
    L.sff_region_filter.argtypes = [PP, i32, i32, P, P, P, P, ctypes.c_size_t, P]
    L.sff_region_filter.restype = i32
    L.sff_sparsify.argtypes = [PP, i32, P, P, P, P]
    L.sff_sparsify.restype = i32
    L.sff_sgm_workspace_bytes.argtypes = [PP, i32]
    L.sff_sgm_workspace_bytes.restype = ctypes.c_size_t
    L.sff_sgm_disparity.argtypes = [PP, i32, P, P, ctypes.c_size_t, i32, i32, P, P,
                                    ctypes.c_size_t, P]
    L.sff_sgm_disparity.restype = i32
    L.sff_disparity_fill.argtypes = [PP, i32, P, P, P, P, P]
    L.sff_disparity_fill.restype = i32
    L.sff_sift_workspace_bytes.argtypes = [PP, i32]
    L.sff_sift_workspace_bytes.restype = ctypes.c_size_t
    L.sff_dense_sift.argtypes = [PP, i32, P, P, P, ctypes.c_size_t, P]
    L.sff_dense_sift.restype = i32
    L.sff_sift_pca.argtypes = [PP, i32, P, P, P, P, P, P, P, ctypes.c_size_t, P]
    L.sff_sift_pca.restype = i32
    L.sff_cost_sift.argtypes = [PP, i32, i32, P, P, P, P]
    L.sff_cost_sift.restype = i32
    L.sff_match_sift.argtypes = [PP, i32, i32, P, P, i32, P, P, P]
    L.sff_match_sift.restype = i32
    L.sff_sift_sqrt.argtypes = [P, P, ctypes.c_int64, P]
    L.sff_sift_sqrt.restype = i32
    L.sff_cost_f32_fwd.argtypes = [i32] * 5 + [P, P, P, P]
    L.sff_cost_f32_fwd.restype = i32
    L.sff_cost_f32_bwd_workspace_bytes.argtypes = [i32] * 3
    L.sff_cost_f32_bwd_workspace_bytes.restype = ctypes.c_size_t
    L.sff_cost_f32_bwd.argtypes = [i32] * 5 + [P, P, P, P, P, ctypes.c_size_t, P]
    L.sff_cost_f32_bwd.restype = i32
    L.sff_conv3x3_bf16_fwd.argtypes = [i32] * 7 + [P, P, P, P, P]
    L.sff_conv3x3_bf16_fwd.restype = i32
    L.sff_featnet_fwd_bf16.argtypes = [i32] * 4 + [P] * 11
    L.sff_featnet_fwd_bf16.restype = i32
    L.sff_conv3x3_bf16_bwd_workspace_bytes.argtypes = [i32] * 5
    L.sff_conv3x3_bf16_bwd_workspace_bytes.restype = ctypes.c_size_t
    L.sff_conv3x3_bf16_dgrad.argtypes = [i32] * 6 + [P, P, P, P, P, ctypes.c_size_t, P]
    L.sff_conv3x3_bf16_dgrad.restype = i32
    L.sff_conv3x3_bf16_wgrad.argtypes = [i32] * 6 + [P, P, P, P, P, P, ctypes.c_size_t, P]
    L.sff_conv3x3_bf16_wgrad.restype = i32
    L.sff_smooth_level.argtypes = [PP, i32, i32, P, P, P, ctypes.c_size_t, P]
    L.sff_smooth_level.restype = i32
    L.sff_quantise_features.argtypes = [i32, i32, i32, P, ctypes.c_float, P, P]
    L.sff_quantise_features.restype = i32
    L.sff_triplet_loss.argtypes = [i32, P, i32, P, ctypes.c_float, ctypes.c_float, P, P, P]
    L.sff_triplet_loss.restype = i32
    L.sff_take_grad_bf16.argtypes = [ctypes.c_size_t, P, P, P]
    L.sff_take_grad_bf16.restype = i32
    L.sff_probe_copy.argtypes = [P, P, ctypes.c_size_t, P]
    L.sff_probe_copy.restype = i32
    L.sff_probe_gather.argtypes = [P, ctypes.c_size_t, i32, i32, i32, ctypes.c_uint64, i32, P, P]
    L.sff_probe_gather.restype = i32
    _lib = L
    return L
