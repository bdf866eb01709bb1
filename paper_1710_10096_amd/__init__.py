"""MI355X (gfx950) implementation of the sparse scene-flow matching stage of
SceneFlowFields (arXiv 1710.10096, Section 3.1): WHT descriptors, exact-NN
initialisation, red-black propagation with Philox random search, and the
forward/inverse consistency check, as HIP kernels behind the C ABI of
include/sff.h.
"""
from ._native import SffParams, LIB_PATH, EXPORTS  # noqa: F401
from .api import (DIR_BOTH, DIR_FORWARD, DIR_INVERSE,  # noqa: F401
                  SffError, desc_channels, grid_shape, sff_consistency, sff_init_nn, sff_init_workspace_bytes, sff_init_nn_bins, sff_init_bins_workspace_bytes, sff_lanczos_q14,
                  sff_match_level, sff_match_level_bins, sff_bin_bytes, sff_region_filter, sff_region_workspace_bytes, sff_sparsify,
                  sff_sgm_disparity, sff_sgm_workspace_bytes, sff_disparity_fill,
                  sff_sift_workspace_bytes, sff_dense_sift, sff_sift_pca, sff_cost_sift, sff_match_sift, sff_sift_sqrt,
                  sff_version, sff_wht_features, sff_wht_workspace_bytes)
from .api import (MatchCost, sff_cost_f32_bwd, sff_cost_f32_bwd_workspace_bytes,  # noqa: F401
                  sff_cost_f32_fwd, sff_conv3x3_bf16_fwd, sff_featnet_fwd_bf16, sff_conv3x3_bf16_dgrad,
                  sff_conv3x3_bf16_wgrad, sff_smooth_level, sff_quantise_features,
                  sff_triplet_loss, sff_take_grad_bf16)
from .pipeline import PairMatcher, match_pairs  # noqa: F401
