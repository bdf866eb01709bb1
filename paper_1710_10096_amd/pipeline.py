"""The matching stage for a batch of pairs (SceneFlowFields, Section 3
overview, up to the consistency check), as a sequence of libsff calls on one
stream: for levels K-1 .. 0, WHT features of the four views, exact-NN
initialisation at the coarsest level, propagation + random search with the
hand-off from the coarser level; then the consistency check at level 0.
The matcher takes the descriptor distances from the WHT bin-sum planes
(``maps="bins"``, the default; descriptors are formed only at the coarsest
level, for the initialisation) or from the descriptor records of every level
(``maps="desc"``); both give the same fields.
Forward and inverse fields run together (SFF_DIR_BOTH).  With ``s_c`` set,
the region filter (Section 3.1, second consistency step) and the 3x3
sparsification (Section 3.2) follow, giving the seeds of the interpolation.

Buffers are allocated once per shape; a call only enqueues kernels.
"""
from __future__ import annotations

import torch

from . import api
from ._native import SffParams


class PairMatcher:
    def __init__(self, params, batch: int = 1, device: str | torch.device = "cuda",
                 s_c: int | None = None, leaves: int = 1, maps: str = "bins"):
        self.p = params if isinstance(params, SffParams) else SffParams.from_dict(params)
        self.batch = int(batch)
        if maps not in ("bins", "desc"):
            raise ValueError("maps must be 'bins' or 'desc'")
        self.maps = maps
        p, B = self.p, self.batch
        dev = torch.device(device)
        ws = max(api.sff_wht_workspace_bytes(p, 4 * B, k) for k in range(p.levels))
        if maps == "desc":
            self.desc = torch.zeros((B, 4, p.H, p.W, api.desc_channels(p.C), 16), dtype=torch.int16,
                                    device=dev)
            ws = max(ws, api.sff_init_workspace_bytes(p, B))
        else:
            # bin-sum planes of one level at a time (the largest level's size)
            nb = max(api.sff_bin_bytes(p, k) for k in range(p.levels))
            self.bins = torch.empty(4 * B * nb, dtype=torch.uint8, device=dev)
            ws = max(ws, api.sff_init_bins_workspace_bytes(p, B))
        self.ws = torch.empty(max(ws, 256), dtype=torch.uint8, device=dev)
        self.hyp, self.cost = [], []
        for k in range(p.levels):
            Hk, Wk = api.grid_shape(p, k)
            self.hyp.append(torch.empty((2, B, Hk, Wk, 4), dtype=torch.int16, device=dev))
            self.cost.append(torch.empty((2, B, Hk, Wk), dtype=torch.int32, device=dev))
        self.valid = torch.empty((B, p.H, p.W), dtype=torch.uint8, device=dev)
        self.err = torch.empty((B, p.H, p.W), dtype=torch.int32, device=dev)
        self.s_c = s_c
        self.leaves = int(leaves)
        if s_c is not None:
            self.keep = torch.empty((B, p.H, p.W), dtype=torch.uint8, device=dev)
            self.seeds = torch.empty((B, (p.H + 2) // 3, (p.W + 2) // 3), dtype=torch.int32,
                                     device=dev)
            self.ws_region = torch.empty(api.sff_region_workspace_bytes(p, B), dtype=torch.uint8,
                                         device=dev)

    def run(self, imgs: torch.Tensor, seeds: torch.Tensor, stream=None, mark=None) -> dict:
        """imgs uint8 [batch][4][H][W][C] (l0, l1, r0, r1); seeds int64 [batch].
        ``mark(name)``, if given, is called before the first and after every
        library call (timing hooks)."""
        mk = mark if mark is not None else (lambda name: None)
        p, B = self.p, self.batch
        if tuple(imgs.shape) != (B, 4, p.H, p.W, p.C):
            raise ValueError(f"imgs must be [{B}, 4, {p.H}, {p.W}, {p.C}]")
        flat_img = imgs.view(4 * B, p.H, p.W, p.C)
        top = p.levels - 1
        mk("start")
        bins = self.maps == "bins"
        for k in range(top, -1, -1):
            if bins:
                api.sff_wht_features(p, flat_img, k, None, self.ws, stream, bins=self.bins,
                                     want_desc=False)
            else:
                flat_desc = self.desc.view(4 * B, p.H, p.W, self.desc.shape[4], 16)
                api.sff_wht_features(p, flat_img, k, flat_desc, self.ws, stream)
            mk(f"features:L{k}")
            coarse = None if k == top else self.hyp[k + 1]
            if k == top:
                if bins:
                    api.sff_init_nn_bins(p, self.bins, B, api.DIR_BOTH, self.hyp[k], self.cost[k],
                                         self.ws, stream, leaves=self.leaves)
                else:
                    api.sff_init_nn(p, self.desc, api.DIR_BOTH, self.hyp[k], self.cost[k], self.ws,
                                    stream, leaves=self.leaves)
                mk(f"init:L{k}")
            if bins:
                api.sff_match_level_bins(p, self.bins, api.DIR_BOTH, k, seeds, self.hyp[k],
                                         self.cost[k], coarse, stream)
            else:
                api.sff_match_level(p, self.desc, api.DIR_BOTH, k, seeds, self.hyp[k],
                                    self.cost[k], coarse, stream)
            mk(f"match:L{k}")
        api.sff_consistency(p, self.hyp[0][0], self.hyp[0][1], self.valid, self.err, stream)
        mk("consistency:L0")
        out = dict(hyp=self.hyp[0], cost=self.cost[0], valid=self.valid, err=self.err)
        if self.s_c is not None:
            self.filter_and_sparsify(stream, mk)
            out.update(keep=self.keep, seeds=self.seeds)
        return out

    def disparity_fill(self, imgs: torch.Tensor, stream=None, mark=None) -> dict:
        """Disparity fill of the last run's result (Section 3.1, last paragraph
        of "Consistency Check"): SGM disparity of the stereo pair at t0 and the
        check of the matched d0 alone against it.  imgs as given to run()."""
        mk = mark if mark is not None else (lambda name: None)
        p, B = self.p, self.batch
        if not hasattr(self, "ws_sgm"):
            dev = self.valid.device
            self.ws_sgm = torch.empty(api.sff_sgm_workspace_bytes(p, B), dtype=torch.uint8,
                                      device=dev)
            self.disp = torch.empty((B, p.H, p.W), dtype=torch.int16, device=dev)
            self.fill = torch.empty((B, p.H, p.W), dtype=torch.uint8, device=dev)
        api.sff_sgm_disparity(p, imgs[:, 0], imgs[:, 2], disp=self.disp, workspace=self.ws_sgm,
                              stream=stream)
        mk("sgm:L0")
        api.sff_disparity_fill(p, self.hyp[0][0], self.valid, self.disp, self.fill, stream)
        mk("fill:L0")
        return dict(disp=self.disp, fill=self.fill)

    def refine_sift(self, imgs: torch.Tensor, seeds: torch.Tensor, iters: int | None = None,
                    stream=None, mark=None) -> dict:
        """Matching with the paper's own cost (Section 3.1, eq. (1) on SIFT-PCA
        features) at full resolution, starting from the last run's level-0
        fields, then the consistency check again."""
        mk = mark if mark is not None else (lambda name: None)
        p, B = self.p, self.batch
        if not hasattr(self, "ws_sift"):
            self.ws_sift = torch.empty(api.sff_sift_workspace_bytes(p, 4 * B), dtype=torch.uint8,
                                       device=self.valid.device)
            self.sift_out = None
            self.cost_sift = torch.empty((2, B, p.H, p.W), dtype=torch.float32,
                                         device=self.valid.device)
        self.sift_out = api.sff_sift_pca(p, imgs, out=self.sift_out, workspace=self.ws_sift,
                                         stream=stream)
        mk("sift_features:L0")
        api.sff_match_sift(p, self.sift_out["phi"], seeds, self.hyp[0], api.DIR_BOTH, iters,
                           self.cost_sift, stream)
        mk("sift_match:L0")
        api.sff_consistency(p, self.hyp[0][0], self.hyp[0][1], self.valid, self.err, stream)
        mk("sift_consistency:L0")
        return dict(hyp=self.hyp[0], cost=self.cost_sift, valid=self.valid, err=self.err)

    def filter_and_sparsify(self, stream=None, mark=None):
        """Region filter and 3x3 sparsification of the last run's result."""
        mk = mark if mark is not None else (lambda name: None)
        p = self.p
        api.sff_region_filter(p, self.hyp[0][0], self.valid, self.s_c, self.keep, self.ws_region,
                              stream)
        mk("region:L0")
        api.sff_sparsify(p, self.keep, self.err, self.seeds, stream)
        mk("sparsify:L0")


def match_pairs(params, imgs: torch.Tensor, seeds: torch.Tensor) -> dict:
    """One-shot convenience wrapper around PairMatcher (returns copies)."""
    m = PairMatcher(params, imgs.shape[0], imgs.device)
    out = m.run(imgs, seeds)
    return {k: v.clone() for k, v in out.items()}
