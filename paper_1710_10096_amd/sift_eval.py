"""Quality and cost of matching with the paper's own cost (Section 3.1,
eq. (1) on SIFT-PCA features) at full resolution, started from the WHT
matcher's result, against the WHT matcher alone, on the same GPU.

    python -m paper_1710_10096_amd.sift_eval [--kitti-pairs 16] [--sintel-pairs 16]
                                             [--iters N] [--out FILE]

Prints one JSON object: per workload the mean consistent-match fraction,
flow endpoint error, disparity errors and 3-px outlier rate of consistent
matches where ground truth is defined, before and after the refinement, and
the time of the SIFT-PCA features and of the refinement.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np
import torch

from sff_inputs import (kitti_batch_specs, kitti_params, make_scene, sintel_params,
                        sintel_sequence_specs)

from .featnet import match_quality
from .pipeline import PairMatcher


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def evaluate(specs, p, dev, iters):
    m = PairMatcher(p, 1, dev)
    before, after = [], []
    t_feat = t_match = 0.0
    for i, spec in enumerate(specs):
        sc = make_scene(spec)
        imgs = torch.from_numpy(sc.stack()[None]).to(dev)
        seeds = torch.tensor([spec.seed], dtype=torch.int64, device=dev)
        gt_ok = sc.vis_T & sc.vis_S & sc.vis_X
        out = m.run(imgs, seeds)
        torch.cuda.synchronize()
        before.append(match_quality(out["hyp"][0, 0].cpu().numpy(), out["valid"][0].cpu().numpy(),
                                    sc.gt_fwd, gt_ok))
        marks = []

        def mark(name, marks=marks):
            e = torch.cuda.Event(enable_timing=True)
            e.record()
            marks.append((name, e))

        mark("start")
        out = m.refine_sift(imgs, seeds, iters=iters, mark=mark)
        torch.cuda.synchronize()
        t_feat += marks[0][1].elapsed_time(marks[1][1])
        t_match += marks[1][1].elapsed_time(marks[2][1])
        after.append(match_quality(out["hyp"][0, 0].cpu().numpy(), out["valid"][0].cpu().numpy(),
                                   sc.gt_fwd, gt_ok))
        if i % 4 == 0:
            _log(f"pair {i}: WHT {before[-1]['consistent_frac']:.3f}/{before[-1]['flow_epe']:.3f} "
                 f"+SIFT {after[-1]['consistent_frac']:.3f}/{after[-1]['flow_epe']:.3f}")
    keys = before[0].keys()
    res = {"wht": {k: float(np.nanmean([r[k] for r in before])) for k in keys},
           "wht_then_sift": {k: float(np.nanmean([r[k] for r in after])) for k in keys}}
    res["sift_features_ms"] = t_feat / len(specs)
    res["sift_match_ms"] = t_match / len(specs)
    res["sift_iters"] = iters
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--kitti-pairs", type=int, default=16)
    ap.add_argument("--sintel-pairs", type=int, default=16)
    ap.add_argument("--iters", type=int, default=None, help="refinement iterations (default: the workload's)")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    dev = torch.device("cuda")
    kp, spr = kitti_params(), sintel_params()
    summary = {
        "kitti_like_1242x375x3": evaluate(kitti_batch_specs()[:a.kitti_pairs], kp, dev,
                                          a.iters if a.iters is not None else kp["iters"]),
        "sintel_like_1024x436x3": evaluate(sintel_sequence_specs(a.sintel_pairs), spr, dev,
                                           a.iters if a.iters is not None else spr["iters"]),
    }
    line = json.dumps(summary)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(line + "\n")


if __name__ == "__main__":
    main()
