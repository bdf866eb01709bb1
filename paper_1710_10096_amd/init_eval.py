"""Quality and cost of the initialisation with several temporal leaves
(Section 3.1, "Initialization": all combinations of the leaves compared by
eq. (1)) against the single-leaf initialisation, on the same GPU: the whole
matching stage with leaves = 1, 2, 4 on KITTI-like pairs (the 16-pair batch
statistics) and on the Sintel-like sequence.

    python -m paper_1710_10096_amd.init_eval [--kitti-pairs 16] [--sintel-pairs 49]
                                             [--out FILE]

Prints one JSON object: per workload and number of leaves the mean consistent-
match fraction, flow endpoint error, disparity errors and 3-px outlier rate of
consistent matches where ground truth is defined, the share of coarsest-level
vectors the combinations changed, and the time of the initialisation call.
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

LEAVES = (1, 2, 4)


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def evaluate(specs, p, dev):
    ms = {k: PairMatcher(p, 1, dev, leaves=k) for k in LEAVES}
    res = {k: [] for k in LEAVES}
    changed = {k: [] for k in LEAVES}
    t_init = {k: 0.0 for k in LEAVES}
    top = p["levels"] - 1
    for i, spec in enumerate(specs):
        sc = make_scene(spec)
        imgs = torch.from_numpy(sc.stack()[None]).to(dev)
        seeds = torch.tensor([spec.seed], dtype=torch.int64, device=dev)
        gt_ok = sc.vis_T & sc.vis_S & sc.vis_X
        init1 = None
        for k, m in ms.items():
            marks = []

            def mark(name, marks=marks):
                e = torch.cuda.Event(enable_timing=True)
                e.record()
                marks.append((name, e))

            out = m.run(imgs, seeds, mark=mark)
            torch.cuda.synchronize()
            for (n0, e0), (n1, e1) in zip(marks[:-1], marks[1:]):
                if n1.startswith("init"):
                    t_init[k] += e0.elapsed_time(e1)
            res[k].append(match_quality(out["hyp"][0, 0].cpu().numpy(),
                                        out["valid"][0].cpu().numpy(), sc.gt_fwd, gt_ok))
            # the coarsest field is overwritten by matching: rerun the init alone
            init = _init_only(m, imgs, top)
            if k == 1:
                init1 = init
            changed[k].append(float((init != init1).any(axis=-1).mean()))
        if i % 8 == 0:
            _log(f"pair {i}: " + " ".join(f"L{k} {res[k][-1]['consistent_frac']:.3f}/"
                                          f"{res[k][-1]['flow_epe']:.3f}" for k in LEAVES))
    out = {}
    for k in LEAVES:
        keys = res[k][0].keys()
        out[f"leaves{k}"] = {key: float(np.nanmean([r[key] for r in res[k]])) for key in keys}
        out[f"leaves{k}"]["init_changed_frac"] = float(np.mean(changed[k]))
        out[f"leaves{k}"]["init_ms"] = t_init[k] / len(specs)
    return out


def _init_only(m, imgs, top):
    from . import api
    p, B = m.p, m.batch
    flat_img = imgs.view(4 * B, p.H, p.W, p.C)
    api.sff_wht_features(p, flat_img, top, None, m.ws, bins=m.bins, want_desc=False)
    hyp, _ = api.sff_init_nn_bins(p, m.bins, B, api.DIR_BOTH, None, None, m.ws, leaves=m.leaves)
    return hyp[0, 0].cpu().numpy()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--kitti-pairs", type=int, default=16)
    ap.add_argument("--sintel-pairs", type=int, default=49)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    dev = torch.device("cuda")
    summary = {
        "kitti_like_1242x375x3_K3_it6": evaluate(kitti_batch_specs()[:a.kitti_pairs],
                                                 kitti_params(), dev),
        "sintel_like_1024x436x3_K3_it6": evaluate(sintel_sequence_specs(a.sintel_pairs),
                                                  sintel_params(), dev),
    }
    line = json.dumps(summary)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(line + "\n")


if __name__ == "__main__":
    main()
