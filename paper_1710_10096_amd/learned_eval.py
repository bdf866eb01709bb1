"""Train the learned feature extractor on consistent WHT matches of KITTI-like
pairs and compare the learned-descriptor matcher with the WHT matcher on a
Sintel-like sequence (1024 x 436, 49 frame pairs), on the same GPU.

    python -m paper_1710_10096_amd.learned_eval [--steps 2000] [--train-pairs 8]
                                                [--eval-pairs 49] [--out FILE]

Prints one JSON object: training loss, and per matcher the mean consistent-
match fraction, flow endpoint error, disparity errors, 3-px outlier rate of
consistent matches where ground truth is defined, and the time per pair.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from sff_inputs import kitti_params, kitti_spec, make_scene, sintel_params, sintel_sequence_specs

from .featnet import FeatNet, LearnedMatcher, match_quality, train
from .pipeline import PairMatcher


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--train-pairs", type=int, default=8)
    ap.add_argument("--eval-pairs", type=int, default=49)
    ap.add_argument("--triples", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    dev = torch.device("cuda")
    net = FeatNet(seed=a.seed, device=dev)
    tr = [make_scene(kitti_spec(seed=200 + i)) for i in range(a.train_pairs)]
    t0 = time.perf_counter()
    loss = train(net, tr, kitti_params(), [200 + i for i in range(a.train_pairs)], steps=a.steps,
                 triples=a.triples, seed=a.seed, log=_log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    _log(f"trained {a.steps} steps in {t_train:.1f} s, final loss {loss:.4f}")

    p = sintel_params()
    wht = PairMatcher(p, 1, dev)
    learned = LearnedMatcher(net, p, 1)
    res = {"wht": [], "learned": []}
    times = {"wht": 0.0, "learned": 0.0}
    for i, spec in enumerate(sintel_sequence_specs(a.eval_pairs)):
        sc = make_scene(spec)
        imgs = torch.from_numpy(sc.stack()[None]).to(dev)
        seeds = torch.tensor([spec.seed], dtype=torch.int64, device=dev)
        gt_ok = sc.vis_T & sc.vis_S & sc.vis_X
        for name, m in (("wht", wht), ("learned", learned)):
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = m.run(imgs, seeds)
            torch.cuda.synchronize()
            times[name] += time.perf_counter() - t
            q = match_quality(out["hyp"][0, 0].cpu().numpy(), out["valid"][0].cpu().numpy(),
                              sc.gt_fwd, gt_ok)
            res[name].append(q)
        if i % 10 == 0:
            _log(f"pair {i}: wht {res['wht'][-1]} learned {res['learned'][-1]}")
    summary = {"train": {"steps": a.steps, "pairs": a.train_pairs, "triples": a.triples,
                         "final_loss": loss, "seconds": t_train},
               "eval": {"workload": "sintel_like_1024x436x3_K3_it6", "pairs": a.eval_pairs}}
    for name in res:
        keys = res[name][0].keys()
        summary[name] = {k: float(np.nanmean([r[k] for r in res[name]])) for k in keys}
        summary[name]["ms_per_pair"] = 1e3 * times[name] / a.eval_pairs
    line = json.dumps(summary)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")
    return summary


if __name__ == "__main__":
    main()
