"""Benchmark of the sparse scene-flow matching stage on one MI355X.

One step = the whole stage on one batch of synthetic pairs resident in HBM:
WHT features of the four views at every level, exact-NN initialisation,
propagation + random search on every level for the forward and inverse
fields, and the consistency check.  Prints one JSON line.

Usage: python bench.py [--steps K] [--warmup W] [--workload kitti|kitti_batch16|tiny]
                       [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure


def workload(name: str):
    from sff_inputs import (kitti_batch_specs, kitti_params, kitti_spec, make_scene, tiny_params,
                            tiny_spec)
    if name == "kitti":
        return [make_scene(kitti_spec())], kitti_params(), [2]
    if name == "kitti_batch16":
        specs = kitti_batch_specs()
        return [make_scene(s) for s in specs], kitti_params(), [s.seed for s in specs]
    if name == "tiny":
        return [make_scene(tiny_spec())], tiny_params(), [1]
    raise SystemExit(f"unknown workload {name}")


def grid(p, k):
    n = 1 << k
    return (p["H"] + n - 1) // n, (p["W"] + n - 1) // n


def eval_count(p) -> int:
    """Hypothesis-cost evaluations per pair (both fields): joint cost of every
    initialised pixel, hand-off recomputations, and per iteration the in-grid
    neighbours plus the random-search samples of every pixel."""
    K = p["levels"]
    total = 0
    for k in range(K):
        Hk, Wk = grid(p, k)
        N = Hk * Wk
        nbrs = 4 * N - 2 * (Hk + Wk)
        total += p["iters"] * (nbrs + p["rs_samples"] * N)
        total += N  # init joint cost at the top level, hand-off recompute below it
    return 2 * total


def algorithmic_bytes(p) -> dict:
    """Bytes the stage must move once per pair (not cache-inflated):
    features 4 K H W 33C; per level-iteration and pixel 128C + 32 (reference and
    three target descriptors, own vector/cost read+write, neighbours' vectors);
    hand-off N_k (20 + 128C); init N_top (128C + 12); consistency 21 H W."""
    C, K, H, W = p["C"], p["levels"], p["H"], p["W"]
    feat = 4 * K * H * W * 33 * C
    it = sum(grid(p, k)[0] * grid(p, k)[1] for k in range(K)) * p["iters"] * (128 * C + 32)
    hand = sum(grid(p, k)[0] * grid(p, k)[1] for k in range(K - 1)) * (20 + 128 * C)
    Ht, Wt = grid(p, K - 1)
    init = Ht * Wt * (128 * C + 12)
    cons = H * W * 21
    return dict(features=feat, iterations=2 * it, handoff=2 * hand, init=2 * init,
                consistency=cons, total=feat + 2 * (it + hand + init) + cons)


def cpu_baseline(scenes, p, seeds) -> dict:
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(os.cpu_count() or 1, 16)
    t0 = time.perf_counter()
    oracle.match_pair(scenes[0].stack(), p, int(seeds[0]), nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": p["H"] * p["W"] / dt, "unit": "px/s", "cores": threads, "kind": "oracle",
            "sample": f"whole stage on 1 pair of the workload ({dt:.2f} s)",
            "cpu": platform.processor() or platform.machine()}


def copy_probe(nbytes: int = 256 * 1024 * 1024, reps: int = 3):
    """A plain device-to-device copy of known size: under rocprofv3 --pmc it
    calibrates FETCH_SIZE / WRITE_SIZE (counter bytes per byte moved)."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes": nbytes, "reps": reps, "GBps": 2 * nbytes / dt / 1e9}), flush=True)


def probes(reps: int = 5) -> dict:
    """Achievable bandwidth of a streaming copy (512 MiB) and of random record
    gathers over a buffer the size of one level's four KITTI-size descriptor
    maps (179 MB), for 96-byte (RGB descriptor) and 128-byte records."""
    import torch
    import paper_1710_10096_amd as sff
    res = {}
    n = 512 * 1024 * 1024
    a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(3)
    b = torch.empty_like(a)
    sff.api.sff_probe_copy(a, b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        sff.api.sff_probe_copy(a, b)
    e1.record()
    torch.cuda.synchronize()
    res["copy_GBps"] = 2 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    buf = torch.empty(4 * 1242 * 375 * 96, dtype=torch.uint8, device="cuda").fill_(1)
    threads, per = 256 * 1024 * 4, 8
    out = torch.empty(threads, dtype=torch.int32, device="cuda")
    for rb in (96, 128):
        sff.api.sff_probe_gather(buf, rb, threads, per, out)
        torch.cuda.synchronize()
        e0.record()
        for r in range(reps):
            sff.api.sff_probe_gather(buf, rb, threads, per, out, seed=r + 2)
        e1.record()
        torch.cuda.synchronize()
        res[f"gather{rb}_GBps"] = rb * threads * per * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="kitti")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 256 MiB device to device three times (counter calibration)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        raise SystemExit(2)

    import torch
    import paper_1710_10096_amd as sff

    scenes, p, seeds = workload(args.workload)
    B = len(scenes)
    imgs = torch.from_numpy(np.stack([s.stack() for s in scenes])).cuda()
    seeds_t = torch.tensor(seeds, dtype=torch.int64, device="cuda")
    m = sff.PairMatcher(p, B)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        m.run(imgs, seeds_t)
    torch.cuda.synchronize()

    # per-call events inside the timed region (same stream as the kernels)
    marks = []

    def mark(name):
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        marks[-1].append((name, e))

    t0 = time.perf_counter()
    for _ in range(args.steps):
        marks.append([])
        m.run(imgs, seeds_t, mark=mark)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt * 1e3 / args.steps

    stage_ms: dict[str, float] = {}
    for step in marks:
        for (n0, e0), (n1, e1) in zip(step[:-1], step[1:]):
            stage_ms[n1] = stage_ms.get(n1, 0.0) + e0.elapsed_time(e1) / args.steps

    npx = p["H"] * p["W"] * B
    ab = algorithmic_bytes(p)
    evals = eval_count(p) * B

    # dominant kernel: the stage with the largest share of the step
    dom = max(stage_ms, key=stage_ms.get)
    k_dom = dom.split(":")[-1]
    K = p["levels"]
    roof = None
    if dom.startswith("match"):
        lvl = int(k_dom[1:])
        Hk, Wk = grid(p, lvl)
        launches = 2 * p["iters"]
        per_launch_bytes = 2 * B * Hk * Wk / 2 * (128 * p["C"] + 32)
        avg_us = stage_ms[dom] * 1e3 / launches
        ach = per_launch_bytes / (avg_us * 1e-6) / 1e9
        roof = {"kernel": "half_step_kernel", "level": lvl, "bound": "hbm", "achieved": ach,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": None, "avg_launch_us": avg_us}
    elif dom.startswith("init"):
        Ht, Wt = grid(p, K - 1)
        per_launch_bytes = 2 * B * Ht * Wt * (128 * p["C"] + 12)
        avg_us = stage_ms[dom] * 1e3
        ach = per_launch_bytes / (avg_us * 1e-6) / 1e9
        roof = {"kernel": "init_nn_kernel", "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None, "avg_launch_us": avg_us}

    out = {
        "metric": "matched_px_per_s", "value": npx / (ms * 1e-3), "unit": "px/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i16",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}_{p['W']}x{p['H']}x{p['C']}_K{K}_it{p['iters']}",
                   "pairs": B, "levels": K, "iters": p["iters"], "fmax": p["fmax"],
                   "dmax": p["dmax"], "parallelism": "single_gpu"},
        "evals_per_s": evals / (ms * 1e-3),
        "algorithmic_bytes": ab["total"] * B,
        "hbm_frac_whole_step": ab["total"] * B / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "roofline": roof,
    }
    out["probes"] = probes()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scenes, p, seeds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
