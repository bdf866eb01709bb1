"""Host logic of bench.py: the algorithmic-byte and evaluation-count models
against their closed forms for the KITTI-size workload, the counter-file
lookup (reported only while the kernel sources hash the same), and the
one-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from sff_inputs import kitti_params  # noqa: E402


def test_algorithmic_bytes_kitti():
    p = kitti_params()
    b = bench.algorithmic_bytes(p)
    H, W, C = 375, 1242, 3
    N = [465750, 621 * 188, 311 * 94]                 # grid pixels of levels 0, 1, 2
    assert b["features"] == 4 * 3 * H * W * 33 * C
    assert b["iterations"] == 2 * sum(N) * 6 * (128 * C + 32)
    assert b["handoff"] == 2 * (N[0] + N[1]) * (20 + 128 * C)
    assert b["init"] == 2 * N[2] * (128 * C + 12)
    assert b["consistency"] == H * W * 21
    assert b["total"] == sum(v for k, v in b.items() if k != "total")
    assert abs(b["total"] / 4.11e9 - 1) < 0.002


def test_eval_count_kitti():
    p = kitti_params()
    per_dir = 0
    for Hk, Wk in ((375, 1242), (188, 621), (94, 311)):
        N = Hk * Wk
        per_dir += 6 * ((4 * N - 2 * (Hk + Wk)) + 6 * N) + N
    assert bench.eval_count(p) == 2 * per_dir
    # 4 neighbours + 6 samples for every pixel and iteration, plus one joint cost
    # per pixel, is 61 * sum N = 37,315,652; the grid border lacks
    # 6 * 2 * sum (Hk + Wk) neighbours
    assert per_dir == 37_315_652 - 6 * 2 * (375 + 1242 + 188 + 621 + 94 + 311)


def test_measured_traffic_needs_matching_sources(tmp_path):
    f = tmp_path / "c.txt"
    h = bench.kernel_source_hash()
    f.write_text(f"x\nTRAFFIC kernel=half_step_kernel workload=kitti bytes_per_launch=123 sources={h}\n")
    assert bench.measured_traffic(str(f), "half_step_kernel", "kitti") == 123.0
    assert bench.measured_traffic(str(f), "half_step_kernel", "tiny") is None
    f.write_text("TRAFFIC kernel=half_step_kernel workload=kitti bytes_per_launch=123 sources=0000\n")
    assert bench.measured_traffic(str(f), "half_step_kernel", "kitti") is None
    assert bench.measured_traffic(str(tmp_path / "missing.txt"), "half_step_kernel", "kitti") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_half_step_bytes_kitti():
    """Per-level algorithmic bytes of the propagation / random-search launches
    (both fields): 416 B per grid pixel and iteration at C = 3, plus the
    404-B hand-off below the top level; 3.52 GB per KITTI-size pair, 16 times
    that for the 16-pair batch."""
    p = kitti_params()
    N = [465750, 621 * 188, 311 * 94]
    b = bench.half_step_bytes(p, 1)
    assert b[0] == 2 * N[0] * (6 * 416 + 404)
    assert b[1] == 2 * N[1] * (6 * 416 + 404)
    assert b[2] == 2 * N[2] * 6 * 416
    assert abs(sum(b) / 3.524e9 - 1) < 0.001
    assert bench.half_step_bytes(p, 16) == [16 * x for x in b]


def test_host_cpu_record():
    h = bench.host_cpu()
    assert isinstance(h["model"], str) and h["model"]
    assert h["logical_cpus"] >= h["usable_cpus"] >= 1


def test_source_hash_ignores_comments_only():
    """The traffic figure is keyed to the kernel code: comments and blank
    space do not change the hash, code (string literals included) does."""
    a = 'int f(int x) {  // doubled\n    return 2 * x; /* fast */ }\nconst char* s = "//kept";\n'
    b = 'int f(int x) {\n\n  return 2 * x;  }\nconst char* s = "//kept";  // new note\n'
    c = 'int f(int x) { return 3 * x; }\nconst char* s = "//kept";\n'
    d = 'int f(int x) { return 2 * x; }\nconst char* s = "//other";\n'
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)
    assert bench._code_only(a) != bench._code_only(d)
