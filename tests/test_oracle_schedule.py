"""The paper's sequential four-corner propagation schedule in the oracle
(Section 3.1, "Multi-Scale Propagation"), kept to measure what the red-black
Jacobi schedule of the GPU path changes.  Pins of the schedule itself, then a
quality comparison of the two schedules on small synthetic pairs."""
import sys

import numpy as np

import oracle
from sff_inputs import SceneSpec, make_scene, params_dict, small_spec


def _descs(imgs, level):
    return [oracle.features(imgs[m], level) for m in range(4)]


def _planted(H, W, corner):
    """A clean one-segment translation (disparity 3, no flow); every grid
    vector wrong (disparities 9) except one pixel, which holds the true vector.
    In columns 0..3 both vectors' stereo and cross targets land on column 0
    (exactly or clamped) and score the same, so a vector never passes there; the planted
    pixels lie outside that zone.  No random search."""
    sc = make_scene(SceneSpec(H=H, W=W, C=1, seed=5, n_segments=(1, 1), d_range=(3, 3),
                              flow_max=0, delta_max=0, occluder=False, salt=0.0))
    D = _descs(sc.stack(), 0)
    true = sc.gt_fwd[H // 2, W // 2].copy()
    hyp = np.zeros((H, W, 4), np.int16)
    hyp[..., 2] = hyp[..., 3] = 9          # wrong disparities everywhere
    i, j = {"tl": (0, 10), "br": (H - 1, W - 1)}[corner]
    hyp[i, j] = true
    cost = np.array([[oracle.cost(D, 1, x, y, hyp[y, x]) for x in range(W)] for y in range(H)],
                    np.uint32)
    return D, hyp, cost, true


def test_scan_carries_a_vector_along_the_whole_path():
    H, W = 20, 28
    D, hyp, cost, true = _planted(H, W, "tl")
    h1, c1 = oracle.match_level_scan(D, 0, 1, 3, 1, 32, 0, 8, 8, hyp, cost)
    # one top-left scan carries the vector planted at (0, 10) to every pixel
    # right of it and below (interior columns: at the right border the
    # rendered scene's hole filling can favour the wrong vector), and to none
    # left of it
    reached = (h1 == true).all(axis=-1)
    assert reached[:, 10:W - 3].all() and not reached[:, :10].any()
    # the red-black schedule moves it one neighbour per half-step
    h2, _ = oracle.match_level(D, 0, 1, 3, 1, 32, 0, 8, 8, hyp, cost)
    reached = (h2 == true).all(axis=-1)
    ii, jj = np.nonzero(reached)
    assert reached.sum() < 6 and (ii + np.abs(jj - 10)).max() <= 2
    # costs are those of the vectors, never above the start
    assert (c1 <= cost).all()
    for y, x in ((0, 0), (7, 13), (H - 1, W - 1)):
        assert c1[y, x] == oracle.cost(D, 1, x, y, h1[y, x])


def test_scan_directions_cycle_through_the_corners():
    """A vector planted in the bottom-right corner does not move in the
    top-left scan (iteration 0) and reaches every pixel in the bottom-right
    scan (iteration 1)."""
    H, W = 14, 17
    D, hyp, cost, true = _planted(H, W, "br")
    h0, _ = oracle.match_level_scan(D, 0, 1, 3, 1, 32, 0, 8, 8, hyp, cost)
    assert (h0 == true).all(axis=-1).sum() <= 3
    h1, _ = oracle.match_level_scan(D, 0, 1, 3, 2, 32, 0, 8, 8, hyp, cost)
    reached = (h1 == true).all(axis=-1)
    assert reached[:-1, 4:W - 3].all() and not reached[:, :4].any()


def test_scan_without_iterations_is_the_start():
    H, W = 9, 11
    D, hyp, cost, _ = _planted(H, W, "tl")
    h, c = oracle.match_level_scan(D, 0, 1, 3, 0, 32, 6, 8, 8, hyp, cost)
    assert np.array_equal(h, hyp) and np.array_equal(c, cost)


def _quality(out, sc):
    v = out["valid"].astype(bool)
    ok = sc.vis_T & sc.vis_S & sc.vis_X
    sel = v & ok
    d = out["hyp"][0].astype(np.float64) - sc.gt_fwd.astype(np.float64)
    epe = np.hypot(d[..., 0], d[..., 1])
    return v.mean(), epe[sel].mean(), np.abs(d[..., 2])[sel].mean()


def test_red_black_versus_scan_quality():
    """Both schedules on small pairs: the red-black schedule keeps density and
    accuracy close to the sequential one (a measurement, with loose bounds)."""
    rows = []
    for seed in (21, 22, 23):
        sc = make_scene(small_spec(64, 96, 3, seed, flow_max=10, d_range=(0, 14)))
        p = params_dict(64, 96, 3, levels=2, iters=4, fmax=16, dmax=16)
        q = [_quality(oracle.match_pair(sc.stack(), p, seed, schedule=s), sc)
             for s in ("red-black", "scan")]
        rows.append(q)
        print(f"[schedule] seed {seed}: red-black frac {q[0][0]:.3f} epe {q[0][1]:.3f} d0 {q[0][2]:.3f}"
              f" | scan frac {q[1][0]:.3f} epe {q[1][1]:.3f} d0 {q[1][2]:.3f}", file=sys.stderr)
    rb = np.array([r[0] for r in rows]), np.array([r[1] for r in rows])
    for (f_rb, e_rb, _), (f_sc, e_sc, _) in rows:
        assert f_rb > 0.5 * f_sc and e_rb < e_sc + 0.5
    assert np.isfinite(rb[1]).all()
