"""GPU parity of the SGM disparity and the disparity fill against the oracle,
bit-exact.  Inputs come from seeded generators or the oracle's own output."""
import sys

import numpy as np
import pytest

import oracle
from sff_inputs import kitti_params, kitti_spec, make_scene, params_dict, small_spec

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sff():
    import torch
    import paper_1710_10096_amd as m
    assert torch.cuda.is_available()
    return m


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


CASES = [  # H, W, C, dmax, P1, P2, batch
    (9, 13, 3, 5, 3, 24, 1), (1, 40, 1, 7, 2, 9, 2), (40, 1, 2, 3, 3, 24, 1), (31, 57, 3, 12, 0, 0, 1),
    (24, 70, 4, 30, 5, 60, 3), (17, 300, 1, 255, 3, 24, 1), (6, 6, 3, 0, 3, 24, 1),
    (20, 90, 3, 64, 10, 231, 1), (12, 100, 3, 191, 3, 24, 2),  # largest P2; dmax + 1 > W
]


@pytest.mark.parametrize("case", CASES, ids=[str(c) for c in CASES])
def test_sgm_parity(sff, case):
    import torch
    H, W, C, dmax, P1, P2, B = case
    rng = np.random.default_rng(H * 31 + W + C + dmax)
    imgs = rng.integers(0, 256, (B, 4, H, W, C), dtype=np.uint8)
    # a shifted copy as the right view so that the disparities are structured
    shift = min(4, max(W - 1, 0))
    imgs[:, 2] = np.roll(imgs[:, 0], -shift, axis=2)
    p = params_dict(H, W, C, levels=1, iters=1, dmax=dmax)
    _say("sgm", case)
    g = dev(imgs)
    disp = sff.sff_sgm_disparity(p, g[:, 0], g[:, 2], P1, P2)
    torch.cuda.synchronize()
    d = disp.cpu().numpy()
    for b in range(B):
        assert np.array_equal(d[b], oracle.sgm(imgs[b, 0], imgs[b, 2], dmax + 1, P1, P2)), (case, b)


def test_sgm_constant_images(sff):
    """Every cost is zero: all disparities tie and the smallest, 0, wins."""
    import torch
    H, W = 33, 170
    imgs = np.full((1, 4, H, W, 3), 77, np.uint8)
    p = params_dict(H, W, 3, levels=1, iters=1, dmax=100)
    _say("sgm constant")
    g = dev(imgs)
    disp = sff.sff_sgm_disparity(p, g[:, 0], g[:, 2])
    torch.cuda.synchronize()
    assert not disp.cpu().numpy().any()
    assert not oracle.sgm(imgs[0, 0], imgs[0, 2], 101, sff.api.SGM_P1, sff.api.SGM_P2).any()


def test_sgm_and_fill_on_matching_output(sff):
    """The KITTI-size stereo pair at t0 and the oracle's own matching result."""
    import torch
    sc = make_scene(kitti_spec())
    p = kitti_params()
    imgs = sc.stack()
    _say("sgm kitti")
    g = dev(imgs[None])
    disp = sff.sff_sgm_disparity(p, g[:, 0], g[:, 2])
    torch.cuda.synchronize()
    want = oracle.sgm(imgs[0], imgs[2], p["dmax"] + 1, sff.api.SGM_P1, sff.api.SGM_P2)
    assert np.array_equal(disp.cpu().numpy()[0], want)
    _say("oracle match_pair kitti")
    ref = oracle.match_pair(imgs, p, 2)
    fill = sff.sff_disparity_fill(p, dev(ref["hyp"][0][None]), dev(ref["valid"][None]),
                                  dev(want[None]))
    torch.cuda.synchronize()
    wf = oracle.disparity_fill(ref["hyp"][0], ref["valid"], want, p["tau"])
    assert np.array_equal(fill.cpu().numpy()[0], wf)
    assert wf.sum() >= ref["valid"].sum()


def test_pipeline_disparity_fill(sff):
    """PairMatcher.disparity_fill after a run, on the tiny pair."""
    import torch
    from sff_inputs import tiny_params, tiny_spec
    sc = make_scene(tiny_spec())
    p = tiny_params()
    imgs = dev(sc.stack()[None])
    _say("pipeline tiny disparity fill")
    m = sff.PairMatcher(p, 1)
    m.run(imgs, dev(np.array([1], np.int64)))
    out = m.disparity_fill(imgs)
    torch.cuda.synchronize()
    ref = oracle.match_pair(sc.stack(), p, 1)
    disp = oracle.sgm(sc.stack()[0], sc.stack()[2], p["dmax"] + 1, sff.api.SGM_P1, sff.api.SGM_P2)
    assert np.array_equal(out["disp"].cpu().numpy()[0], disp)
    assert np.array_equal(out["fill"].cpu().numpy()[0],
                          oracle.disparity_fill(ref["hyp"][0], ref["valid"], disp, p["tau"]))
