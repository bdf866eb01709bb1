"""GPU parity: every libsff entry point against the CPU oracle, bit-exact
(integer path: descriptors, vectors, costs, argmin tie-breaks, masks, errors).

Inputs are seeded synthetic scenes; expected values come only from ``oracle``.
"""
import sys
import zlib

import numpy as np
import pytest

import oracle
from sff_inputs import (make_scene, small_spec, tiny_spec, tiny_params, kitti_spec,
                        kitti_params, params_dict)

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


def host(t, u32=False):
    a = t.cpu().numpy()
    return a.view(np.uint32) if u32 else a


def _imgs_stack(scenes):
    return np.stack([sc.stack() for sc in scenes], axis=0)  # [B][4][H][W][C]


def _oracle_descs(imgs_b, level):
    """imgs_b [4][H][W][C] -> 4 oracle descriptor maps."""
    return [oracle.features(imgs_b[m], level) for m in range(4)]


# ------------------------------------------------------------- features ----
FEATURE_CASES = [
    ("tiny_l0", 96, 160, 1, 1, [0]),
    ("ragged_c3", 37, 53, 3, 3, [0, 1, 2]),
    ("ragged_c2_l4", 29, 71, 2, 4, [0, 3]),
    ("c4", 20, 24, 4, 2, [0, 1]),
    ("one_pixel", 1, 1, 1, 2, [0, 1]),
    ("thin_row", 1, 40, 3, 3, [2]),
]


@pytest.mark.parametrize("case", FEATURE_CASES, ids=[c[0] for c in FEATURE_CASES])
def test_wht_features_parity(sff, case):
    name, H, W, C, levels, lvls = case
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    imgs = rng.integers(0, 256, (4, H, W, C), dtype=np.uint8)
    p = params_dict(H, W, C, levels=levels, iters=1)
    Cp = sff.desc_channels(C)
    for lv in lvls:
        _say("features", name, "level", lv)
        # padding channels of a record are never written: pre-fill a sentinel
        out = dev(np.full((4, H, W, Cp, 16), 0x5A5A, np.int16))
        d = host(sff.sff_wht_features(p, dev(imgs), lv, out))
        for m in range(4):
            assert np.array_equal(d[m][:, :, :C], oracle.features(imgs[m], lv)), (name, lv, m)
        assert (d[:, :, :, C:] == 0x5A5A).all()


def test_wht_features_kitti_full(sff):
    sc = make_scene(kitti_spec())
    p = kitti_params()
    imgs = sc.stack()
    g = dev(imgs)
    for lv in range(3):
        _say("features kitti level", lv)
        d = host(sff.sff_wht_features(p, g, lv))
        for m in range(4):
            assert np.array_equal(d[m][:, :, :p["C"]], oracle.features(imgs[m], lv)), (lv, m)


def _bins_expected(S, level):
    """Bin-sum planes of one smoothed image S [H][W][C] in the layout of
    include/sff.h, from the plain definition: bin at extended position
    (ex, ey) = (X + 3n, Y + 3n) sums S at X + {0, n}, Y + {0, n} (clamped);
    entry (r, q) of plane (py, px) holds extended rows (r + m) P + py, m = 0..3,
    at extended column q P + px; C uint16 channels per bin, or for C = 3 the
    four bins b_0..b_3 of an entry packed into four uint32 words (channels 0
    and 1 in the halves' low 10 bits, channel 2 split over their bits 10..15:
    the layout include/sff.h documents)."""
    H, W, C = S.shape
    n, P = 1 << level, 2 << level
    Hq, Wq = (H - 1) // P + 1, -(-((W - 1) // P + 4) // 16) * 16
    ey = np.arange(P * (Hq + 3)) - 3 * n
    ex = np.arange(P * Wq) - 3 * n
    Si = S.astype(np.int64)
    b = np.zeros((ey.size, ex.size, C), np.int64)
    for a in (0, n):
        for c in (0, n):
            b += Si[np.clip(ey + a, 0, H - 1)][:, np.clip(ex + c, 0, W - 1)]
    out = np.zeros((P, P, Hq, Wq, 4, C), np.uint16)
    for py in range(P):
        for px in range(P):
            for m in range(4):
                out[py, px, :, :, m] = b[(np.arange(Hq) + m) * P + py][:, np.arange(Wq) * P + px]
    if C == 3:
        b = out.astype(np.uint32)  # [..., m, c]
        c2 = b[..., 2]
        lo, hi = c2 & 0x3F, c2 >> 6
        w = np.empty(out.shape[:4] + (4,), np.uint32)
        w[..., 0] = b[..., 0, 0] | (b[..., 1, 0] << 16) | (lo[..., 0] << 10) | (lo[..., 1] << 26)
        w[..., 1] = b[..., 2, 0] | (b[..., 3, 0] << 16) | (hi[..., 0] << 10) | (hi[..., 1] << 26)
        w[..., 2] = b[..., 0, 1] | (b[..., 1, 1] << 16) | (lo[..., 2] << 10) | (lo[..., 3] << 26)
        w[..., 3] = b[..., 2, 1] | (b[..., 3, 1] << 16) | (hi[..., 2] << 10) | (hi[..., 3] << 26)
        return w
    return out


BIN_CASES = [("ragged_c3", 37, 53, 3, 3), ("c1_l2", 29, 71, 1, 3), ("c2", 20, 24, 2, 2),
             ("c4", 13, 40, 4, 2), ("one_pixel", 1, 1, 3, 2),
             # every tile shape of the plane kernel (P = 2 .. 32), several tiles a level
             ("c1_l5", 40, 300, 1, 5), ("c2_l4", 70, 150, 2, 4)]


@pytest.mark.parametrize("case", BIN_CASES, ids=[c[0] for c in BIN_CASES])
def test_wht_bins_layout(sff, case):
    """The bin-sum planes against the layout written out from the oracle's
    smoothed image; descriptors and planes from one call agree with the
    descriptors alone."""
    import torch
    name, H, W, C, levels = case
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    imgs = rng.integers(0, 256, (4, H, W, C), dtype=np.uint8)
    p = params_dict(H, W, C, levels=levels, iters=1)
    for lv in range(levels):
        _say("bins", name, "level", lv)
        nb = sff.sff_bin_bytes(p, lv)
        bins = torch.zeros(4 * nb, dtype=torch.uint8, device="cuda")
        d = host(sff.sff_wht_features(p, dev(imgs), lv, bins=bins))
        for m in range(4):
            S = imgs[m] if lv == 0 else oracle.smooth(imgs[m], 1 << lv)
            exp = _bins_expected(S, lv)
            g = host(bins)[m * nb:(m + 1) * nb].view(exp.dtype).reshape(exp.shape)
            assert np.array_equal(g, exp), (name, lv, m)
            assert np.array_equal(d[m][:, :, :C], oracle.features(imgs[m], lv)), (name, lv, m)
        only = host(sff.sff_wht_features(p, dev(imgs), lv, want_desc=False))
        assert np.array_equal(only, host(bins))


# ----------------------------------------------------------------- init ----
INIT_CASES = [
    # name, H, W, C, levels, fmax, dmax, seed
    ("tiny", 96, 160, 1, 1, 32, 32, 1),
    ("ragged_l2", 45, 77, 3, 2, 12, 10, 3),
    ("ragged_l3_c2", 50, 83, 2, 3, 20, 17, 4),
    ("c4_l1", 24, 40, 4, 1, 7, 9, 5),
    ("fmax0", 20, 30, 1, 1, 0, 0, 6),
]


def _init(sff, p, imgs_dev, maps, dir, leaves=1):
    """Initialisation of one pair from its descriptor records or bin planes."""
    top = p["levels"] - 1
    if maps == "desc":
        desc = sff.sff_wht_features(p, imgs_dev, top).view(1, 4, p["H"], p["W"],
                                                          sff.desc_channels(p["C"]), 16)
        return sff.sff_init_nn(p, desc, dir, leaves=leaves)
    bins = sff.sff_wht_features(p, imgs_dev, top, want_desc=False)
    return sff.sff_init_nn_bins(p, bins, 1, dir, leaves=leaves)


@pytest.mark.parametrize("maps", ["desc", "bins"])
@pytest.mark.parametrize("leaves", [1, 2, 4])
@pytest.mark.parametrize("case", INIT_CASES, ids=[c[0] for c in INIT_CASES])
def test_init_nn_parity(sff, case, leaves, maps):
    """Descriptor-record (int8 MFMA) and bin-plane (fp16 MFMA) initialisation
    against the oracle's exact nearest neighbours."""
    name, H, W, C, levels, fmax, dmax, seed = case
    sc = make_scene(small_spec(H, W, C, seed, flow_max=min(fmax, 10), d_range=(0, min(dmax, 10))))
    p = params_dict(H, W, C, levels=levels, iters=1, fmax=fmax, dmax=dmax)
    top = levels - 1
    imgs = sc.stack()
    D = _oracle_descs(imgs, top)
    _say("init", name, maps, "leaves", leaves, "both directions")
    hyp, cost = _init(sff, p, dev(imgs), maps, sff.DIR_BOTH, leaves)
    h, c = host(hyp), host(cost, u32=True)
    for di, s in enumerate((1, -1)):
        oh, oc = oracle.init_nn(D, top, s, fmax, dmax, leaves=leaves)
        assert np.array_equal(h[di, 0], oh), (name, s)
        assert np.array_equal(c[di, 0], oc), (name, s)
    _say("init", name, maps, "leaves", leaves, "single directions")
    for s in (1, -1):
        hyp1, cost1 = _init(sff, p, dev(imgs), maps, s, leaves)
        assert np.array_equal(host(hyp1)[0, 0], h[0 if s > 0 else 1, 0])
        assert np.array_equal(host(cost1, u32=True)[0, 0], c[0 if s > 0 else 1, 0])


def test_init_bins_extreme_contrast(sff):
    """Bin values at both ends (0 and 1020 after the 2x2 sums) on every
    channel: the fp16 products and their fp32 sums stay exact (C = 4, the
    largest K)."""
    H, W, C = 24, 48, 4
    rng = np.random.default_rng(9)
    imgs = (rng.integers(0, 2, (4, H, W, C)) * 255).astype(np.uint8)
    p = params_dict(H, W, C, levels=1, iters=1, fmax=12, dmax=10)
    D = _oracle_descs(imgs, 0)
    _say("init bins extreme contrast")
    hyp, cost = _init(sff, p, dev(imgs), "bins", sff.DIR_BOTH)
    for di, s in enumerate((1, -1)):
        oh, oc = oracle.init_nn(D, 0, s, 12, 10)
        assert np.array_equal(host(hyp)[di, 0], oh)
        assert np.array_equal(host(cost, u32=True)[di, 0], oc)


def test_init_bins_large_keys(sff):
    """Bright references against dark targets (views 0, 3 near 255, views 1, 2
    near 0, small noise): every temporal key |a - b|^2 - |a'|^2 is far above
    2^24, where fp32 keys round, so the scan must fall back to int32 keys; the
    noise makes neighbouring keys differ by a few units."""
    H, W, C = 24, 40, 4
    rng = np.random.default_rng(21)
    imgs = rng.integers(0, 4, (4, H, W, C)).astype(np.uint8)
    imgs[0] = 255 - imgs[0]
    imgs[3] = 255 - imgs[3]
    p = params_dict(H, W, C, levels=1, iters=1, fmax=12, dmax=10)
    D = _oracle_descs(imgs, 0)
    _say("init bins large keys")
    hyp, cost = _init(sff, p, dev(imgs), "bins", sff.DIR_BOTH)
    for di, s in enumerate((1, -1)):
        oh, oc = oracle.init_nn(D, 0, s, 12, 10)
        assert np.array_equal(host(hyp)[di, 0], oh)
        assert np.array_equal(host(cost, u32=True)[di, 0], oc)


@pytest.mark.parametrize("maps", ["desc", "bins"])
def test_init_nn_kitti_full(sff, maps):
    sc = make_scene(kitti_spec())
    p = kitti_params()
    imgs = sc.stack()
    top = p["levels"] - 1
    _say("init kitti", maps)
    hyp, cost = _init(sff, p, dev(imgs), maps, sff.DIR_BOTH)
    D = _oracle_descs(imgs, top)
    for di, s in enumerate((1, -1)):
        oh, oc = oracle.init_nn(D, top, s, p["fmax"], p["dmax"])
        assert np.array_equal(host(hyp)[di, 0], oh)
        assert np.array_equal(host(cost, u32=True)[di, 0], oc)


# ---------------------------------------------------------- match level ----
LEVEL_CASES = [
    # name, H, W, C, levels, level, iters, rs_samples, batch
    ("top_tiny", 96, 160, 1, 1, 0, 4, 6, 1),
    ("top_ragged_l2", 45, 77, 3, 3, 2, 3, 6, 2),
    ("handoff_l1", 45, 77, 3, 3, 1, 2, 6, 2),
    ("handoff_l0_c2", 38, 61, 2, 2, 0, 3, 4, 1),
    ("handoff_only", 38, 61, 1, 2, 0, 0, 6, 1),
    ("no_search", 30, 50, 1, 1, 0, 3, 0, 3),
    ("odd_sizes", 17, 9, 2, 2, 1, 5, 6, 1),
    ("c4_handoff", 29, 53, 4, 2, 0, 2, 6, 1),
    ("wide_c3", 11, 300, 3, 1, 0, 2, 6, 1),
    # sample counts that are not multiples of the cooperative group of three
    ("rs5_c3", 33, 70, 3, 1, 0, 2, 5, 1),
    ("rs1", 20, 40, 1, 2, 0, 2, 1, 2),
]


MATCH_KERNELS = [("desc", "lane"), ("desc", "coop-narrow"), ("desc", "coop-wide"),
                 ("desc", "coop-narrow-32"), ("desc", "coop-wide-32"),
                 ("bins", "lane"), ("bins", "coop"), ("bins", "coop-32"), ("bins", "coop-43-32"),
                 ("bins", "coop-46-32"), ("bins", "coop-xts"), ("bins", "coop-46-16-xts"),
                 # the two fields on two streams (forced; by default only for large launches)
                 ("bins", "coop-xts+split"), ("bins", "coop-46-16-xts+split"), ("bins", "lane+split")]


@pytest.mark.parametrize("kernel", MATCH_KERNELS, ids=[f"{a}-{b}" for a, b in MATCH_KERNELS])
@pytest.mark.parametrize("case", LEVEL_CASES, ids=[c[0] for c in LEVEL_CASES])
def test_match_level_parity(sff, case, kernel, monkeypatch):
    """Every gather kernel against the oracle: descriptor records (per-lane;
    wave-cooperative scoring 2 neighbours and 3 samples, or 4 and 3, at a
    time, with 64 or 32 pixels per wave) and bin-sum planes (per-lane;
    cooperative with 64, 32 or 16 pixels per wave, one view a round with the
    early-out between views or all three views in one round); SFF_MATCH_EVAL
    forces one, SFF_MATCH_SPLIT=1 the two fields on two streams."""
    import torch
    maps, evaluator = kernel
    evaluator, _, split = evaluator.partition("+")
    monkeypatch.setenv("SFF_MATCH_EVAL", evaluator)
    monkeypatch.setenv("SFF_MATCH_SPLIT", "1" if split else "0")
    name, H, W, C, levels, level, iters, rs, B = case
    fmax, dmax = 16, 12
    p = params_dict(H, W, C, levels=levels, iters=iters, rs_samples=rs, fmax=fmax, dmax=dmax)
    scenes = [make_scene(small_spec(H, W, C, 100 + 7 * b, flow_max=8, d_range=(0, 10)))
              for b in range(B)]
    imgs = _imgs_stack(scenes)
    seeds = np.array([11 + 1000003 * b for b in range(B)], np.int64)
    flat = dev(imgs.reshape(4 * B, H, W, C))
    if maps == "desc":
        desc_l = sff.sff_wht_features(p, flat, level).view(B, 4, H, W, sff.desc_channels(C), 16)
        match = sff.sff_match_level
    else:
        desc_l = sff.sff_wht_features(p, flat, level, want_desc=False)
        match = sff.sff_match_level_bins
    Dl = [_oracle_descs(imgs[b], level) for b in range(B)]
    if level < levels - 1:
        # a coarse field: oracle init at the next level (both sides get the same input)
        Dc = [_oracle_descs(imgs[b], level + 1) for b in range(B)]
        coarse = np.stack([np.stack([oracle.init_nn(Dc[b], level + 1, s, fmax, dmax)[0]
                                     for b in range(B)]) for s in (1, -1)])
        _say("match_level", name, maps, evaluator, "hand-off")
        hyp, cost = match(p, desc_l, sff.DIR_BOTH, level, dev(seeds), hyp_coarse=dev(coarse))
        for di, s in enumerate((1, -1)):
            for b in range(B):
                oh, oc = oracle.match_level(Dl[b], level, s, int(seeds[b]), iters, 32, rs, fmax,
                                            dmax, None, None, hyp_coarse=coarse[di, b])
                assert np.array_equal(host(hyp)[di, b], oh), (name, s, b)
                assert np.array_equal(host(cost, u32=True)[di, b], oc), (name, s, b)
    else:
        start = np.stack([np.stack([oracle.init_nn(Dl[b], level, s, fmax, dmax)[0]
                                    for b in range(B)]) for s in (1, -1)])
        startc = np.stack([np.stack([oracle.init_nn(Dl[b], level, s, fmax, dmax)[1]
                                     for b in range(B)]) for s in (1, -1)])
        _say("match_level", name, maps, evaluator, "from init")
        hyp = dev(start)
        cost = dev(startc.view(np.int32))
        match(p, desc_l, sff.DIR_BOTH, level, dev(seeds), hyp, cost)
        for di, s in enumerate((1, -1)):
            for b in range(B):
                oh, oc = oracle.match_level(Dl[b], level, s, int(seeds[b]), iters, 32, rs, fmax,
                                            dmax, start[di, b], startc[di, b])
                assert np.array_equal(host(hyp)[di, b], oh), (name, s, b)
                assert np.array_equal(host(cost, u32=True)[di, b], oc), (name, s, b)
        # one direction at a time gives the same fields
        for di, s in enumerate((1, -1)):
            h1 = dev(start[di:di + 1])
            c1 = dev(startc[di:di + 1].view(np.int32))
            match(p, desc_l, s, level, dev(seeds), h1, c1)
            assert np.array_equal(host(h1)[0], host(hyp)[di])
    torch.cuda.synchronize()


# ---------------------------------------------------------- consistency ----
def test_consistency_parity(sff):
    rng = np.random.default_rng(12)
    H, W, B = 41, 67, 3
    p = params_dict(H, W, 1, levels=1, iters=1, fmax=20, dmax=15, tau=1)
    fwd = np.empty((B, H, W, 4), np.int16)
    inv = np.empty((B, H, W, 4), np.int16)
    for arr in (fwd, inv):
        arr[..., :2] = rng.integers(-20, 21, (B, H, W, 2))
        arr[..., 2:] = rng.integers(0, 16, (B, H, W, 2))
    # make a share of pixels exactly or nearly consistent
    sc = make_scene(small_spec(H, W, 1, 77, flow_max=6, d_range=(0, 8), delta_max=2))
    fwd[0] = sc.gt_fwd
    inv[0] = np.where(sc.inv_mask[..., None], sc.gt_inv, inv[0])
    for tau in (0, 1, 3):
        p["tau"] = tau
        _say("consistency tau", tau)
        valid, err = sff.sff_consistency(p, dev(fwd), dev(inv))
        for b in range(B):
            ov, oe = oracle.consistency(fwd[b], inv[b], tau)
            assert np.array_equal(host(valid)[b], ov)
            assert np.array_equal(host(err, u32=True)[b], oe)
    assert host(valid)[0].mean() > 0.3


# ---------------------------------------------------------- whole stage ----
def _check_pipeline(sff, scenes, p, seeds, stream=None, maps="bins"):
    import torch
    B = len(scenes)
    imgs = _imgs_stack(scenes)
    m = sff.PairMatcher(p, B, maps=maps)
    out = m.run(dev(imgs), dev(np.array(seeds, np.int64)), stream)
    if stream is not None:
        stream.synchronize()
    torch.cuda.synchronize()
    hyp, cost = host(out["hyp"]), host(out["cost"], u32=True)
    valid, err = host(out["valid"]), host(out["err"], u32=True)
    for b in range(B):
        ref = oracle.match_pair(imgs[b], p, int(seeds[b]))
        assert np.array_equal(hyp[:, b], ref["hyp"]), b
        assert np.array_equal(cost[:, b], ref["cost"]), b
        assert np.array_equal(valid[b], ref["valid"]), b
        assert np.array_equal(err[b], ref["err"]), b
    return out


def test_pipeline_tiny(sff):
    _say("pipeline tiny")
    _check_pipeline(sff, [make_scene(tiny_spec())], tiny_params(), [1])


@pytest.mark.parametrize("split", ["auto", "1"])
def test_pipeline_ragged_batch_on_side_stream(sff, split, monkeypatch):
    """The whole stage on a stream other than the current one; with the two
    fields on two streams forced at every level, the helper stream must wait
    for the features and init on that stream and the consistency check for it."""
    import torch
    if split != "auto":
        monkeypatch.setenv("SFF_MATCH_SPLIT", split)
    p = params_dict(53, 91, 3, levels=3, iters=3, fmax=24, dmax=20)
    scenes = [make_scene(small_spec(53, 91, 3, 300 + b, flow_max=12, d_range=(0, 16)))
              for b in range(3)]
    st = torch.cuda.Stream()
    _say("pipeline ragged batch 3 on side stream, split", split)
    with torch.cuda.stream(st):
        _check_pipeline(sff, scenes, p, [5, 6, 7], stream=st)


def test_pipeline_graph_replay(sff, monkeypatch):
    """The whole stage captured in a HIP graph (the two fields of every level
    on two streams, forced, so the helper stream joins the capture) and
    replayed three times, with eager work and synchronisations between the
    replays: every replay equals the eager run, which equals the oracle."""
    import torch
    monkeypatch.setenv("SFF_MATCH_SPLIT", "1")
    p = params_dict(53, 91, 3, levels=3, iters=2, fmax=24, dmax=20)
    scenes = [make_scene(small_spec(53, 91, 3, 700 + b, flow_max=12, d_range=(0, 16))) for b in range(2)]
    _say("pipeline graph replay, split forced")
    out = _check_pipeline(sff, scenes, p, [8, 9])
    m = sff.PairMatcher(p, 2)
    imgs = dev(_imgs_stack(scenes))
    seeds = dev(np.array([8, 9], np.int64))
    m.run(imgs, seeds)  # eager first: the library's helper stream exists before capture
    torch.cuda.synchronize()
    ref = {k: host(v).copy() for k, v in out.items() if k in ("hyp", "cost", "valid", "err")}
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            m.run(imgs, seeds, stream=s)
    torch.cuda.synchronize()
    for i in range(3):
        m.hyp[0].zero_()
        m.valid.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in ref:
            v = {"hyp": m.hyp[0], "cost": m.cost[0], "valid": m.valid, "err": m.err}[k]
            assert np.array_equal(host(v), ref[k]), (i, k)


PIPE_KERNELS = [("bins", "auto"), ("bins", "auto+nosplit"), ("bins", "lane"), ("bins", "coop"),
                ("bins", "coop-32"),
                ("bins", "coop-43-32"), ("bins", "coop-46-32"), ("bins", "coop-xts"),
                ("bins", "coop-46-16-xts"),
                ("desc", "auto"), ("desc", "lane"), ("desc", "coop-narrow"), ("desc", "coop-wide"),
                ("desc", "coop-narrow-32"), ("desc", "coop-wide-32")]


@pytest.mark.parametrize("kernel", PIPE_KERNELS, ids=[f"{a}-{b}" for a, b in PIPE_KERNELS])
def test_pipeline_kitti_full(sff, kernel, monkeypatch):
    """The KITTI-size pair end to end against the oracle with every gather
    kernel; by default levels 0 and 1 run the two fields on two streams,
    "+nosplit" runs them in one launch sequence."""
    maps, evaluator = kernel
    evaluator, _, split = evaluator.partition("+")
    monkeypatch.setenv("SFF_MATCH_EVAL", evaluator)
    if split:
        monkeypatch.setenv("SFF_MATCH_SPLIT", "0")
    _say("pipeline kitti 1242x375", maps, evaluator)
    _check_pipeline(sff, [make_scene(kitti_spec())], kitti_params(), [2], maps=maps)


def test_invalid_batch_raises(sff):
    import torch
    p = tiny_params()
    img = torch.zeros((0, 96, 160, 1), dtype=torch.uint8, device="cuda")
    with pytest.raises(sff.SffError):
        sff.sff_wht_features(p, img, 0, torch.zeros((0, 96, 160, 1, 16), dtype=torch.int16,
                                                   device="cuda"))


def test_pipeline_batch16_small(sff):
    """Sixteen 96x160 pairs with distinct seeds in one batch (two levels)."""
    B, H, W, C = 16, 96, 160, 1
    p = params_dict(H, W, C, levels=2, iters=2, fmax=16, dmax=12)
    scenes = [make_scene(small_spec(H, W, C, 500 + b, flow_max=8, d_range=(0, 10))) for b in range(B)]
    imgs = _imgs_stack(scenes)
    seeds = np.arange(B, dtype=np.int64) * 7919 + 3
    _say("pipeline batch 16, 96x160")
    out = sff.PairMatcher(p, B).run(dev(imgs), dev(seeds))
    hyp, cost = host(out["hyp"]), host(out["cost"], u32=True)
    valid, err = host(out["valid"]), host(out["err"], u32=True)
    for b in range(B):
        ref = oracle.match_pair(imgs[b], p, int(seeds[b]))
        assert np.array_equal(hyp[:, b], ref["hyp"]), b
        assert np.array_equal(cost[:, b], ref["cost"]), b
        assert np.array_equal(valid[b], ref["valid"]), b
        assert np.array_equal(err[b], ref["err"]), b


def test_pipeline_kitti_batch16(sff):
    """Sixteen KITTI-like pairs (per-pair seeds, flow <= 64 for pairs 0-7 and
    <= 256 for 8-15) in one batch, every pair against the oracle."""
    from sff_inputs import kitti_batch_specs
    specs = kitti_batch_specs()
    scenes = [make_scene(s) for s in specs]
    _say("pipeline kitti batch 16")
    _check_pipeline(sff, scenes, kitti_params(), [s.seed for s in specs])


def test_pipeline_kitti_leaves4(sff):
    """The whole stage with four temporal leaves at the KITTI size."""
    import torch
    sc = make_scene(kitti_spec())
    p = kitti_params()
    _say("pipeline kitti leaves 4")
    out = sff.PairMatcher(p, 1, leaves=4).run(dev(sc.stack()[None]), dev(np.array([2], np.int64)))
    torch.cuda.synchronize()
    ref = oracle.match_pair(sc.stack(), p, 2, leaves=4)
    assert np.array_equal(host(out["hyp"])[:, 0], ref["hyp"])
    assert np.array_equal(host(out["cost"], u32=True)[:, 0], ref["cost"])
    assert np.array_equal(host(out["valid"])[0], ref["valid"])

