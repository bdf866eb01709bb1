"""The allocation-free features entry point (fixed device scratch) against
sff_wht_features with a caller workspace: descriptors and bin-sum planes
bit-identical on two calls in a row, the second with a smaller input, and
requests beyond the scratch rejected before any launch."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def test_noalloc_features_match_workspace_call():
    import torch
    import paper_1710_10096_amd as sff
    from paper_1710_10096_amd._native import lib
    from paper_1710_10096_amd.api import _params
    from sff_inputs import params_dict
    assert torch.cuda.is_available()
    L = lib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rng = np.random.default_rng(77)
    # second call smaller than the first; both at a smoothed level and level 0
    for (nimg, H, W, C, level) in [(8, 375, 1242, 3, 2), (3, 41, 67, 3, 1), (4, 96, 160, 1, 0)]:
        _say("noalloc", nimg, H, W, C, "level", level)
        p = params_dict(H, W, C, levels=3, iters=1)
        pp = _params(p)
        img = torch.from_numpy(rng.integers(0, 256, (nimg, H, W, C), dtype=np.uint8)).cuda()
        Cp = sff.desc_channels(C)
        nb = sff.sff_bin_bytes(p, level)
        want_desc = sff.sff_wht_features(p, img, level)
        want_bins = sff.sff_wht_features(p, img, level, want_desc=False)
        desc = torch.full((nimg, H, W, Cp, 16), 0x5A5A, dtype=torch.int16, device="cuda")
        bins = torch.zeros(nimg * nb, dtype=torch.uint8, device="cuda")
        rc = L.sff_wht_features_noalloc(ctypes.byref(pp), nimg, level,
                                        ctypes.c_void_p(img.data_ptr()),
                                        ctypes.c_void_p(desc.data_ptr()),
                                        ctypes.c_void_p(bins.data_ptr()), st)
        assert rc == 0, rc
        torch.cuda.synchronize()
        assert torch.equal(desc[..., :C, :], want_desc[..., :C, :])
        assert torch.equal(bins, want_bins)


def test_noalloc_rejects_oversize_requests():
    import torch
    from paper_1710_10096_amd._native import lib
    from paper_1710_10096_amd.api import _params
    from sff_inputs import params_dict
    L = lib()
    cap = L.sff_wht_scratch_bytes()
    assert cap == 32 << 20
    # 64 images of 375 x 1242 x 3 at level 1 need ~90 MB of scratch
    p = _params(params_dict(375, 1242, 3, levels=2, iters=1))
    dummy = torch.zeros(16, dtype=torch.uint8, device="cuda")
    f = ctypes.c_void_p(dummy.data_ptr())
    assert L.sff_wht_features_noalloc(ctypes.byref(p), 64, 1, f, f, None, None) == 4
