"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol include/sff.h declares, and rejects bad arguments on the host before
touching the device."""
import ctypes
import os
import re

import pytest

from paper_1710_10096_amd import _native
from paper_1710_10096_amd._native import SffParams

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gpu_visible():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


# The argument checks below pass fake device addresses that validation must
# reject; they are host-logic tests and never run where a GPU is visible.
host_only = pytest.mark.skipif(_gpu_visible(), reason="host-only validation test (fake pointers)")


def declared_symbols():
    names = []
    for f in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            # declarations: lines outside comment blocks naming sff_* before "("
            names += re.findall(r"^(?!\s*(?:/\*|\*))[^\n;(]*?\b(sff_[a-z0-9_]+)\s*\(", txt,
                                re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = _native.lib()
    decl = declared_symbols()
    assert len(decl) >= 8
    for name in decl:
        assert hasattr(L, name), name
    assert set(_native.EXPORTS) <= set(decl)


def test_params_struct_matches_header():
    txt = open(os.path.join(ROOT, "include", "sff.h")).read()
    body = txt[txt.index("typedef struct sff_params"):txt.index("} sff_params;")]
    fields = re.findall(r"(\w+)(?=[,;])", re.sub(r"/\*.*?\*/", "", body, flags=re.S))
    fields = [f for f in fields if f not in ("int32_t",)]
    assert fields == [n for n, _ in SffParams._fields_]
    assert ctypes.sizeof(SffParams) == 40


def test_status_strings_and_version():
    L = _native.lib()
    assert L.sff_status_string(0) == b"ok"
    assert L.sff_status_string(1) == b"invalid argument"
    assert L.sff_status_string(99) == b"unknown status"
    assert L.sff_version() >= 300


def test_descriptor_record_channels():
    """Records are padded to a power-of-two channel count (32/64/128 bytes)."""
    L = _native.lib()
    assert [L.sff_desc_channels(c) for c in range(6)] == [0, 1, 2, 4, 4, 0]


def test_bin_plane_sizes():
    """Bytes of one image's bin-sum planes: P^2 planes of Hq x Wq entries of
    8 C bytes (16 for C = 3, whose bins are packed in one word), P =
    2^(level+1), Hq = (H-1)/P + 1, Wq = (W-1)/P + 4 rounded up to 16 (the
    layout include/sff.h documents)."""
    L = _native.lib()
    for H, W, C, lv in ((375, 1242, 3, 0), (375, 1242, 3, 2), (1, 1, 1, 0), (29, 71, 2, 3)):
        p = SffParams(H=H, W=W, C=C, levels=lv + 1, iters=1, rs_r0=32, rs_samples=6, fmax=8,
                      dmax=8, tau=1)
        P = 2 << lv
        Hq, Wq = (H - 1) // P + 1, -(-((W - 1) // P + 4) // 16) * 16
        entry = 16 if C == 3 else 8 * C
        assert L.sff_bin_bytes(ctypes.byref(p), lv) == P * P * Hq * Wq * entry
        assert L.sff_bin_bytes(ctypes.byref(p), lv + 1) == 0


def _good():
    return SffParams(H=96, W=160, C=1, levels=1, iters=4, rs_r0=32, rs_samples=6, fmax=32, dmax=32,
                     tau=1)


BAD = [dict(H=0), dict(W=-1), dict(C=0), dict(C=5), dict(levels=0), dict(levels=6),
       dict(iters=-1), dict(rs_samples=17), dict(rs_r0=0), dict(fmax=9000), dict(dmax=-1),
       dict(tau=-2), dict(H=20000)]


@host_only
@pytest.mark.parametrize("bad", BAD)
def test_invalid_params_rejected_without_launch(bad):
    L = _native.lib()
    p = _good()
    for k, v in bad.items():
        setattr(p, k, v)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert L.sff_wht_features(ctypes.byref(p), 1, 0, fake, fake, fake, None, 0, None) == 1
    assert L.sff_init_nn(ctypes.byref(p), 1, 0, fake, fake, fake, fake, 1 << 30, None) == 1
    assert L.sff_init_workspace_bytes(ctypes.byref(p), 1) == 0
    assert L.sff_init_bins_workspace_bytes(ctypes.byref(p), 1) == 0
    assert L.sff_init_nn_bins(ctypes.byref(p), 1, 0, 1, fake, fake, fake, fake, 1 << 30, None) == 1
    assert L.sff_match_level(ctypes.byref(p), 1, 0, 0, fake, fake, None, fake, fake, None) == 1
    assert L.sff_match_level_bins(ctypes.byref(p), 1, 0, 0, fake, fake, None, fake, fake, None) == 1
    assert L.sff_bin_bytes(ctypes.byref(p), 0) == 0
    assert L.sff_consistency(ctypes.byref(p), 1, fake, fake, fake, fake, None) == 1
    assert L.sff_wht_workspace_bytes(ctypes.byref(p), 4, 0) == 0


@host_only
def test_invalid_arguments_rejected():
    L = _native.lib()
    p = _good()
    P = ctypes.byref(p)
    f = ctypes.c_void_p(0x1000)
    # null pointers
    assert L.sff_wht_features(P, 1, 0, None, f, None, None, 0, None) == 1
    assert L.sff_wht_features(P, 1, 0, f, None, None, None, 0, None) == 1      # neither output
    assert L.sff_wht_features(P, 1, 0, f, None, ctypes.c_void_p(0x1008), None, 0, None) == 1  # bins misaligned
    assert L.sff_match_level_bins(P, 1, 0, 0, None, f, None, f, f, None) == 1
    assert L.sff_match_level_bins(P, 1, 0, 0, ctypes.c_void_p(0x1008), f, None, f, f, None) == 1
    assert L.sff_match_level_bins(P, 1, 0, 1, f, f, None, f, f, None) == 1  # level >= levels
    assert L.sff_match_level_bins(P, 1, 0, 0, f, f, f, f, f, None) == 1     # hand-off at top
    assert L.sff_init_nn(P, 1, 0, f, None, f, f, 1 << 30, None) == 1
    assert L.sff_match_level(P, 1, 0, 0, f, None, None, f, f, None) == 1
    assert L.sff_consistency(P, 1, f, f, None, f, None) == 1
    # bad batch / direction / level
    assert L.sff_init_nn(P, 0, 0, f, f, f, f, 1 << 30, None) == 1
    assert L.sff_init_nn(P, 1, 2, f, f, f, f, 1 << 30, None) == 1
    assert L.sff_match_level(P, 1, 0, 1, f, f, None, f, f, None) == 1      # level >= levels
    assert L.sff_match_level(P, 1, 0, 0, f, f, f, f, f, None) == 1         # hand-off at top
    assert L.sff_wht_features(P, 1, 1, f, f, None, None, 0, None) == 1    # level >= levels
    # bin-plane initialisation
    need_b = L.sff_init_bins_workspace_bytes(P, 1)
    assert need_b > 0 and L.sff_init_bins_workspace_bytes(P, 0) == 0
    assert L.sff_init_nn_bins(P, 1, 0, 1, None, f, f, f, need_b, None) == 1
    assert L.sff_init_nn_bins(P, 1, 2, 1, f, f, f, f, need_b, None) == 1             # dir 2
    assert L.sff_init_nn_bins(P, 1, 0, 3, f, f, f, f, need_b, None) == 2             # leaves 3
    assert L.sff_init_nn_bins(P, 1, 0, 1, ctypes.c_void_p(0x1008), f, f, f, need_b, None) == 1
    assert L.sff_init_nn_bins(P, 1, 0, 1, f, f, f, f, need_b - 1, None) == 4
    assert L.sff_init_nn_bins(P, 1, 0, 1, f, f, f, ctypes.c_void_p(0x1010), need_b, None) == 4
    # temporal leaves: 1, 2 or 4
    need_i = L.sff_init_workspace_bytes(P, 1)
    assert L.sff_init_nn_leaves(P, 1, 0, 0, f, f, f, f, need_i, None) == 1
    assert L.sff_init_nn_leaves(P, 1, 0, 3, f, f, f, f, need_i, None) == 2
    assert L.sff_init_nn_leaves(P, 1, 0, 8, f, f, f, f, need_i, None) == 2
    # misaligned descriptor pointer
    assert L.sff_init_nn(P, 1, 0, ctypes.c_void_p(0x1002), f, f, f, 1 << 30, None) == 1
    # init workspace missing, too small or misaligned
    need = L.sff_init_workspace_bytes(P, 1)
    assert need > 0
    assert L.sff_init_nn(P, 1, 0, f, f, f, None, need, None) == 4
    assert L.sff_init_nn(P, 1, 0, f, f, f, f, need - 1, None) == 4
    assert L.sff_init_nn(P, 1, 0, f, f, f, ctypes.c_void_p(0x1010), need, None) == 4
    # workspace missing at level >= 1
    p2 = _good()
    p2.levels = 3
    need = L.sff_wht_workspace_bytes(ctypes.byref(p2), 4, 1)
    assert need > 0
    assert L.sff_wht_workspace_bytes(ctypes.byref(p2), 4, 0) == 0
    assert L.sff_wht_features(ctypes.byref(p2), 4, 1, f, f, None, None, 0, None) == 4
    assert L.sff_wht_features(ctypes.byref(p2), 4, 1, f, f, None, f, need - 1, None) == 4
    assert L.sff_wht_features(ctypes.byref(p2), 4, 1, f, None, f, f, need - 1, None) == 4
    # region filter and sparsification
    need = L.sff_region_workspace_bytes(P, 1)
    assert need == 3 * ((96 * 160 * 4 + 255) // 256 * 256)
    assert L.sff_region_workspace_bytes(P, 0) == 0
    assert L.sff_region_filter(P, 1, 0, f, f, f, f, need, None) == 1        # s_c < 1
    assert L.sff_region_filter(P, 1, 150, None, f, f, f, need, None) == 1
    assert L.sff_region_filter(P, 1, 150, ctypes.c_void_p(0x1004), f, f, f, need, None) == 1
    assert L.sff_region_filter(P, 1, 150, f, f, f, f, need - 1, None) == 4
    assert L.sff_region_filter(P, 1, 150, f, f, f, ctypes.c_void_p(0x1010), need, None) == 4
    assert L.sff_sparsify(P, 1, f, f, None, None) == 1
    assert L.sff_sparsify(P, 0, f, f, f, None) == 1
    assert L.sff_sparsify(P, 1, f, ctypes.c_void_p(0x1002), f, None) == 1
    # SGM disparity and fill
    need_s = L.sff_sgm_workspace_bytes(P, 1)
    assert need_s > 0
    assert L.sff_sgm_disparity(P, 1, f, f, 0, 5, 3, f, f, need_s, None) == 1      # P2 < P1
    assert L.sff_sgm_disparity(P, 1, f, f, 0, 3, 232, f, f, need_s, None) == 1    # P2 > 231
    assert L.sff_sgm_disparity(P, 2, f, f, 16, 3, 24, f, f, need_s, None) == 1   # stride < image
    assert L.sff_sgm_disparity(P, 1, f, f, 0, 3, 24, f, f, need_s - 1, None) == 4
    p4 = _good()
    p4.dmax = 300
    assert L.sff_sgm_disparity(ctypes.byref(p4), 1, f, f, 0, 3, 24, f, f, 1 << 40, None) == 2
    assert L.sff_disparity_fill(P, 1, f, f, None, f, None) == 1
    # SIFT-PCA features and cost
    need_f = L.sff_sift_workspace_bytes(P, 4)
    assert need_f > L.sff_sift_workspace_bytes(P, 1) > 0
    assert L.sff_sift_workspace_bytes(P, 0) == 0
    assert L.sff_dense_sift(P, 0, f, f, f, need_f, None) == 1
    assert L.sff_dense_sift(P, 1, f, ctypes.c_void_p(0x1004), f, need_f, None) == 1   # sift not 16-B aligned
    assert L.sff_dense_sift(P, 4, f, f, f, need_f - 1, None) == 4
    assert L.sff_dense_sift(P, 4, f, f, ctypes.c_void_p(0x1010), need_f, None) == 4
    assert L.sff_sift_pca(P, 1, f, f, f, f, None, f, f, need_f, None) == 1
    assert L.sff_sift_pca(P, 1, f, f, f, f, f, ctypes.c_void_p(0x1008), f, need_f, None) == 1
    assert L.sff_sift_pca(P, 1, f, ctypes.c_void_p(0x1004), f, f, f, f, f, need_f, None) == 1
    assert L.sff_sift_pca(P, 1, f, f, f, f, f, f, f, need_f - 1, None) == 4
    assert L.sff_sift_pca(P, 2, f, f, f, f, f, f, f, need_f, None) == 4          # sized for one pair
    assert L.sff_cost_sift(P, 1, 0, f, f, f, None) == 1                          # dir 0
    assert L.sff_cost_sift(P, 1, 1, ctypes.c_void_p(0x1008), f, f, None) == 1    # phi not 16-B aligned
    assert L.sff_cost_sift(P, 0, 1, f, f, f, None) == 1
    assert L.sff_match_sift(P, 1, 2, f, f, 1, f, f, None) == 1                   # dir 2
    assert L.sff_match_sift(P, 1, 0, f, f, -1, f, f, None) == 1                  # iters < 0
    assert L.sff_match_sift(P, 1, 0, f, None, 1, f, f, None) == 1                # no seeds
    assert L.sff_match_sift(P, 1, 0, ctypes.c_void_p(0x1004), f, 1, f, f, None) == 1
    assert L.sff_sift_sqrt(None, f, 4, None) == 1
    assert L.sff_sift_sqrt(f, f, -1, None) == 1
    assert L.sff_sift_sqrt(ctypes.c_void_p(0x1002), f, 4, None) == 1            # in not 4-B aligned
    assert L.sff_sift_sqrt(f, f, (1 << 31) + 1, None) == 1
    assert L.sff_sift_sqrt(f, f, 0, None) == 0                                    # nothing to do
    # overlapping hand-off buffers
    p3 = _good()
    p3.levels = 2
    base = 0x100000
    assert L.sff_match_level(ctypes.byref(p3), 1, 0, 0, f, f, ctypes.c_void_p(base + 64),
                             ctypes.c_void_p(base), f, None) == 1
    assert L.sff_match_level_bins(ctypes.byref(p3), 1, 0, 0, f, f, ctypes.c_void_p(base + 64),
                                  ctypes.c_void_p(base), f, None) == 1


def test_lanczos_table_identical_to_oracle():
    import oracle
    from paper_1710_10096_amd import sff_lanczos_q14
    for n in (2, 4, 8, 16):
        assert sff_lanczos_q14(n) == oracle.lanczos_q14(n).tolist()
    L = _native.lib()
    buf = (ctypes.c_int32 * 6)()
    assert L.sff_lanczos_q14(1, ctypes.cast(buf, ctypes.c_void_p)) == 1
    assert L.sff_lanczos_q14(32, ctypes.cast(buf, ctypes.c_void_p)) == 1
