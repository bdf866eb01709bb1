/*
 * sff.h -- C ABI of libsff, the MI355X (gfx950) implementation of the sparse
 * scene-flow matching stage of SceneFlowFields (Schuster, Wasenmueller,
 * Kuschk, Bailer, Stricker; arXiv 1710.10096, Section 3.1 "Sparse
 * Correspondences").
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Array pointers are DEVICE pointers (HIP global memory) unless the comment
 *    says "host".  The caller allocates and owns every buffer; the library
 *    neither allocates device memory, nor keeps pointers after the call
 *    returns, nor synchronises.
 *  - All work is enqueued on `stream` (a hipStream_t; NULL = the default
 *    stream).  Results are ready when the stream reaches that point.
 *  - Arguments are checked on the host before anything is enqueued.  On an
 *    error the call returns a non-zero sff_status, enqueues nothing and leaves
 *    every output untouched.  A launch failure reported by the runtime after
 *    enqueueing returns SFF_ERR_HIP; faults inside kernels surface at the
 *    caller's next synchronisation.
 *  - The library is thread-safe.  Its state, per device, is the fixed scratch
 *    array of sff_wht_features_noalloc and one helper stream with two events
 *    (sff_match_level_bins, sff_cost_f32_bwd), created on first use and kept
 *    until the process ends.
 *
 * Data layouts (row-major)
 *  - image  uint8  [n][H][W][C]                 C = 1..4 channels
 *  - desc   int16  [n][H][W][Cp][16]            16 = 4x4 lowest-sequency WHT
 *                                                coefficients, index a*4 + b
 *                                                (a vertical, b horizontal);
 *    Cp = sff_desc_channels(C) = 1, 2, 4, 4 for C = 1..4: each pixel's record
 *    is padded to 32, 64 or 128 bytes so that it never straddles a 128-byte
 *    cache line.  Channels C..Cp-1 are never written nor read by the library.
 *  - bins   level-k bin-sum planes, sff_bin_bytes(p, k) bytes per image:
 *    the 2 x 2-bin sums the WHT descriptors are formed from.  The descriptor
 *    block is the 4-point Hadamard transform (both axes) of a pixel's 4 x 4
 *    grid of bin sums, so descriptor squared distances are exactly 16 times
 *    bin-grid squared distances.  Bin (i, j) of pixel (X, Y) sums the level-k
 *    image at X + n (2j - 3 + b), Y + n (2i - 3 + a), a, b in {0, 1}
 *    (replicated border).  With P = 2n, Hq = (H - 1) / P + 1 and Wq =
 *    ((W - 1) / P + 4) rounded up to a multiple of 16, an image is P * P
 *    planes (py * P + px) of Hq x Wq entries; entry (r, q) of plane (py, px)
 *    holds the bins at extended column q P + px and extended rows (r + m) P +
 *    py, m = 0..3 (extended coordinate = coordinate + 3n), in the order m,
 *    channel: C uint16 per bin, 8 C bytes per entry; for C = 3 the entry's
 *    bins b_m (10-bit channels b_m[c], at most 1020) are packed into four
 *    uint32 words: word 0 = b_0[0] | b_1[0] << 16, word 1 = b_2[0] | b_3[0] <<
 *    16, word 2 = b_0[1] | b_1[1] << 16, word 3 = b_2[1] | b_3[1] << 16, plus
 *    channel 2: the low 6 bits of b_0[2] and b_1[2] at bits 10 and 26 of word
 *    0 and their high 4 bits at bits 10 and 26 of word 1, b_2[2] and b_3[2]
 *    likewise in words 2 and 3 (16 bytes per entry).  The 4 x 4 grid of pixel (X, Y) is then the 4
 *    consecutive entries q = X / P .. + 3 of row Y / P of plane
 *    (Y mod P, X mod P): 4 entries of contiguous bytes.
 *  - the four views of a pair are stored consecutively in the canonical order
 *    (I_l^0, I_l^1, I_r^0, I_r^1); `batch` pairs make n = 4 * batch images.
 *  - hyp    int16  [ndir][batch][Hk][Wk][4]     (u, v, d0, d1), full-res px
 *  - cost   uint32 [ndir][batch][Hk][Wk]
 *    with level k, n = 2^k, Hk = ceil(H / n), Wk = ceil(W / n); ndir = 2 when
 *    dir = SFF_DIR_BOTH (forward field first), else 1.
 */
#ifndef SFF_H
#define SFF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SFF_OK = 0,
    SFF_ERR_INVALID_ARG = 1, /* bad pointer, size or parameter            */
    SFF_ERR_UNSUPPORTED = 2, /* valid but outside what this build handles */
    SFF_ERR_HIP = 3,         /* the HIP runtime reported an error         */
    SFF_ERR_WORKSPACE = 4    /* workspace missing or too small            */
} sff_status;

/* Direction of a field (Section 3.1, "Consistency Check"): the forward field
 * has reference I_l^0; the inverse field has reference I_r^1, with temporal
 * order and viewpoints swapped. */
enum { SFF_DIR_FORWARD = 1, SFF_DIR_INVERSE = -1, SFF_DIR_BOTH = 0 };

/* Matcher parameters.  Limits checked by every call:
 *   1 <= H, W <= 16384; 1 <= C <= 4; 1 <= levels <= 5; 0 <= iters <= 64;
 *   0 <= rs_samples <= 16; 1 <= rs_r0 <= 4096; 0 <= fmax, dmax <= 8192;
 *   0 <= tau <= 8192.                                                        */
typedef struct sff_params {
    int32_t H, W, C;    /* full-resolution image size and channel count       */
    int32_t levels;     /* pyramid levels K (k subscales + full resolution)   */
    int32_t iters;      /* propagation + random-search iterations per level   */
    int32_t rs_r0;      /* random-search radius of sample 0, in level pixels  */
    int32_t rs_samples; /* random-search samples per pixel and half-step      */
    int32_t fmax;       /* |u|, |v| <= fmax (full-res px)                     */
    int32_t dmax;       /* 0 <= d0, d1 <= dmax (full-res px)                  */
    int32_t tau;        /* consistency threshold tau_c in px (Section 5: 1)   */
} sff_params;

/* Human-readable text for a status code (static storage; never NULL). */
const char* sff_status_string(int32_t status);

/* Library ABI version (major * 10000 + minor * 100 + patch). */
int32_t sff_version(void);

/* Channels Cp of a stored descriptor record for C image channels: 1, 2, 4, 4
 * for C = 1..4; 0 for C outside 1..4. */
int32_t sff_desc_channels(int32_t C);

/* Host-only helper: the Q14 Lanczos-3 weights the smoothing uses for pyramid
 * factor n (2 <= n <= 16), table[p * 6 + t] for phase p = x mod n and tap t
 * at floor((x + 0.5) / n - 0.5) - 2 + t.  `table` is a HOST array of n * 6
 * int32.  Returns SFF_ERR_INVALID_ARG for a bad n or NULL table. */
sff_status sff_lanczos_q14(int32_t n, int32_t* table);

/* Device workspace (bytes) that sff_wht_features needs for `nimg` images at
 * `level`; 0 for level 0. */
size_t sff_wht_workspace_bytes(const sff_params* p, int32_t nimg, int32_t level);

/* Bytes of one image's bin-sum planes at `level` (layout above); 0 for bad
 * arguments. */
size_t sff_bin_bytes(const sff_params* p, int32_t level);

/* WHT feature vectors at one pyramid level (Section 3.1, "Initialization" --
 * WHT features; "Multi-Scale Propagation" -- scale simulation).
 *   For level k >= 1 each image is first smoothed: area-based downsampling by
 *   n = 2^k (rounded block mean, replicated border), then separable Lanczos-3
 *   upsampling back to H x W with Q14 weights (sff_lanczos_q14), each pass
 *   rounded, the second clamped to 0..255.  Level 0 uses the image itself.
 *   Then, at EVERY full-resolution pixel q and channel c, the 8x8 patch sampled
 *   every n-th pixel at offsets -3..+4 (replicated border) is transformed by
 *   the unnormalised 2-D Walsh-Hadamard transform and the 16 coefficients of
 *   vertical/horizontal sequency < 4 are stored (exact in int16).  The
 *   transform is taken in two stages, 2 x 2-bin sums then a 4-point Hadamard
 *   transform per axis; the first stage's sums can be written as bin-sum
 *   planes (layout above), from which sff_match_level_bins evaluates the
 *   descriptor distances.
 * img:  [nimg][H][W][C] uint8, read only.
 * desc: [nimg][H][W][Cp][16] int16, channels 0..C-1 written; or NULL.
 * bins: nimg images of sff_bin_bytes(p, level) bytes, written; or NULL.
 *   At least one of desc and bins; both 16-byte aligned.
 * workspace: device buffer of at least sff_wht_workspace_bytes(p, nimg, level)
 *   bytes (may be NULL at level 0); contents on entry are ignored.
 * Errors: SFF_ERR_INVALID_ARG (NULL pointers, nimg < 1, level outside
 *   0..levels-1, bad params), SFF_ERR_WORKSPACE (workspace too small),
 *   SFF_ERR_UNSUPPORTED (descriptors at level 4 with C >= 3). */
sff_status sff_wht_features(const sff_params* p, int32_t nimg, int32_t level, const uint8_t* img,
                            int16_t* desc, uint16_t* bins, void* workspace, size_t workspace_bytes,
                            void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * computation as sff_wht_features without a workspace argument.  The block
 * means and smoothed images of level >= 1 go to a fixed scratch array of
 * sff_wht_scratch_bytes() bytes (32 MiB) in device memory that the library
 * holds on each GPU it runs on until the process ends; its address on a
 * device is looked up on the first call with that device current.  Nothing
 * is allocated by the call.  Every call on one GPU shares that GPU's array
 * (the call writes all of the scratch it reads, so nothing needs clearing):
 * calls that overlap on one GPU (different streams, or different host threads
 * without ordering) race and must not be made.
 * Errors: as sff_wht_features; SFF_ERR_WORKSPACE when the call needs more
 *   than sff_wht_scratch_bytes() (nimg H W C plus the block means, each
 *   rounded up to 256 bytes, at level >= 1); SFF_ERR_HIP if the scratch's
 *   address cannot be obtained. */
size_t sff_wht_scratch_bytes(void);
sff_status sff_wht_features_noalloc(const sff_params* p, int32_t nimg, int32_t level,
                                    const uint8_t* img, int16_t* desc, uint16_t* bins,
                                    void* stream);

/* Device workspace (bytes) that sff_init_nn needs for `batch` pairs. */
size_t sff_init_workspace_bytes(const sff_params* p, int32_t batch);

/* Initialisation at the coarsest level k = levels - 1 (Section 3.1,
 * "Initialization"), read as exact nearest neighbours in descriptor space:
 * for every grid pixel p = (n j, n i), among grid targets (multiples of n)
 * inside the image,
 *   temporal partner: the box |u|, |v| <= fmax;
 *   stereo partner:   the same row (epipolar), 0 <= d0 <= dmax;
 *   cross partner:    row y + v*, 0 <= d1 <= dmax, target x + u* - s d1;
 * each the exact argmin of the descriptor SSD with ties to the smallest target
 * index y*W + x.  The combination is the hypothesis; its cost is eq. (1).
 * desc: level-(levels-1) descriptors [batch][4][H][W][Cp][16].
 * dir:  SFF_DIR_FORWARD, SFF_DIR_INVERSE or SFF_DIR_BOTH.
 * hyp/cost: coarsest-level field, written.
 * workspace: device buffer, 256-byte aligned, of at least
 *   sff_init_workspace_bytes(p, batch) bytes; contents on entry are ignored.
 * Errors: SFF_ERR_INVALID_ARG; SFF_ERR_WORKSPACE (missing, misaligned or too
 *   small workspace). */
sff_status sff_init_nn(const sff_params* p, int32_t batch, int32_t dir, const int16_t* desc,
                       int16_t* hyp, uint32_t* cost, void* workspace, size_t workspace_bytes,
                       void* stream);

/* The same initialisation with several leaves of the temporal search
 * (Section 3.1, "Initialization": all combinations of the leaves compared by
 * the data term).  The `leaves` temporal targets of smallest descriptor
 * distance (ties to the smaller target index) are each paired with their own
 * cross partner (argmin on row y + v) and with the stereo partner; the
 * combination with the smallest eq. (1) cost wins, ties to the earlier
 * temporal leaf.  (Eq. (1) is a sum over the three views, so more stereo or
 * cross leaves could not change the winner.)  leaves = 1 is sff_init_nn.
 * leaves: 1, 2 or 4.  Other arguments as sff_init_nn.
 * Errors: as sff_init_nn; SFF_ERR_INVALID_ARG for leaves < 1,
 *   SFF_ERR_UNSUPPORTED for other values. */
sff_status sff_init_nn_leaves(const sff_params* p, int32_t batch, int32_t dir, int32_t leaves,
                              const int16_t* desc, int16_t* hyp, uint32_t* cost, void* workspace,
                              size_t workspace_bytes, void* stream);

/* Device workspace (bytes) that sff_init_nn_bins needs for `batch` pairs. */
size_t sff_init_bins_workspace_bytes(const sff_params* p, int32_t batch);

/* The initialisation of sff_init_nn / sff_init_nn_leaves (`leaves` = 1, 2 or
 * 4) from the coarsest level's bin-sum planes instead of its descriptors, with
 * the same results: descriptor distances are 16 times bin-grid distances, so
 * the argmins, ties and costs are the same.  The temporal search runs on fp16
 * MFMA with centred bins (bin - 510, exact in fp16; the products' sums are
 * exact in fp32).
 * bins: level-(levels-1) planes of the 4 views of each pair, [batch][4] images
 *   of sff_bin_bytes bytes, 16-byte aligned.
 * workspace: 256-byte aligned, at least sff_init_bins_workspace_bytes(p, batch)
 *   bytes; contents on entry are ignored.
 * Errors: as sff_init_nn_leaves; SFF_ERR_UNSUPPORTED when an image's planes
 *   reach 2 GiB. */
sff_status sff_init_nn_bins(const sff_params* p, int32_t batch, int32_t dir, int32_t leaves,
                            const uint16_t* bins, int16_t* hyp, uint32_t* cost, void* workspace,
                            size_t workspace_bytes, void* stream);

/* Propagation and random search at one level (Section 3.1, "Multi-Scale
 * Propagation"), eq. (1) cost: sum over the temporal (x + u, y + v), stereo
 * (x - s d0, y) and cross (x + u - s d1, y + v) partners of the squared
 * distance of level-k descriptors, targets clamped to the image, uint32.
 *   hand-off (hyp_coarse != NULL): every pixel starts from its parent's vector
 *     hyp_coarse[i >> 1][j >> 1] with its cost recomputed at this level;
 *     otherwise hyp/cost already hold the starting field (the initialisation).
 *   iterations: red pixels ((i + j) even) then black ones; each takes the
 *     cheapest of [own, left, up, right, down] under strict improvement, then
 *     rs_samples random-search samples around that vector: sample t moves each
 *     component by a uniform integer in [-r_t, r_t], r_t = max(1, rs_r0 >> t)
 *     * n, clamped to |u|,|v| <= fmax, 0 <= d <= dmax; Philox4x32-10 with key
 *     = seeds[b] and counter (i*Wk + j, it, (k << 16) | (t << 8) | (s < 0), 0),
 *     offset = floor(x_c (2 r_t + 1) / 2^32) - r_t; kept on strict improvement.
 * desc:  level-k descriptors [batch][4][H][W][Cp][16].
 * seeds: [batch] uint64, device.
 * hyp_coarse: level-(k+1) field [ndir][batch][H(k+1)][W(k+1)][4] or NULL;
 *   must not overlap hyp.
 * hyp/cost: level-k field, read and written in place.
 * Two kernels with identical results gather the descriptors: one lane per
 *   pixel below 20000 pixel updates per launch (ndir * batch * H(k) *
 *   ceil(W(k) / 2)), wave-cooperative loads otherwise (32 pixels per wave below
 *   50000 updates, 64 above); the environment variable SFF_MATCH_EVAL=lane|
 *   coop|coop-narrow|coop-wide|coop-narrow-32|coop-wide-32 forces one (testing
 *   and timing).  The cooperative loads use 32-bit offsets: for descriptor maps of
 *   2 GiB or more (H * W > 16.7 M at C = 3 or 4) the per-lane kernel runs
 *   whatever the variable says.
 * Errors: SFF_ERR_INVALID_ARG (also for level >= levels - 1 with a non-NULL
 *   hyp_coarse, and for overlapping hyp/hyp_coarse). */
sff_status sff_match_level(const sff_params* p, int32_t batch, int32_t dir, int32_t level,
                           const int16_t* desc, const uint64_t* seeds, const int16_t* hyp_coarse,
                           int16_t* hyp, uint32_t* cost, void* stream);

/* The same level with the descriptor distances taken from the WHT bin-sum
 * planes (16 x the bin-grid squared distance, exactly the descriptor squared
 * distance, so hyp and cost equal those of sff_match_level on the level's WHT
 * descriptors).  bins: level-k planes of the 4 views of each pair,
 * [batch][4] images of sff_bin_bytes(p, level) bytes (sff_wht_features),
 * 16-byte aligned.  Other arguments as for sff_match_level.  Wave-cooperative
 * gathers from 20000 pixel updates per launch (below 50000: 16 pixels per
 * wave, all 4 neighbours and all samples at once, three views a round; below
 * 262144: 32 pixels per wave, groups of 4 neighbours and 3 samples, view by
 * view; above: 64 pixels per wave, one candidate at a time, three views a
 * round), one lane per pixel below;
 * SFF_MATCH_EVAL=lane|coop|coop-32|coop-43-32|coop-46-32|coop-xts|
 * coop-46-16-xts forces one (identical results).  With dir = SFF_DIR_BOTH
 * and 100000 or more updates the two fields run on two streams: `stream` and
 * a helper stream of the library, which waits for the work enqueued on
 * `stream` before the call, and which `stream` waits for after it (so the
 * call is ordered on `stream` as any other); SFF_MATCH_SPLIT=0|1 forces one
 * sequence or the split (identical results).
 * Errors: as sff_match_level; SFF_ERR_UNSUPPORTED when an image's planes
 *   reach 2 GiB (32-bit gather offsets). */
sff_status sff_match_level_bins(const sff_params* p, int32_t batch, int32_t dir, int32_t level,
                                const uint16_t* bins, const uint64_t* seeds,
                                const int16_t* hyp_coarse, int16_t* hyp, uint32_t* cost,
                                void* stream);

/* Consistency check (Section 3.1, "Consistency Check"; tau_c, Section 5).
 * For every pixel p with forward vector (u, v, d0, d1): if a forward target
 * lies outside the image the match is invalid and err = UINT32_MAX; otherwise,
 * with (u', v', d0', d1') the inverse field at q = (x + u - d1, y + v),
 * e0 = d0 - d1', e1 = d1 - d0', ef = (u + u' + d1' - d0', v + v');
 * valid = 1 iff e0^2, e1^2 and |ef|^2 are all <= tau^2; err = their maximum.
 * hyp_fwd, hyp_inv: level-0 fields [batch][H][W][4].
 * valid: [batch][H][W] uint8 (0/1), err: [batch][H][W] uint32, written.
 * Errors: SFF_ERR_INVALID_ARG. */
sff_status sff_consistency(const sff_params* p, int32_t batch, const int16_t* hyp_fwd,
                           const int16_t* hyp_inv, uint8_t* valid, uint32_t* err, void* stream);

/* Device workspace (bytes) that sff_region_filter needs for `batch` fields
 * (12 bytes per pixel); 0 for invalid arguments. */
size_t sff_region_workspace_bytes(const sff_params* p, int32_t batch);

/* Region filter (Section 3.1, "Consistency Check", second step; the paper
 * uses s_c = 150, Section 5).  Consistent pixels form regions: two
 * 4-neighbours belong to one region when both are valid and every component
 * of their vectors differs by at most p->tau.  A region is dropped when it has
 * fewer than s_c pixels and some inconsistent 4-neighbour of one of its pixels
 * has a vector within p->tau of that pixel's (a removed outlier that could
 * join it).  The result does not depend on the order of evaluation.
 * hyp_fwd: level-0 forward field [batch][H][W][4] (8-byte aligned);
 * valid: [batch][H][W] uint8 from sff_consistency;
 * keep: [batch][H][W] uint8 (0/1), written;
 * workspace: at least sff_region_workspace_bytes(p, batch) bytes, 256-byte
 *   aligned; contents on entry are ignored.
 * Errors: SFF_ERR_INVALID_ARG (also s_c < 1), SFF_ERR_WORKSPACE. */
sff_status sff_region_filter(const sff_params* p, int32_t batch, int32_t s_c,
                             const int16_t* hyp_fwd, const uint8_t* valid, uint8_t* keep,
                             void* workspace, size_t workspace_bytes, void* stream);

/* Sparsification (Section 3.2, "Sparsification"): in each non-overlapping
 * 3 x 3 block (aligned at the origin, cut at the right and bottom borders) the
 * kept match with the lowest consistency error, ties to the lowest raster
 * index y * W + x.
 * keep: [batch][H][W] uint8; err: [batch][H][W] uint32 (from sff_consistency);
 * seeds: [batch][ceil(H/3)][ceil(W/3)] int32, written: the pixel index y*W + x
 *   of the block's seed, or -1 for a block without a kept match.
 * Errors: SFF_ERR_INVALID_ARG. */
sff_status sff_sparsify(const sff_params* p, int32_t batch, const uint8_t* keep,
                        const uint32_t* err, int32_t* seeds, void* stream);

/* Device workspace (bytes) that sff_sgm_disparity needs for `batch` pairs
 * (about 10 + 1024 / W + 8 (dmax + 1) bytes per pixel); 0 for invalid
 * arguments. */
size_t sff_sgm_workspace_bytes(const sff_params* p, int32_t batch);

/* Disparity by semi-global matching (Hirschmueller, TPAMI 2008), the second
 * disparity map of the disparity fill (Section 3.1, last paragraph of
 * "Consistency Check").  Grey = rounded channel mean; cost = Hamming distance
 * of 5 x 5 census words (bit k: neighbour k, row-major without the centre,
 * darker than the centre; replicated border) of left pixel x and right pixel
 * x - d (clamped), d = 0..dmax; aggregation along 8 paths with penalties P1
 * (disparity change 1) and P2 (larger changes); disparity = argmin over d of
 * the summed path costs, the smallest d on ties.
 * left, right: image pairs [H][W][C] uint8, pair b at byte offset
 *   b * pair_stride of each pointer (pair_stride >= H W C when batch > 1).
 * disp: [batch][H][W] int16, written.  P1 >= 0, P1 <= P2 <= 231 (path costs
 *   are stored in 8 bits).
 * workspace: at least sff_sgm_workspace_bytes(p, batch) bytes, 256-byte
 *   aligned; contents on entry are ignored.
 * Errors: SFF_ERR_INVALID_ARG, SFF_ERR_UNSUPPORTED (dmax + 1 > 256),
 *   SFF_ERR_WORKSPACE. */
sff_status sff_sgm_disparity(const sff_params* p, int32_t batch, const uint8_t* left,
                             const uint8_t* right, size_t pair_stride, int32_t P1, int32_t P2,
                             int16_t* disp, void* workspace, size_t workspace_bytes, void* stream);

/* Disparity fill (Section 3.1, last paragraph of "Consistency Check"):
 * fill = 1 where the joint check kept the match (valid), or where it removed
 * it but the match's disparity d0 keeps the stereo target in the image
 * (x - d0 >= 0) and |d0 - disp| <= p->tau (the check of the disparity match
 * alone against the SGM map).
 * hyp_fwd: level-0 forward field [batch][H][W][4]; valid: [batch][H][W] uint8;
 * disp: [batch][H][W] int16 (sff_sgm_disparity); fill: [batch][H][W] uint8.
 * Errors: SFF_ERR_INVALID_ARG. */
sff_status sff_disparity_fill(const sff_params* p, int32_t batch, const int16_t* hyp_fwd,
                              const uint8_t* valid, const int16_t* disp, uint8_t* fill,
                              void* stream);

/* ---------------------------------------------------------------------------
 * The paper's own matching cost (Section 3.1, "Matching Cost", eq. (1)): the
 * Euclidean distances between the first three principal components of dense
 * SIFT features, summed over a 7 x 7 window and the temporal, stereo and
 * cross correspondences; the principal axes are those of the SIFT features of
 * all four images of the pair; boundary pixels replicated.  FP32 features,
 * FP64 statistics.
 *
 * Dense SIFT (SIFT flow, Liu et al. 2011; Lowe 2004): central-difference
 * gradients of the grey (channel mean) image with clamped neighbours, 8
 * orientation bins of 45 degrees (bin b centred at b * 45 degrees, y down),
 * magnitude split linearly between the two nearest centres; 4 x 4 cells of
 * 3 x 3 pixels over rows and columns -6 .. +5 around the pixel, pixels outside
 * clamped; entry (4 i + j) * 8 + b for cell row i, cell column j, bin b;
 * normalised to unit length, clamped at 0.2, normalised again (zero stays
 * zero). */

/* Device workspace (bytes) of sff_dense_sift for nimg images and of
 * sff_sift_pca for nimg = 4 * batch images: orientation and cell-sum planes
 * (about 64 bytes per pixel and image) plus FP64 partial sums (up to 34 MB
 * per pair); 0 for invalid arguments. */
size_t sff_sift_workspace_bytes(const sff_params* p, int32_t nimg);

/* Dense SIFT of nimg images [nimg][H][W][C] uint8 (C = p->C) into
 * sift [nimg][H][W][128] float32 (16-byte aligned).
 * Errors: SFF_ERR_INVALID_ARG, SFF_ERR_WORKSPACE. */
sff_status sff_dense_sift(const sff_params* p, int32_t nimg, const uint8_t* img, float* sift,
                          void* workspace, size_t workspace_bytes, void* stream);

/* Features of eq. (1) for batch pairs imgs [batch][4][H][W][C] uint8 (views
 * l0, l1, r0, r1): per pair the mean [128] and covariance [128][128] (1/N,
 * N = 4 H W) of the SIFT features of its four images, the three largest
 * eigenvalues [3] and their unit eigenvectors axes [3][128] (each signed so
 * that its component of largest magnitude is positive), and
 * phi [batch][4][H][W][4] float32 = (axes (f - mean), 0) per pixel.
 * FP64 outputs 8-byte aligned, phi 16-byte aligned; all caller-owned.
 * workspace: sff_sift_workspace_bytes(p, 4 * batch) bytes, 256-byte aligned.
 * The eigenvectors come from a subspace iteration that stops when the
 * residuals of the three leading pairs fall below 1e-12 of the largest
 * eigenvalue (at most 4000 iterations); for a zero covariance the axes are
 * arbitrary unit vectors and phi is zero.
 * Errors: SFF_ERR_INVALID_ARG, SFF_ERR_WORKSPACE. */
sff_status sff_sift_pca(const sff_params* p, int32_t batch, const uint8_t* imgs, double* mean,
                        double* cov, double* eigval, double* axes, float* phi, void* workspace,
                        size_t workspace_bytes, void* stream);

/* Eq. (1) per pixel at fixed full-resolution vectors hyp [batch][H][W][4]
 * int16 (u, v, d0, d1), from phi [batch][4][H][W][4] float32 (first three
 * components used):
 *   cost(p) = sum_{w in {-3..3}^2} sum_{corr in T, S, X}
 *             || phi_R(clamp(p + w)) - phi_corr(clamp(p + w + o_corr)) ||_2,
 *   o_T = (u, v), o_S = (-s d0, 0), o_X = (u - s d1, v), s = dir, with
 *   (R, T, S, X) = (l0, l1, r0, r1) for SFF_DIR_FORWARD and (r1, r0, l1, l0)
 *   for SFF_DIR_INVERSE.  cost: [batch][H][W] float32.
 * Errors: SFF_ERR_INVALID_ARG (shapes, alignment, dir). */
sff_status sff_cost_sift(const sff_params* p, int32_t batch, int32_t dir, const float* phi,
                         const int16_t* hyp, float* cost, void* stream);

/* Full-resolution matching with the cost above (Section 3.1, "Multi-Scale
 * Propagation" at the finest scale, with the eq. (1) of "Matching Cost"),
 * starting from the field in hyp: the cost of every pixel's vector, then
 * `iters` iterations of red-black propagation (left, up, right, down) and
 * p->rs_samples random-search samples (radius p->rs_r0 >> t, Philox4x32-10
 * with key = seeds[b] and counter (y W + x, it, (16 << 16) | (t << 8) |
 * (s < 0), 0)), strict improvement, vectors clamped to p->fmax / p->dmax.
 * Costs in FP32 summed in a fixed order (window rows, columns, then the
 * temporal, stereo and cross distances ((e0^2 + e1^2) + e2^2, correctly
 * rounded root), each operation rounded), so results are reproducible bit for
 * bit; sff_cost_sift uses the same arithmetic.
 * phi: [batch][4][H][W][4] float32 (sff_sift_pca); seeds: [batch] uint64;
 * hyp: [ndir][batch][H][W][4] int16, read and written (ndir = 2 for
 * SFF_DIR_BOTH, forward first); cost: [ndir][batch][H][W] float32, written.
 * The window gathers are shared by the 64 pixels of a wave (each window
 * column loaded by one lane, the owner adding its distances in the order
 * above); SFF_SIFT_EVAL=lane runs the one-lane-per-pixel kernel instead (same
 * results; testing and timing).
 * Errors: SFF_ERR_INVALID_ARG. */
sff_status sff_match_sift(const sff_params* p, int32_t batch, int32_t dir, const float* phi,
                          const uint64_t* seeds, int32_t iters, int16_t* hyp, float* cost,
                          void* stream);

/* The square root that the cost above applies to each squared distance, over
 * an array: out[i] = sqrt(in[i]) correctly rounded (IEEE round to nearest even)
 * for finite in[i] >= +0 (other inputs: unspecified), i < n.  in/out: device,
 * 4-byte aligned, n in [0, 2^31].  Exposed so that the rounding can be checked
 * against the host.  Errors: SFF_ERR_INVALID_ARG. */
sff_status sff_sift_sqrt(const float* in, float* out, int64_t n, void* stream);

/* ---------------------------------------------------------------------------
 * Window form of the matching cost on real-valued feature maps (eq. (1),
 * Section 3.1: feature distances summed over a window around the pixel for the
 * temporal, stereo and cross correspondences, replicated borders), FP32:
 *   cost(p) = sum_corr sum_{w in {-3..4}^2} sum_c
 *             (F_R(clamp(p + w), c) - F_corr(clamp(t_corr(p) + w), c))^2,
 *   t_corr(p) = clamp(p + o_corr), o_T = (u, v), o_S = (-s d0, 0),
 *   o_X = (u - s d1, v), s = dir.
 * feat: [batch][4][H][W][cf] float32, views in the canonical order, 16-byte
 *   aligned; cf in {4, 8, 16, 32, 64}.
 * hyp:  [batch][H][W][4] int16 full-resolution vectors (held fixed).
 * dir:  SFF_DIR_FORWARD or SFF_DIR_INVERSE.
 * Each pixel is summed by cf / 4 lanes (four channels each, lane sums added
 * by a butterfly): deterministic, FP32 with partial sums (relative error below
 * ~(3 cf + 16) 2^-24); SFF_COST_F32_EVAL=lane sums each pixel in one lane
 * (another rounding within the same bound; testing and timing).
 * Errors: SFF_ERR_INVALID_ARG (shapes, alignment, dir, batch*H*W >= 2^31). */
sff_status sff_cost_f32_fwd(int32_t batch, int32_t H, int32_t W, int32_t cf, int32_t dir,
                            const float* feat, const int16_t* hyp, float* cost_px, void* stream);

/* Device workspace (bytes) that sff_cost_f32_bwd needs. */
size_t sff_cost_f32_bwd_workspace_bytes(int32_t batch, int32_t H, int32_t W);

/* Gradient of L = sum_p grad_cost[p] * cost(p) with respect to all four
 * feature maps (chain rule: each term with difference delta contributes
 * +2 g delta to its reference entry and -2 g delta to its target entry).
 * grad_cost: [batch][H][W] float32.  grad_feat: [batch][4][H][W][cf] float32,
 * fully overwritten.  Deterministic: the same inputs give the same bits.
 * Each gradient entry is gathered by cf / 4 lanes, four channels each;
 * SFF_COST_F32_EVAL=lane gathers with one lane per entry (same bits; testing
 * and timing).  The reference-map gradient runs on the library's helper
 * stream beside the target-map gradients, joined to `stream` before the call
 * returns as for sff_match_level_bins (SFF_COST_F32_SPLIT=0: all on `stream`;
 * same bits).
 * workspace: device buffer, 256-byte aligned, at least
 *   sff_cost_f32_bwd_workspace_bytes(batch, H, W) bytes.
 * Errors: SFF_ERR_INVALID_ARG, SFF_ERR_WORKSPACE. */
sff_status sff_cost_f32_bwd(int32_t batch, int32_t H, int32_t W, int32_t cf, int32_t dir,
                            const float* feat, const int16_t* hyp, const float* grad_cost,
                            float* grad_feat, void* workspace, size_t workspace_bytes,
                            void* stream);

/* ---------------------------------------------------------------------------
 * Learned features in place of the WHT features of the matching cost
 * (Section 3.1): 3x3 convolutions, BF16 NHWC tensors (raw bfloat16 bits as
 * uint16_t), FP32 accumulation on the matrix cores, zero padding, dilation
 * `dil` (1..16).  Weights [cout][3][3][cin] BF16, tap (ky, kx) reading offset
 * ((ky - 1) dil, (kx - 1) dil); bias [cout] FP32.  Supported: cin in {3, 32},
 * cout = 32.  Results are rounded to BF16 (nearest even) on store.
 *   y = act(bias + sum_tap W_tap x_shifted), act = ReLU if relu != 0.
 * For cin = 32 and 16-byte aligned tensors the forward, input-gradient and
 * weight-gradient kernels read their inputs in 16-byte pieces (the forward
 * without an im2col tile); SFF_CONV_IM2COL=1 forces the element-wise kernels
 * (same results).
 * Errors: SFF_ERR_INVALID_ARG (shapes, NULL pointers, y not 8-byte aligned). */
sff_status sff_conv3x3_bf16_fwd(int32_t n, int32_t H, int32_t W, int32_t cin, int32_t cout,
                                int32_t dil, int32_t relu, const uint16_t* x, const uint16_t* w,
                                const float* bias, uint16_t* y, void* stream);

/* The learned-feature network's forward pass in one launch (dilation 1):
 * y = conv4(relu(conv3(relu(conv2(relu(conv1(x))))))), conv1 3 -> 32, conv2..4
 * 32 -> 32, each a 3x3 convolution as sff_conv3x3_bf16_fwd computes it
 * (weights w_l [32][3][3][cin], bias b_l [32] FP32 or NULL, zero padding),
 * the activations between layers kept on chip.  x [n][H][W][3], y
 * [n][H][W][32], BF16 bits.  Bit-identical to the four sff_conv3x3_bf16_fwd
 * calls (each layer's output rounded to BF16 the same way).  y 8-byte aligned,
 * w1..w3 16-byte aligned.  Errors: SFF_ERR_INVALID_ARG (shapes, NULL pointers,
 * alignment), SFF_ERR_UNSUPPORTED (dil != 1: use the per-layer calls). */
sff_status sff_featnet_fwd_bf16(int32_t n, int32_t H, int32_t W, int32_t dil, const uint16_t* x,
                                const uint16_t* w0, const float* b0, const uint16_t* w1,
                                const float* b1, const uint16_t* w2, const float* b2,
                                const uint16_t* w3, const float* b3, uint16_t* y, void* stream);

/* Device workspace (bytes) for sff_conv3x3_bf16_dgrad / _wgrad. */
size_t sff_conv3x3_bf16_bwd_workspace_bytes(int32_t n, int32_t H, int32_t W, int32_t cin,
                                            int32_t cout);

/* Input gradient (cin = 32): dx = sum over the outputs that read each input of
 * W times dz, with dz = dy * (relu_out > 0) when relu_out (the layer's ReLU
 * output) is given, dz = dy when it is NULL.  dy [n][H][W][cout], dx
 * [n][H][W][cin], BF16.  Errors: SFF_ERR_INVALID_ARG, SFF_ERR_WORKSPACE. */
sff_status sff_conv3x3_bf16_dgrad(int32_t n, int32_t H, int32_t W, int32_t cin, int32_t cout,
                                  int32_t dil, const uint16_t* dy, const uint16_t* relu_out,
                                  const uint16_t* w, uint16_t* dx, void* workspace,
                                  size_t workspace_bytes, void* stream);

/* Weight and bias gradients: dw [cout][3][3][cin] = sum_p dz[p] x[p + tap]^T,
 * db [cout] = sum_p dz[p], FP32, dz as for dgrad.  Per-block partial sums are
 * reduced in a fixed order (deterministic).  Errors: SFF_ERR_INVALID_ARG,
 * SFF_ERR_WORKSPACE. */
sff_status sff_conv3x3_bf16_wgrad(int32_t n, int32_t H, int32_t W, int32_t cin, int32_t cout,
                                  int32_t dil, const uint16_t* x, const uint16_t* dy,
                                  const uint16_t* relu_out, float* dw, float* db, void* workspace,
                                  size_t workspace_bytes, void* stream);

/* The level-k image of the scale simulation alone (Section 3.1, "Multi-Scale
 * Propagation"; the smoothing step of sff_wht_features): img [nimg][H][W][C]
 * -> out [nimg][H][W][C] uint8 (a copy at level 0).  workspace as for
 * sff_wht_features.  Used to feed learned features per level.
 * Errors: SFF_ERR_INVALID_ARG, SFF_ERR_WORKSPACE. */
sff_status sff_smooth_level(const sff_params* p, int32_t nimg, int32_t level, const uint8_t* img,
                            uint8_t* out, void* workspace, size_t workspace_bytes, void* stream);

/* Learned descriptors: per-pixel L2 normalisation of 32-channel BF16 features
 * feat [n][H][W][32], scaled and rounded to int16: desc = rint(scale f / |f|)
 * (0 < scale <= 8192).  desc [n][H][W][32] is a C = 2 descriptor map for
 * sff_init_nn / sff_match_level (squared distances stay far below 2^31 per
 * map).  Errors: SFF_ERR_INVALID_ARG. */
sff_status sff_quantise_features(int32_t n, int32_t H, int32_t W, const uint16_t* feat, float scale,
                                 int16_t* desc, void* stream);

/* Triplet loss on normalised 32-channel BF16 features feat [npx][32]: for
 * triple t = (a, p, n) of pixel indices (triplets [ntrip][3] int32, device),
 * loss[t] = max(0, margin + |a^ - p^|^2 - |a^ - n^|^2); weight * dloss/dfeat
 * is ADDED to grad [npx][32] FP32 (atomic adds: summation order may vary).
 * Triples with an index outside [0, npx) give loss 0 and no gradient.
 * Errors: SFF_ERR_INVALID_ARG. */
sff_status sff_triplet_loss(int32_t npx, const uint16_t* feat, int32_t ntrip,
                            const int32_t* triplets, float margin, float weight, float* loss,
                            float* grad, void* stream);

/* out[i] = bf16(grad[i]) (nearest even), then grad[i] = 0, for i < n. */
sff_status sff_take_grad_bf16(size_t n, float* grad, uint16_t* out, void* stream);

/* ---------------------------------------------------------------------------
 * Calibration kernels for the roofline (no part of the method).
 * sff_probe_copy: dst[i] = src[i] for `bytes` bytes (multiple of 16, both
 *   16-byte aligned), streaming 16-byte loads and stores.
 * sff_probe_gather: `threads` threads (multiple of 256) each own `per_thread`
 *   records of `record_bytes` bytes (16..256, multiple of 16) at pseudo-random
 *   record indices of buf [buf_bytes] (16-byte aligned) and write one folded
 *   word to out[thread] (out holds `threads` uint32).  coop = 0: each thread
 *   loads its own records; coop = 1: the records of a 64-lane wave are loaded
 *   by consecutive lanes, 16 bytes each (same records and bytes).
 * Errors: SFF_ERR_INVALID_ARG. */
sff_status sff_probe_copy(const void* src, void* dst, size_t bytes, void* stream);
sff_status sff_probe_gather(const void* buf, size_t buf_bytes, int32_t record_bytes,
                            int32_t threads, int32_t per_thread, uint64_t seed, int32_t coop,
                            uint32_t* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SFF_H */
