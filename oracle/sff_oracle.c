/*
 * Plain CPU oracle of the sparse scene-flow matching stage of SceneFlowFields
 * (Schuster et al., arXiv 1710.10096, Section 3.1).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition that the GPU library is checked against.  Only the test suite, the
 * smoke check and the bench's CPU-baseline leg may load it; the product path
 * never does.  It shares no code, header, table or constant generator with the
 * GPU library.
 *
 * Every function below cites the passage it follows.  Integer arithmetic
 * throughout; the only floating point is the FP64 evaluation of the Lanczos
 * weights before they are quantised to Q14 integers.
 *
 * Layouts (all row-major, no padding):
 *   image  uint8 [H][W][C]
 *   desc   int16 [H][W][C][16]     16 = 4x4 low-sequency WHT coefficients
 *   hyp    int16 [Hk][Wk][4]       (u, v, d0, d1) in full-resolution pixels
 *   cost   uint32 [Hk][Wk]
 * Images of a direction: the four maps are always passed in the canonical order
 * (l0, l1, r0, r1) = (I_l^0, I_l^1, I_r^0, I_r^1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR 1

static int clampi(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }

/* floor(a / b) for b > 0 */
static int32_t floordiv(int32_t a, int32_t b) {
    int32_t q = a / b;
    if ((a % b) != 0 && (a < 0)) q -= 1;
    return q;
}

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 counter-based generator, from its published definition       */
/* (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", */
/* SC'11): 10 rounds of two 32x32->64 multiplies with a Weyl key schedule.      */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------- */
/* Scale simulation (Section 3.1, "Multi-Scale Propagation"): the level-k     */
/* image is smoothed by area-based downsampling by n = 2^k followed by Lanczos */
/* upsampling back to full resolution.  Reading: Lanczos-3, pixel-centre       */
/* alignment, weights quantised to Q14 per phase (x mod n).                   */
/* ------------------------------------------------------------------------- */
static double sinc(double t) {
    if (t == 0.0) return 1.0;
    const double pt = 3.14159265358979323846 * t;
    return sin(pt) / pt;
}
static double lanczos3(double t) {
    if (t <= -3.0 || t >= 3.0) return 0.0;
    return sinc(t) * sinc(t / 3.0);
}

/* Source coordinate of output x = n*j + p is s = (x + 0.5)/n - 0.5
 * = j + (p + 0.5)/n - 0.5.  floor part i0(p) in {-1, 0}, fraction f(p). */
static void phase_geometry(int n, int p, int* i0, double* f) {
    double s = (p + 0.5) / n - 0.5;
    double fl = floor(s);
    *i0 = (int)fl;
    *f = s - fl;
}

/* Six taps per phase: tap t (0..5) sits at floor(s) - 2 + t, distance f + 2 - t.
 * Weights: FP64, normalised, rounded half away from zero to Q14; the residual
 * goes to the tap nearest s so each phase sums to exactly 16384. */
void orc_lanczos_q14(int n, int32_t* table /* [n][6] */) {
    for (int p = 0; p < n; ++p) {
        int i0;
        double f;
        phase_geometry(n, p, &i0, &f);
        double w[6], sum = 0.0;
        for (int t = 0; t < 6; ++t) {
            w[t] = lanczos3(f + 2.0 - t);
            sum += w[t];
        }
        int32_t q[6], qsum = 0;
        for (int t = 0; t < 6; ++t) {
            double x = w[t] / sum * 16384.0;
            q[t] = (int32_t)(x >= 0 ? floor(x + 0.5) : -floor(-x + 0.5));
            qsum += q[t];
        }
        int nearest = (f < 0.5) ? 2 : 3;
        q[nearest] += 16384 - qsum;
        for (int t = 0; t < 6; ++t) table[p * 6 + t] = q[t];
    }
}

/* S_k of one image (all channels).  n = 1 returns the image unchanged. */
int orc_smooth(const uint8_t* img, int H, int W, int C, int n, uint8_t* out) {
    if (n == 1) {
        memcpy(out, img, (size_t)H * W * C);
        return ORC_OK;
    }
    const int Hk = (H + n - 1) / n, Wk = (W + n - 1) / n;
    int32_t* A = (int32_t*)malloc(sizeof(int32_t) * (size_t)Hk * Wk * C);
    int32_t* h = (int32_t*)malloc(sizeof(int32_t) * (size_t)Hk * W * C);
    int32_t* table = (int32_t*)malloc(sizeof(int32_t) * (size_t)n * 6);
    int* i0 = (int*)malloc(sizeof(int) * (size_t)n);
    if (!A || !h || !table || !i0) {
        free(A); free(h); free(table); free(i0);
        return ORC_ERR;
    }
    orc_lanczos_q14(n, table);
    for (int p = 0; p < n; ++p) {
        double f;
        phase_geometry(n, p, &i0[p], &f);
    }
    /* area-based downsampling: rounded mean of the n x n block, replicated border */
    for (int i = 0; i < Hk; ++i)
        for (int j = 0; j < Wk; ++j)
            for (int c = 0; c < C; ++c) {
                int32_t s = 0;
                for (int a = 0; a < n; ++a)
                    for (int b = 0; b < n; ++b) {
                        int y = clampi(n * i + a, 0, H - 1), x = clampi(n * j + b, 0, W - 1);
                        s += img[((size_t)y * W + x) * C + c];
                    }
                A[((size_t)i * Wk + j) * C + c] = (s + n * n / 2) / (n * n);
            }
    /* horizontal Lanczos pass on the rows of A, to full width */
    for (int i = 0; i < Hk; ++i)
        for (int x = 0; x < W; ++x) {
            int p = x % n, j = x / n;
            for (int c = 0; c < C; ++c) {
                int32_t acc = 0;
                for (int t = 0; t < 6; ++t) {
                    int jj = clampi(j + i0[p] - 2 + t, 0, Wk - 1);
                    acc += table[p * 6 + t] * A[((size_t)i * Wk + jj) * C + c];
                }
                h[((size_t)i * W + x) * C + c] = floordiv(acc + 8192, 16384);
            }
        }
    /* vertical Lanczos pass to full height, clamped to 0..255 */
    for (int y = 0; y < H; ++y) {
        int p = y % n, i = y / n;
        for (int x = 0; x < W; ++x)
            for (int c = 0; c < C; ++c) {
                int32_t acc = 0;
                for (int t = 0; t < 6; ++t) {
                    int ii = clampi(i + i0[p] - 2 + t, 0, Hk - 1);
                    acc += table[p * 6 + t] * h[((size_t)ii * W + x) * C + c];
                }
                out[((size_t)y * W + x) * C + c] = (uint8_t)clampi(floordiv(acc + 8192, 16384), 0, 255);
            }
    }
    free(A); free(h); free(table); free(i0);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* WHT feature vectors (Section 3.1, "Initialization"; Section 3 overview).   */
/* Reading: 8x8 patch of the level-k image sampled every n-th pixel at offsets */
/* -3..+4, replicated border; the 16 coefficients are the 4x4 lowest-sequency  */
/* block of the unnormalised 2-D Walsh-Hadamard transform, index a*4 + b with  */
/* a the vertical and b the horizontal sequency.                               */
/* ------------------------------------------------------------------------- */

/* Walsh function of sequency a at position i (length 8):
 * (-1)^popcount(r_a & i), r_a = bit-reversal (3 bits) of the Gray code of a. */
static int walsh8(int a, int i) {
    int g = a ^ (a >> 1);
    int r = ((g & 1) << 2) | (g & 2) | ((g >> 2) & 1);
    return (__builtin_popcount(r & i) & 1) ? -1 : 1;
}

int orc_wht(const uint8_t* S, int H, int W, int C, int n, int16_t* desc) {
    int w[4][8];
    for (int a = 0; a < 4; ++a)
        for (int i = 0; i < 8; ++i) w[a][i] = walsh8(a, i);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int c = 0; c < C; ++c) {
                int32_t P[8][8];
                for (int i = 0; i < 8; ++i)
                    for (int j = 0; j < 8; ++j) {
                        int yy = clampi(y + n * (i - 3), 0, H - 1);
                        int xx = clampi(x + n * (j - 3), 0, W - 1);
                        P[i][j] = S[((size_t)yy * W + xx) * C + c];
                    }
                /* c_ab = sum_i w_a(i) sum_j w_b(j) P(i, j): rows first, then columns */
                int32_t rowt[8][4];
                for (int i = 0; i < 8; ++i)
                    for (int b = 0; b < 4; ++b) {
                        int32_t s = 0;
                        for (int j = 0; j < 8; ++j) s += w[b][j] * P[i][j];
                        rowt[i][b] = s;
                    }
                int16_t* d = desc + (((size_t)y * W + x) * C + c) * 16;
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) {
                        int32_t s = 0;
                        for (int i = 0; i < 8; ++i) s += w[a][i] * rowt[i][b];
                        d[a * 4 + b] = (int16_t)s;
                    }
            }
    return ORC_OK;
}

/* Level-k descriptors of one image: smoothing (k >= 1) then WHT. */
int orc_features(const uint8_t* img, int H, int W, int C, int level, int16_t* desc) {
    const int n = 1 << level;
    uint8_t* S = (uint8_t*)malloc((size_t)H * W * C);
    if (!S) return ORC_ERR;
    int st = orc_smooth(img, H, W, C, n, S);
    if (st == ORC_OK) st = orc_wht(S, H, W, C, n, desc);
    free(S);
    return st;
}

/* ------------------------------------------------------------------------- */
/* Matching cost, eq. (1): the sum over three correspondences -- temporal     */
/* left (I_l^1 at p + (u, v)), stereo at t0 (I_r^0 at p + (-d0, 0)) and cross  */
/* (I_r^1 at p + (u - d1, v)) -- of feature distances.  Reading: squared L2    */
/* distance of the WHT descriptors (the descriptor's 8x8 patch is the window), */
/* summed over channels, accumulated in uint32; targets clamped to the image   */
/* (replicated border).  For the inverse field (s = -1) the reference is       */
/* I_r^1, the temporal partner I_r^0, the stereo partner I_l^1 and the cross   */
/* partner I_l^0, and the disparity offsets change sign.                       */
/* ------------------------------------------------------------------------- */
typedef struct {
    const int16_t* R; /* reference */
    const int16_t* T; /* temporal partner */
    const int16_t* S; /* stereo partner */
    const int16_t* X; /* cross partner */
    int H, W, C, s;
} orc_views;

static orc_views make_views(const int16_t* l0, const int16_t* l1, const int16_t* r0,
                            const int16_t* r1, int H, int W, int C, int s) {
    orc_views v;
    if (s > 0) { v.R = l0; v.T = l1; v.S = r0; v.X = r1; }
    else       { v.R = r1; v.T = r0; v.S = l1; v.X = l0; }
    v.H = H; v.W = W; v.C = C; v.s = s;
    return v;
}

static uint32_t ssd_at(const orc_views* V, const int16_t* img, int x, int y, int tx, int ty) {
    tx = clampi(tx, 0, V->W - 1);
    ty = clampi(ty, 0, V->H - 1);
    const int16_t* a = V->R + ((size_t)y * V->W + x) * V->C * 16;
    const int16_t* b = img + ((size_t)ty * V->W + tx) * V->C * 16;
    uint32_t acc = 0;
    for (int e = 0; e < V->C * 16; ++e) {
        int32_t d = (int32_t)a[e] - (int32_t)b[e];
        acc += (uint32_t)(d * d);
    }
    return acc;
}

static uint32_t cost_eq1(const orc_views* V, int x, int y, const int16_t h[4]) {
    const int u = h[0], v = h[1], d0 = h[2], d1 = h[3], s = V->s;
    uint32_t c = 0;
    c += ssd_at(V, V->T, x, y, x + u, y + v);          /* temporal */
    c += ssd_at(V, V->S, x, y, x - s * d0, y);         /* stereo at t0 */
    c += ssd_at(V, V->X, x, y, x + u - s * d1, y + v); /* cross */
    return c;
}

/* Exposed for tests: cost of hypothesis h at full-resolution pixel (x, y). */
uint32_t orc_cost(const int16_t* l0, const int16_t* l1, const int16_t* r0, const int16_t* r1,
                  int H, int W, int C, int s, int x, int y, const int16_t h[4]) {
    orc_views V = make_views(l0, l1, r0, r1, H, W, C, s);
    return cost_eq1(&V, x, y, h);
}

/* ------------------------------------------------------------------------- */
/* Initialisation (Section 3.1, "Initialization"), coarsest level only.        */
/* Reading of the kD-tree search as exact nearest neighbours in descriptor     */
/* space, one search per non-reference frame:                                  */
/*   temporal: grid targets in the box |u|, |v| <= fmax;                       */
/*   stereo:   epipolar -- same row, 0 <= d0 <= dmax;                          */
/*   cross:    epipolar -- row y + v*, 0 <= d1 <= dmax, target x + u* - s d1;  */
/* targets restricted to the level grid (multiples of n) inside the image,     */
/* ties to the smallest target index y*W + x.  The single combination of the   */
/* three returned leaves is the hypothesis; its cost is eq. (1).              */
/* ------------------------------------------------------------------------- */
int orc_init_nn_leaves(const int16_t* l0, const int16_t* l1, const int16_t* r0,
                       const int16_t* r1, int H, int W, int C, int level, int s, int fmax,
                       int dmax, int leaves, int nthreads, int16_t* hyp, uint32_t* cost);

int orc_init_nn(const int16_t* l0, const int16_t* l1, const int16_t* r0, const int16_t* r1,
                int H, int W, int C, int level, int s, int fmax, int dmax, int nthreads,
                int16_t* hyp, uint32_t* cost) {
    return orc_init_nn_leaves(l0, l1, r0, r1, H, W, C, level, s, fmax, dmax, 1, nthreads, hyp,
                              cost);
}

/* The same initialisation with several leaves of the temporal tree: the     */
/* `leaves` temporal targets of smallest descriptor distance (ties to the     */
/* smaller target index), each combined with its own cross partner (argmin on */
/* its row y + v) and with the stereo partner, all combinations compared by   */
/* the data term eq. (1) (the paper's "comparing all combinations of the      */
/* leafs").  Eq. (1) is a sum over the three views, so more stereo or cross   */
/* leaves cannot change the winner: the best combination pairs each temporal  */
/* leaf with the best cross target of its row.  Ties between combinations go  */
/* to the earlier temporal leaf.  leaves = 1 is the plain initialisation.     */
int orc_init_nn_leaves(const int16_t* l0, const int16_t* l1, const int16_t* r0,
                       const int16_t* r1, int H, int W, int C, int level, int s, int fmax,
                       int dmax, int leaves, int nthreads, int16_t* hyp, uint32_t* cost) {
    if (leaves < 1) return ORC_ERR;
    const int n = 1 << level;
    const int Hk = (H + n - 1) / n, Wk = (W + n - 1) / n;
    orc_views V = make_views(l0, l1, r0, r1, H, W, C, s);
    const int fm = (fmax / n) * n, dm = (dmax / n) * n;
    set_threads(nthreads);
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < Hk; ++i) {
        uint32_t* le = (uint32_t*)malloc(sizeof(uint32_t) * leaves);
        int* lu = (int*)malloc(sizeof(int) * leaves);
        int* lv = (int*)malloc(sizeof(int) * leaves);
        if (!le || !lu || !lv) {
            free(le); free(lu); free(lv);
#pragma omp atomic write
            fail = 1;
            continue;
        }
        for (int j = 0; j < Wk; ++j) {
            const int x = n * j, y = n * i;
            /* temporal partner: the `leaves` best targets, scanned in
             * increasing linear index, kept sorted by distance; a target
             * enters after every kept target of equal distance (the earlier
             * index stays first) */
            int nl = 0;
            for (int v = -fm; v <= fm; v += n) {
                int ty = y + v;
                if (ty < 0 || ty >= H) continue;
                for (int u = -fm; u <= fm; u += n) {
                    int tx = x + u;
                    if (tx < 0 || tx >= W) continue;
                    uint32_t e = ssd_at(&V, V.T, x, y, tx, ty);
                    if (nl == leaves && e >= le[nl - 1]) continue;
                    int pos = nl < leaves ? nl : leaves - 1;
                    while (pos > 0 && le[pos - 1] > e) {
                        le[pos] = le[pos - 1]; lu[pos] = lu[pos - 1]; lv[pos] = lv[pos - 1];
                        --pos;
                    }
                    le[pos] = e; lu[pos] = u; lv[pos] = v;
                    if (nl < leaves) ++nl;
                }
            }
            /* stereo partner, same row: target tx = x - s*d0 */
            uint32_t bestS = UINT32_MAX;
            int bd0 = 0;
            for (int tx = 0; tx < W; ++tx) {
                int d0 = s * (x - tx);
                if (d0 < 0 || d0 > dm || (d0 % n) != 0) continue;
                uint32_t e = ssd_at(&V, V.S, x, y, tx, y);
                if (e < bestS) { bestS = e; bd0 = d0; }
            }
            /* each temporal leaf with its cross partner on row y + v:
             * target tx = x + u - s*d1; keep the cheapest combination */
            uint64_t bestJ = UINT64_MAX;
            int bu = 0, bv = 0, bd1 = 0;
            for (int l = 0; l < nl; ++l) {
                uint32_t bestX = UINT32_MAX;
                int d1l = 0;
                for (int tx = 0; tx < W; ++tx) {
                    int d1 = s * (x + lu[l] - tx);
                    if (d1 < 0 || d1 > dm || (d1 % n) != 0) continue;
                    uint32_t e = ssd_at(&V, V.X, x, y, tx, y + lv[l]);
                    if (e < bestX) { bestX = e; d1l = d1; }
                }
                const uint64_t joint = (uint64_t)le[l] + bestS + bestX;
                if (joint < bestJ) { bestJ = joint; bu = lu[l]; bv = lv[l]; bd1 = d1l; }
            }
            int16_t* h = hyp + ((size_t)i * Wk + j) * 4;
            h[0] = (int16_t)bu; h[1] = (int16_t)bv; h[2] = (int16_t)bd0; h[3] = (int16_t)bd1;
            cost[(size_t)i * Wk + j] = cost_eq1(&V, x, y, h);
        }
        free(le); free(lu); free(lv);
    }
    return fail ? ORC_ERR : ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Multi-scale propagation and random search (Section 3.1, "Multi-Scale      */
/* Propagation").  One level k, grid G_k = {(n j, n i)}.                      */
/*                                                                           */
/* Readings: (1) hand-off -- for k below the coarsest level, every pixel      */
/* starts from its parent's vector (i >> 1, j >> 1) with the cost recomputed */
/* at level k ("let the propagation fill the gaps"); vectors are kept in      */
/* full-resolution pixels.  (2) Propagation uses the four directions equally  */
/* in a red-black order: per iteration, first all pixels with (i + j) even,   */
/* then all with (i + j) odd; a pixel takes a neighbour's vector only if its  */
/* cost is strictly smaller, neighbours scanned left, up, right, down.        */
/* (3) Random search follows each colour's propagation: S samples around the  */
/* propagated vector, sample t drawn uniformly on the integers of            */
/* [-r_t, r_t] per component with r_t = max(1, R0 >> t) * n (pixel units of  */
/* the current scale), clamped to the search bounds, kept only on strict      */
/* improvement.  (4) Random numbers: Philox4x32-10 with key = seed and        */
/* counter (i*Wk + j, it, (k << 16) | (t << 8) | (s < 0), 0); component c     */
/* offset = floor(x_c (2r+1) / 2^32) - r.                                     */
/* ------------------------------------------------------------------------- */
typedef struct {
    int iters, rs_r0, rs_samples, fmax, dmax;
} orc_level_params;

static void hyp_copy(int16_t* dst, const int16_t* src) {
    dst[0] = src[0]; dst[1] = src[1]; dst[2] = src[2]; dst[3] = src[3];
}

/* Random-search sample t of grid pixel (i, j) in iteration it: each component
 * of the centre moves by an integer drawn uniformly from [-r_t, r_t],
 * r_t = max(1, R0 >> t) * n, then is clamped to the search bounds. */
void orc_rs_candidate(uint64_t seed, int level, int s, int i, int j, int Wk, int it, int t,
                      int rs_r0, int fmax, int dmax, const int16_t centre[4], int16_t cand[4]) {
    const int n = 1 << level;
    int r = rs_r0 >> t;
    if (r < 1) r = 1;
    r *= n;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const uint32_t ctr[4] = {(uint32_t)(i * Wk + j), (uint32_t)it,
                             ((uint32_t)level << 16) | ((uint32_t)t << 8) | (s < 0 ? 1u : 0u), 0u};
    uint32_t rnd[4];
    orc_philox4x32_10(ctr, key, rnd);
    int off[4];
    for (int c = 0; c < 4; ++c) off[c] = (int)(((uint64_t)rnd[c] * (uint64_t)(2 * r + 1)) >> 32) - r;
    cand[0] = (int16_t)clampi(centre[0] + off[0], -fmax, fmax);
    cand[1] = (int16_t)clampi(centre[1] + off[1], -fmax, fmax);
    cand[2] = (int16_t)clampi(centre[2] + off[2], 0, dmax);
    cand[3] = (int16_t)clampi(centre[3] + off[3], 0, dmax);
}

static void update_pixel(const orc_views* V, int level, int Hk, int Wk, int i, int j, int it,
                         uint64_t seed, const orc_level_params* P, int16_t* hyp, uint32_t* cost) {
    const int n = 1 << level;
    const int x = n * j, y = n * i;
    int16_t* own = hyp + ((size_t)i * Wk + j) * 4;
    int16_t best[4];
    hyp_copy(best, own);
    uint32_t bestc = cost[(size_t)i * Wk + j];
    /* propagation: left, up, right, down */
    const int di[4] = {0, -1, 0, 1};
    const int dj[4] = {-1, 0, 1, 0};
    for (int q = 0; q < 4; ++q) {
        int ni = i + di[q], nj = j + dj[q];
        if (ni < 0 || ni >= Hk || nj < 0 || nj >= Wk) continue;
        const int16_t* nh = hyp + ((size_t)ni * Wk + nj) * 4;
        uint32_t c = cost_eq1(V, x, y, nh);
        if (c < bestc) { bestc = c; hyp_copy(best, nh); }
    }
    /* random search around the propagated vector */
    int16_t centre[4];
    hyp_copy(centre, best);
    for (int t = 0; t < P->rs_samples; ++t) {
        int16_t cand[4];
        orc_rs_candidate(seed, level, V->s, i, j, Wk, it, t, P->rs_r0, P->fmax, P->dmax, centre,
                         cand);
        uint32_t c = cost_eq1(V, x, y, cand);
        if (c < bestc) { bestc = c; hyp_copy(best, cand); }
    }
    hyp_copy(own, best);
    cost[(size_t)i * Wk + j] = bestc;
}

/* hyp/cost: level-k field [Hk][Wk].  If hyp_coarse is non-NULL it is the
 * level k+1 field and the hand-off initialises hyp/cost; otherwise hyp/cost
 * already hold the starting field (the initialisation at the coarsest level).
 * order = 1 visits the pixels of each colour in reverse (race-freedom check). */
int orc_match_level(const int16_t* l0, const int16_t* l1, const int16_t* r0, const int16_t* r1,
                    int H, int W, int C, int level, int s, uint64_t seed, int iters, int rs_r0,
                    int rs_samples, int fmax, int dmax, const int16_t* hyp_coarse, int order,
                    int nthreads, int16_t* hyp, uint32_t* cost) {
    const int n = 1 << level;
    const int Hk = (H + n - 1) / n, Wk = (W + n - 1) / n;
    orc_views V = make_views(l0, l1, r0, r1, H, W, C, s);
    orc_level_params P = {iters, rs_r0, rs_samples, fmax, dmax};
    set_threads(nthreads);
    if (hyp_coarse) {
        const int Wc = (W + 2 * n - 1) / (2 * n);
#pragma omp parallel for schedule(static)
        for (int i = 0; i < Hk; ++i)
            for (int j = 0; j < Wk; ++j) {
                int16_t* h = hyp + ((size_t)i * Wk + j) * 4;
                hyp_copy(h, hyp_coarse + ((size_t)(i >> 1) * Wc + (j >> 1)) * 4);
                cost[(size_t)i * Wk + j] = cost_eq1(&V, n * j, n * i, h);
            }
    }
    for (int it = 0; it < iters; ++it)
        for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(dynamic, 4)
            for (int ii = 0; ii < Hk; ++ii) {
                int i = order ? (Hk - 1 - ii) : ii;
                for (int jj = 0; jj < Wk; ++jj) {
                    int j = order ? (Wk - 1 - jj) : jj;
                    if (((i + j) & 1) != colour) continue;
                    update_pixel(&V, level, Hk, Wk, i, j, it, seed, &P, hyp, cost);
                }
            }
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* The paper's own propagation schedule (Section 3.1, "Multi-Scale            */
/* Propagation"), kept to measure what the red-black Jacobi schedule changes  */
/* (CPU only).  Iteration it scans the grid sequentially from corner it mod 4 */
/* (top-left, bottom-right, top-right, bottom-left), so each direction is     */
/* used equally; each pixel takes the cheapest of its own vector and the      */
/* vectors of its two already-visited neighbours (the one before it in the   */
/* row, then the one in the previous row; strict improvement), so a better    */
/* vector travels along the whole scan path.  After the scan every pixel runs */
/* the random search around its vector, with the same samples as the         */
/* red-black schedule (iteration counter it).                                 */
/* ------------------------------------------------------------------------- */
int orc_match_level_scan(const int16_t* l0, const int16_t* l1, const int16_t* r0,
                         const int16_t* r1, int H, int W, int C, int level, int s, uint64_t seed,
                         int iters, int rs_r0, int rs_samples, int fmax, int dmax,
                         const int16_t* hyp_coarse, int nthreads, int16_t* hyp, uint32_t* cost) {
    const int n = 1 << level;
    const int Hk = (H + n - 1) / n, Wk = (W + n - 1) / n;
    orc_views V = make_views(l0, l1, r0, r1, H, W, C, s);
    set_threads(nthreads);
    if (hyp_coarse) {
        const int Wc = (W + 2 * n - 1) / (2 * n);
        for (int i = 0; i < Hk; ++i)
            for (int j = 0; j < Wk; ++j) {
                int16_t* h = hyp + ((size_t)i * Wk + j) * 4;
                hyp_copy(h, hyp_coarse + ((size_t)(i >> 1) * Wc + (j >> 1)) * 4);
                cost[(size_t)i * Wk + j] = cost_eq1(&V, n * j, n * i, h);
            }
    }
    for (int it = 0; it < iters; ++it) {
        const int dir = it & 3;
        const int sy = (dir == 0 || dir == 2) ? 1 : -1;  /* rows top-down or bottom-up */
        const int sx = (dir == 0 || dir == 3) ? 1 : -1;  /* columns left-right or right-left */
        for (int ii = 0; ii < Hk; ++ii) {
            const int i = sy > 0 ? ii : Hk - 1 - ii;
            for (int jj = 0; jj < Wk; ++jj) {
                const int j = sx > 0 ? jj : Wk - 1 - jj;
                int16_t* own = hyp + ((size_t)i * Wk + j) * 4;
                uint32_t* oc = cost + (size_t)i * Wk + j;
                const int pi[2] = {i, i - sy}, pj[2] = {j - sx, j};
                for (int q = 0; q < 2; ++q) {
                    if (pi[q] < 0 || pi[q] >= Hk || pj[q] < 0 || pj[q] >= Wk) continue;
                    const int16_t* nh = hyp + ((size_t)pi[q] * Wk + pj[q]) * 4;
                    const uint32_t c = cost_eq1(&V, n * j, n * i, nh);
                    if (c < *oc) { *oc = c; hyp_copy(own, nh); }
                }
            }
        }
#pragma omp parallel for schedule(dynamic, 4)
        for (int i = 0; i < Hk; ++i)
            for (int j = 0; j < Wk; ++j) {
                int16_t* own = hyp + ((size_t)i * Wk + j) * 4;
                int16_t centre[4], best[4];
                hyp_copy(centre, own);
                hyp_copy(best, own);
                uint32_t bestc = cost[(size_t)i * Wk + j];
                for (int t = 0; t < rs_samples; ++t) {
                    int16_t cand[4];
                    orc_rs_candidate(seed, level, s, i, j, Wk, it, t, rs_r0, fmax, dmax, centre, cand);
                    const uint32_t c = cost_eq1(&V, n * j, n * i, cand);
                    if (c < bestc) { bestc = c; hyp_copy(best, cand); }
                }
                hyp_copy(own, best);
                cost[(size_t)i * Wk + j] = bestc;
            }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Consistency check (Section 3.1, "Consistency Check"; tau_c, Section 5).    */
/* The inverse field has reference I_r^1.  At the cross target q = p +        */
/* (u - d1, v) its vector (u', v', d0', d1') implies a left flow               */
/* (d0' - u' - d1', -v'), a disparity d1' at t0 and d0' at t1.  Reading: the   */
/* vector survives iff all three forward targets lie inside the image and     */
/* (d0 - d1')^2 <= tau^2, (d1 - d0')^2 <= tau^2 and the Euclidean flow         */
/* difference |(u + u' + d1' - d0', v + v')|^2 <= tau^2.  err = the largest of */
/* the three squares, UINT32_MAX when a target is outside the image.          */
/* ------------------------------------------------------------------------- */
int orc_consistency(const int16_t* hyp_fwd, const int16_t* hyp_inv, int H, int W, int tau,
                    uint8_t* valid, uint32_t* err) {
    const int64_t t2 = (int64_t)tau * tau;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const int16_t* h = hyp_fwd + ((size_t)y * W + x) * 4;
            const int u = h[0], v = h[1], d0 = h[2], d1 = h[3];
            const size_t o = (size_t)y * W + x;
            int txT = x + u, tyT = y + v, txS = x - d0, txX = x + u - d1, tyX = y + v;
            int inb = txT >= 0 && txT < W && tyT >= 0 && tyT < H && txS >= 0 && txS < W &&
                      txX >= 0 && txX < W && tyX >= 0 && tyX < H;
            if (!inb) {
                valid[o] = 0;
                err[o] = UINT32_MAX;
                continue;
            }
            const int16_t* g = hyp_inv + ((size_t)tyX * W + txX) * 4;
            const int64_t ui = g[0], vi = g[1], d0i = g[2], d1i = g[3];
            int64_t e0 = (int64_t)d0 - d1i;
            int64_t e1 = (int64_t)d1 - d0i;
            int64_t efx = (int64_t)u + ui + d1i - d0i;
            int64_t efy = (int64_t)v + vi;
            int64_t a = e0 * e0, b = e1 * e1, f = efx * efx + efy * efy;
            int64_t m = a > b ? a : b;
            m = m > f ? m : f;
            valid[o] = (a <= t2 && b <= t2 && f <= t2) ? 1 : 0;
            err[o] = (uint32_t)m;
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Region filter (Section 3.1, "Consistency Check", second step; s_c, Section */
/* 5).  The consistent pixels are grouped into regions: two 4-neighbours     */
/* belong to one region when both are consistent and their vectors are       */
/* approximately the same -- read as every component (u, v, d0, d1) differing */
/* by at most tau px.  A region is removed when it has fewer than s_c pixels  */
/* and one of the already removed pixels (consistency outliers) next to it   */
/* could be added by the same rule, i.e. some inconsistent 4-neighbour of a  */
/* region pixel has approximately that pixel's vector.                        */
/* hyp: forward field int16 [H][W][4]; valid: consistency result u8 [H][W];   */
/* keep: u8 [H][W] output, 1 for a surviving match.                           */
/* Plain breadth-first region growing in raster order.                        */
/* ------------------------------------------------------------------------- */
static int similar_vec(const int16_t* a, const int16_t* b, int tau) {
    for (int c = 0; c < 4; ++c) {
        const int d = (int)a[c] - (int)b[c];
        if (d > tau || d < -tau) return 0;
    }
    return 1;
}

int orc_region_filter(const int16_t* hyp, const uint8_t* valid, int H, int W, int tau, int s_c,
                      uint8_t* keep) {
    const size_t npx = (size_t)H * W;
    int32_t* label = (int32_t*)malloc(sizeof(int32_t) * npx);
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * npx);
    int32_t* size = (int32_t*)malloc(sizeof(int32_t) * npx);
    uint8_t* flag = (uint8_t*)malloc(npx);
    if (!label || !queue || !size || !flag) {
        free(label); free(queue); free(size); free(flag);
        return ORC_ERR;
    }
    static const int DX[4] = {-1, 1, 0, 0}, DY[4] = {0, 0, -1, 1};
    for (size_t p = 0; p < npx; ++p) label[p] = -1;
    int nreg = 0;
    for (int y0 = 0; y0 < H; ++y0)
        for (int x0 = 0; x0 < W; ++x0) {
            const size_t p0 = (size_t)y0 * W + x0;
            if (!valid[p0] || label[p0] >= 0) continue;
            /* grow region nreg from p0 */
            size_t head = 0, tail = 0;
            label[p0] = nreg;
            queue[tail++] = (int32_t)p0;
            while (head < tail) {
                const int32_t p = queue[head++];
                const int x = p % W, y = p / W;
                for (int k = 0; k < 4; ++k) {
                    const int xn = x + DX[k], yn = y + DY[k];
                    if (xn < 0 || xn >= W || yn < 0 || yn >= H) continue;
                    const size_t q = (size_t)yn * W + xn;
                    if (!valid[q] || label[q] >= 0) continue;
                    if (!similar_vec(hyp + (size_t)p * 4, hyp + q * 4, tau)) continue;
                    label[q] = nreg;
                    queue[tail++] = (int32_t)q;
                }
            }
            size[nreg] = (int32_t)tail;
            flag[nreg] = 0;
            ++nreg;
        }
    /* outliers that could join a neighbouring region */
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const size_t p = (size_t)y * W + x;
            if (valid[p]) continue;
            for (int k = 0; k < 4; ++k) {
                const int xn = x + DX[k], yn = y + DY[k];
                if (xn < 0 || xn >= W || yn < 0 || yn >= H) continue;
                const size_t q = (size_t)yn * W + xn;
                if (valid[q] && similar_vec(hyp + p * 4, hyp + q * 4, tau)) flag[label[q]] = 1;
            }
        }
    for (size_t p = 0; p < npx; ++p)
        keep[p] = (valid[p] && !(flag[label[p]] && size[label[p]] < s_c)) ? 1 : 0;
    free(label); free(queue); free(size); free(flag);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Sparsification (Section 3.2 "Sparsification"): in every non-overlapping    */
/* 3 x 3 block (aligned at the origin; blocks at the right and bottom border  */
/* are cut by the image), the surviving match with the lowest consistency     */
/* error; ties to the lowest raster index y * W + x.  seeds: int32             */
/* [ceil(H/3)][ceil(W/3)], the pixel index y * W + x, or -1 for a block       */
/* without a surviving match.                                                 */
/* ------------------------------------------------------------------------- */
int orc_sparsify(const uint8_t* keep, const uint32_t* err, int H, int W, int32_t* seeds) {
    const int Hb = (H + 2) / 3, Wb = (W + 2) / 3;
    for (int bi = 0; bi < Hb; ++bi)
        for (int bj = 0; bj < Wb; ++bj) {
            int32_t best = -1;
            for (int y = 3 * bi; y < 3 * bi + 3 && y < H; ++y)
                for (int x = 3 * bj; x < 3 * bj + 3 && x < W; ++x) {
                    const int32_t p = y * W + x;
                    if (keep[p] && (best < 0 || err[p] < err[best])) best = p;
                }
            seeds[(size_t)bi * Wb + bj] = best;
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Disparity fill (Section 3.1, "Consistency Check", last paragraph): a second */
/* disparity map by semi-global matching (Hirschmueller, TPAMI 2008) and a    */
/* check of the disparity matches alone against it with the same tau.        */
/* Readings (the paper only cites SGM): grey = rounded mean of the channels;  */
/* 5 x 5 census (bit k set when neighbour k, row-major without the centre, is */
/* darker than the centre; replicated border); matching cost = Hamming        */
/* distance of the census words of (x, y) in the left and (x - d, y) in the   */
/* right image, x - d clamped to the image, d = 0..D-1; aggregation along 8   */
/* paths with penalties P1 (|change| = 1) and P2 (larger changes); the        */
/* disparity minimises the summed path costs, ties to the smaller d.          */
/* ------------------------------------------------------------------------- */
static uint32_t census5(const uint8_t* g, int H, int W, int x, int y) {
    const int c = g[(size_t)y * W + x];
    uint32_t w = 0;
    int k = 0;
    for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
            if (dx == 0 && dy == 0) continue;
            const int v = g[(size_t)clampi(y + dy, 0, H - 1) * W + clampi(x + dx, 0, W - 1)];
            if (v < c) w |= 1u << k;
            ++k;
        }
    return w;
}

static int popcount32(uint32_t v) {
    int n = 0;
    while (v) { v &= v - 1; ++n; }
    return n;
}

/* grey: uint8 [H][W] from an image [H][W][C]. */
int orc_grey(const uint8_t* img, int H, int W, int C, uint8_t* grey) {
    for (size_t p = 0; p < (size_t)H * W; ++p) {
        int sum = 0;
        for (int c = 0; c < C; ++c) sum += img[p * C + c];
        grey[p] = (uint8_t)((sum + C / 2) / C);
    }
    return ORC_OK;
}

/* census: uint32 [H][W] of a grey image. */
int orc_census(const uint8_t* grey, int H, int W, uint32_t* out) {
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) out[(size_t)y * W + x] = census5(grey, H, W, x, y);
    return ORC_OK;
}

/* cost: uint8 [H][W][D], Hamming distance of the census words. */
int orc_sgm_cost(const uint32_t* cl, const uint32_t* cr, int H, int W, int D, uint8_t* cost) {
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int d = 0; d < D; ++d)
                cost[((size_t)y * W + x) * D + d] =
                    (uint8_t)popcount32(cl[(size_t)y * W + x] ^ cr[(size_t)y * W + clampi(x - d, 0, W - 1)]);
    return ORC_OK;
}

/* Aggregated cost along one path direction (dx, dy) (each in -1..1, not both
 * 0): L(p, d) = C(p, d) + min(L(q, d), L(q, d - 1) + P1, L(q, d + 1) + P1,
 * min_k L(q, k) + P2) - min_k L(q, k) with q = p - (dx, dy); L(p, d) = C(p, d)
 * where q lies outside the image.  L: int32 [H][W][D]. */
int orc_sgm_path(const uint8_t* cost, int H, int W, int D, int P1, int P2, int dx, int dy,
                 int32_t* L) {
    /* visit pixels so that q = p - (dx, dy) is always done before p */
    for (int yy = 0; yy < H; ++yy) {
        const int y = dy >= 0 ? yy : H - 1 - yy;
        for (int xx = 0; xx < W; ++xx) {
            const int x = dx >= 0 ? xx : W - 1 - xx;
            const uint8_t* c = cost + ((size_t)y * W + x) * D;
            int32_t* l = L + ((size_t)y * W + x) * D;
            const int qx = x - dx, qy = y - dy;
            if (qx < 0 || qx >= W || qy < 0 || qy >= H) {
                for (int d = 0; d < D; ++d) l[d] = c[d];
                continue;
            }
            const int32_t* lq = L + ((size_t)qy * W + qx) * D;
            int32_t m = lq[0];
            for (int d = 1; d < D; ++d) m = lq[d] < m ? lq[d] : m;
            for (int d = 0; d < D; ++d) {
                int32_t best = lq[d];
                if (d > 0 && lq[d - 1] + P1 < best) best = lq[d - 1] + P1;
                if (d + 1 < D && lq[d + 1] + P1 < best) best = lq[d + 1] + P1;
                if (m + P2 < best) best = m + P2;
                l[d] = c[d] + best - m;
            }
        }
    }
    return ORC_OK;
}

/* SGM disparity of a rectified pair (left, right images [H][W][C]): disp
 * int16 [H][W] in 0..D-1. */
int orc_sgm(const uint8_t* left, const uint8_t* right, int H, int W, int C, int D, int P1, int P2,
            int16_t* disp) {
    const size_t npx = (size_t)H * W;
    uint8_t* gl = (uint8_t*)malloc(npx);
    uint8_t* gr = (uint8_t*)malloc(npx);
    uint32_t* cl = (uint32_t*)malloc(sizeof(uint32_t) * npx);
    uint32_t* cr = (uint32_t*)malloc(sizeof(uint32_t) * npx);
    uint8_t* cost = (uint8_t*)malloc(npx * D);
    int32_t* L = (int32_t*)malloc(sizeof(int32_t) * npx * D);
    int32_t* S = (int32_t*)calloc(npx * D, sizeof(int32_t));
    int rc = ORC_ERR;
    if (gl && gr && cl && cr && cost && L && S) {
        orc_grey(left, H, W, C, gl);
        orc_grey(right, H, W, C, gr);
        orc_census(gl, H, W, cl);
        orc_census(gr, H, W, cr);
        orc_sgm_cost(cl, cr, H, W, D, cost);
        static const int DIRS[8][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1},
                                       {1, 1}, {-1, -1}, {1, -1}, {-1, 1}};
        for (int r = 0; r < 8; ++r) {
            orc_sgm_path(cost, H, W, D, P1, P2, DIRS[r][0], DIRS[r][1], L);
            for (size_t k = 0; k < npx * D; ++k) S[k] += L[k];
        }
        for (size_t p = 0; p < npx; ++p) {
            int best = 0;
            for (int d = 1; d < D; ++d)
                if (S[p * D + d] < S[p * D + best]) best = d;
            disp[p] = (int16_t)best;
        }
        rc = ORC_OK;
    }
    free(gl); free(gr); free(cl); free(cr); free(cost); free(L); free(S);
    return rc;
}

/* Disparity fill: fill[p] = 1 where the joint check kept the match, or where
 * it removed it but the match's own disparity d0 lies inside the image target
 * and within tau of the SGM disparity.  hyp: forward field [H][W][4]. */
int orc_disparity_fill(const int16_t* hyp, const uint8_t* valid, const int16_t* disp, int H,
                       int W, int tau, uint8_t* fill) {
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const size_t p = (size_t)y * W + x;
            const int d0 = hyp[p * 4 + 2];
            const int e = d0 - disp[p];
            fill[p] = (valid[p] || (x - d0 >= 0 && e <= tau && e >= -tau)) ? 1 : 0;
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Whole stage for one pair (Section 3 overview up to the consistency check): */
/* descriptors of the four images at every level, then for the forward        */
/* (s = +1) and inverse (s = -1) fields: exact-NN initialisation at the       */
/* coarsest level, propagation + random search from the coarsest level down   */
/* to full resolution, and finally the consistency check.                    */
/* imgs: uint8 [4][H][W][C] in order (l0, l1, r0, r1).                        */
/* hyp_out: int16 [2][H][W][4] (forward, inverse), cost_out uint32 [2][H][W]. */
/* ------------------------------------------------------------------------- */
int orc_match_pair_schedule(const uint8_t* imgs, int H, int W, int C, int levels, int iters,
                            int rs_r0, int rs_samples, int fmax, int dmax, int tau, uint64_t seed,
                            int nthreads, int scan, int leaves, int16_t* hyp_out,
                            uint32_t* cost_out, uint8_t* valid, uint32_t* err);

int orc_match_pair(const uint8_t* imgs, int H, int W, int C, int levels, int iters, int rs_r0,
                   int rs_samples, int fmax, int dmax, int tau, uint64_t seed, int nthreads,
                   int16_t* hyp_out, uint32_t* cost_out, uint8_t* valid, uint32_t* err) {
    return orc_match_pair_schedule(imgs, H, W, C, levels, iters, rs_r0, rs_samples, fmax, dmax,
                                   tau, seed, nthreads, 0, 1, hyp_out, cost_out, valid, err);
}

/* scan = 0: red-black schedule (the one the GPU path implements); scan = 1:
 * the sequential four-corner schedule above.  leaves: temporal leaves of the
 * initialisation (1 = the plain one). */
int orc_match_pair_schedule(const uint8_t* imgs, int H, int W, int C, int levels, int iters,
                            int rs_r0, int rs_samples, int fmax, int dmax, int tau, uint64_t seed,
                            int nthreads, int scan, int leaves, int16_t* hyp_out,
                            uint32_t* cost_out, uint8_t* valid, uint32_t* err) {
    const size_t npx = (size_t)H * W;
    const size_t dsz = npx * C * 16;
    int16_t* desc = (int16_t*)malloc(sizeof(int16_t) * dsz * 4);
    int16_t* hyp_c = (int16_t*)malloc(sizeof(int16_t) * npx * 4);
    if (!desc || !hyp_c) {
        free(desc); free(hyp_c);
        return ORC_ERR;
    }
    set_threads(nthreads);
    for (int k = levels - 1; k >= 0; --k) {
        for (int m = 0; m < 4; ++m)
            orc_features(imgs + npx * C * m, H, W, C, k, desc + dsz * m);
        const int16_t *l0 = desc, *l1 = desc + dsz, *r0 = desc + 2 * dsz, *r1 = desc + 3 * dsz;
        for (int dir = 0; dir < 2; ++dir) {
            const int s = dir == 0 ? 1 : -1;
            int16_t* hyp = hyp_out + (size_t)dir * npx * 4;
            uint32_t* cst = cost_out + (size_t)dir * npx;
            if (k == levels - 1) {
                if (orc_init_nn_leaves(l0, l1, r0, r1, H, W, C, k, s, fmax, dmax, leaves, nthreads,
                                       hyp, cst) != ORC_OK) {
                    free(desc); free(hyp_c);
                    return ORC_ERR;
                }
                if (scan)
                    orc_match_level_scan(l0, l1, r0, r1, H, W, C, k, s, seed, iters, rs_r0,
                                         rs_samples, fmax, dmax, NULL, nthreads, hyp, cst);
                else
                    orc_match_level(l0, l1, r0, r1, H, W, C, k, s, seed, iters, rs_r0, rs_samples,
                                    fmax, dmax, NULL, 0, nthreads, hyp, cst);
            } else {
                const int n = 1 << (k + 1);
                const size_t nc = (size_t)((H + n - 1) / n) * ((W + n - 1) / n);
                memcpy(hyp_c, hyp, sizeof(int16_t) * nc * 4);
                if (scan)
                    orc_match_level_scan(l0, l1, r0, r1, H, W, C, k, s, seed, iters, rs_r0,
                                         rs_samples, fmax, dmax, hyp_c, nthreads, hyp, cst);
                else
                    orc_match_level(l0, l1, r0, r1, H, W, C, k, s, seed, iters, rs_r0, rs_samples,
                                    fmax, dmax, hyp_c, 0, nthreads, hyp, cst);
            }
        }
    }
    orc_consistency(hyp_out, hyp_out + npx * 4, H, W, tau, valid, err);
    free(desc); free(hyp_c);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Full-resolution matching with the paper's own cost (Section 3.1,          */
/* "Matching Cost", eq. (1), and "Multi-Scale Propagation" at the finest      */
/* scale), starting from a given field.  Features phi [4][H][W][4] float      */
/* (first three principal components of the SIFT features, views l0, l1, r0, */
/* r1; the fourth component is ignored).  Cost of h at (x, y), in FP32 with   */
/* every operation rounded as written (the library computes the same sums in  */
/* the same order):                                                          */
/*   for wy = -3..3, wx = -3..3, for the temporal, stereo, cross partners in  */
/*   that order: sum += sqrt(e0^2 + e1^2 + e2^2), e = phi_R(clamp(p + w)) -   */
/*   phi_corr(clamp(p + w + o_corr)), squares added left to right.            */
/* Schedule, tie rule and random search as in orc_match_level at level 0,     */
/* with its own random stream: the counter's level field is 16 (no image      */
/* level reaches it) and the radii are R0 >> t (n = 1).                       */
/* ------------------------------------------------------------------------- */
typedef struct {
    const float *R, *T, *S, *X;
    int H, W, s;
} orc_fviews;

static float fdist3(const float* a, const float* b) {
    const float e0 = a[0] - b[0], e1 = a[1] - b[1], e2 = a[2] - b[2];
    float q = e0 * e0;
    const float q1 = e1 * e1;
    q = q + q1;
    const float q2 = e2 * e2;
    q = q + q2;
    return sqrtf(q);
}

static float cost_sift(const orc_fviews* V, int x, int y, const int16_t h[4]) {
    const int H = V->H, W = V->W, s = V->s;
    const int u = h[0], v = h[1], d0 = h[2], d1 = h[3];
    float sum = 0.f;
    for (int wy = -3; wy <= 3; ++wy)
        for (int wx = -3; wx <= 3; ++wx) {
            const int py = y + wy, px = x + wx;
            const float* r = V->R + ((size_t)clampi(py, 0, H - 1) * W + clampi(px, 0, W - 1)) * 4;
            const float* t = V->T + ((size_t)clampi(py + v, 0, H - 1) * W + clampi(px + u, 0, W - 1)) * 4;
            const float* sv = V->S + ((size_t)clampi(py, 0, H - 1) * W + clampi(px - s * d0, 0, W - 1)) * 4;
            const float* xv =
                V->X + ((size_t)clampi(py + v, 0, H - 1) * W + clampi(px + u - s * d1, 0, W - 1)) * 4;
            sum = sum + fdist3(r, t);
            sum = sum + fdist3(r, sv);
            sum = sum + fdist3(r, xv);
        }
    return sum;
}

/* Exposed for tests: eq. (1) with SIFT-PCA features at every pixel. */
int orc_cost_sift(const float* phi, int H, int W, int s, const int16_t* hyp, float* cost) {
    const size_t npx = (size_t)H * W;
    orc_fviews V = {phi + (size_t)(s > 0 ? 0 : 3) * npx * 4, phi + (size_t)(s > 0 ? 1 : 2) * npx * 4,
                    phi + (size_t)(s > 0 ? 2 : 1) * npx * 4, phi + (size_t)(s > 0 ? 3 : 0) * npx * 4,
                    H, W, s};
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) cost[(size_t)y * W + x] = cost_sift(&V, x, y, hyp + ((size_t)y * W + x) * 4);
    return ORC_OK;
}

#define ORC_SIFT_LEVEL_TAG 16

static void update_pixel_sift(const orc_fviews* V, int i, int j, int it, uint64_t seed,
                              const orc_level_params* P, int16_t* hyp, float* cost) {
    const int H = V->H, W = V->W;
    int16_t* own = hyp + ((size_t)i * W + j) * 4;
    int16_t best[4];
    hyp_copy(best, own);
    float bestc = cost[(size_t)i * W + j];
    const int di[4] = {0, -1, 0, 1};
    const int dj[4] = {-1, 0, 1, 0};
    for (int q = 0; q < 4; ++q) {
        const int ni = i + di[q], nj = j + dj[q];
        if (ni < 0 || ni >= H || nj < 0 || nj >= W) continue;
        const int16_t* nh = hyp + ((size_t)ni * W + nj) * 4;
        const float c = cost_sift(V, j, i, nh);
        if (c < bestc) { bestc = c; hyp_copy(best, nh); }
    }
    int16_t centre[4];
    hyp_copy(centre, best);
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int t = 0; t < P->rs_samples; ++t) {
        int r = P->rs_r0 >> t;
        if (r < 1) r = 1;
        const uint32_t ctr[4] = {(uint32_t)(i * W + j), (uint32_t)it,
                                 ((uint32_t)ORC_SIFT_LEVEL_TAG << 16) | ((uint32_t)t << 8) |
                                     (V->s < 0 ? 1u : 0u),
                                 0u};
        uint32_t rnd[4];
        orc_philox4x32_10(ctr, key, rnd);
        int off[4];
        for (int c = 0; c < 4; ++c) off[c] = (int)(((uint64_t)rnd[c] * (uint64_t)(2 * r + 1)) >> 32) - r;
        int16_t cand[4];
        cand[0] = (int16_t)clampi(centre[0] + off[0], -P->fmax, P->fmax);
        cand[1] = (int16_t)clampi(centre[1] + off[1], -P->fmax, P->fmax);
        cand[2] = (int16_t)clampi(centre[2] + off[2], 0, P->dmax);
        cand[3] = (int16_t)clampi(centre[3] + off[3], 0, P->dmax);
        const float c = cost_sift(V, j, i, cand);
        if (c < bestc) { bestc = c; hyp_copy(best, cand); }
    }
    hyp_copy(own, best);
    cost[(size_t)i * W + j] = bestc;
}

/* hyp [H][W][4] in/out (the starting field), cost [H][W] out. */
int orc_match_sift(const float* phi, int H, int W, int s, uint64_t seed, int iters, int rs_r0,
                   int rs_samples, int fmax, int dmax, int order, int nthreads, int16_t* hyp,
                   float* cost) {
    const size_t npx = (size_t)H * W;
    orc_fviews V = {phi + (size_t)(s > 0 ? 0 : 3) * npx * 4, phi + (size_t)(s > 0 ? 1 : 2) * npx * 4,
                    phi + (size_t)(s > 0 ? 2 : 1) * npx * 4, phi + (size_t)(s > 0 ? 3 : 0) * npx * 4,
                    H, W, s};
    orc_level_params P = {iters, rs_r0, rs_samples, fmax, dmax};
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) cost[(size_t)y * W + x] = cost_sift(&V, x, y, hyp + ((size_t)y * W + x) * 4);
    for (int it = 0; it < iters; ++it)
        for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(dynamic, 4)
            for (int ii = 0; ii < H; ++ii) {
                const int i = order ? (H - 1 - ii) : ii;
                for (int jj = 0; jj < W; ++jj) {
                    const int j = order ? (W - 1 - jj) : jj;
                    if (((i + j) & 1) != colour) continue;
                    update_pixel_sift(&V, i, j, it, seed, &P, hyp, cost);
                }
            }
        }
    return ORC_OK;
}
