// The paper's own matching cost (SceneFlowFields, Section 3.1, "Matching
// Cost", eq. (1)): per pixel, the Euclidean distances between the first three
// principal components of dense SIFT features, summed over a 7 x 7 window and
// the temporal, stereo and cross correspondences; principal axes from the SIFT
// features of all four images of the pair; boundary pixels replicated.
//
// Dense SIFT as in SIFT flow (Liu et al., TPAMI 2011) after Lowe (IJCV 2004):
// central-difference gradients, 8 orientation bins of 45 degrees with linear
// interpolation between bin centres, 4 x 4 cells of 3 x 3 pixels around the
// pixel (rows and columns -6 .. +5, flat window, clamped), unit length, clamp
// at 0.2, unit length again.  The gradients are taken on the channel sum
// (integers, exact in FP32): a constant factor changes neither orientations
// nor the normalised descriptor.
//
// Pipeline of sff_sift_pca: orientation planes -> cell-sum planes -> Gram
// matrix and sum of all descriptors of the pair (FP64 accumulation, partial
// per block, reduced in a fixed order) -> covariance -> the three leading
// eigenvectors (subspace iteration on a power of the covariance, in one
// block) -> projected features.
// Descriptors are recomputed from the cell-sum planes in the Gram and the
// projection pass instead of being stored (512 B per pixel).
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "sff_internal.hpp"

namespace sff {
namespace {

constexpr int kBins = 8;
constexpr int kCell = 3;
constexpr int kHalf = 6;                    // descriptor window -6 .. +5
constexpr int kExt = 2 * kHalf - kCell;     // 9 extra rows / columns of the cell-sum planes
constexpr int kDesc = 128;
constexpr float kClampV = 0.2f;
constexpr int kGramPx = 64;                 // descriptors per Gram step (4 threads each)
constexpr int kMaxGramBlocks = 512;  // two blocks per CU
constexpr int kPart = kDesc * kDesc + kDesc;  // doubles per Gram partial
constexpr int kSub = 8;                     // subspace dimension of the eigen iteration
constexpr int kCheck = 4;                   // iterations between Rayleigh-Ritz checks
constexpr int kMaxIter = 4000;
constexpr int kWinR = 3;                    // cost window -3 .. +3
constexpr int kCT = 16;                     // cost tile side

struct SiftGeom {
    int H, W, He, We;
    size_t npx, plane_o, plane_c;  // pixels, orientation plane, cell-sum plane (elements)
};

inline SiftGeom sift_geom(const sff_params& p) {
    SiftGeom g;
    g.H = p.H;
    g.W = p.W;
    g.He = p.H + kExt;
    g.We = p.W + kExt;
    g.npx = (size_t)p.H * p.W;
    g.plane_o = g.npx;
    g.plane_c = (size_t)g.He * g.We;
    return g;
}

inline int gram_blocks(const SiftGeom& g) {
    const size_t per = 4 * g.npx;
    const size_t nb = (per + 32 * kGramPx - 1) / (32 * kGramPx);
    return (int)std::max<size_t>(1, std::min<size_t>(kMaxGramBlocks, nb));
}

struct SiftWs {
    size_t O, Cs, part, gsum, sq, ax32, total;
};

inline SiftWs sift_ws(const SiftGeom& g, int nimg) {
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const int pairs = (nimg + 3) / 4;
    SiftWs L;
    L.O = 0;
    L.Cs = L.O + al((size_t)nimg * kBins * g.plane_o * sizeof(float));
    L.part = L.Cs + al((size_t)nimg * kBins * g.plane_c * sizeof(float));
    L.gsum = L.part + al((size_t)pairs * gram_blocks(g) * kPart * sizeof(double));
    L.sq = L.gsum + al((size_t)pairs * kPart * sizeof(double));
    L.ax32 = L.sq + al((size_t)pairs * 2 * kDesc * kDesc * sizeof(double));
    L.total = L.ax32 + al((size_t)pairs * 4 * kDesc * sizeof(float));
    return L;
}

// ------------------------------------------------------------------ SIFT --

// Orientation energy of one pixel: the gradient magnitude split between the
// two bins whose centres enclose its orientation; 8 planes per image.
__global__ void __launch_bounds__(256) orient_kernel(const uint8_t* __restrict__ img,
                                                     float* __restrict__ O, int H, int W, int C) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= H * W) return;
    const int m = blockIdx.y;
    const uint8_t* im = img + (size_t)m * H * W * C;
    const int y = p / W, x = p - y * W;
    auto sum = [&](int yy, int xx) {
        const uint8_t* q = im + ((size_t)yy * W + xx) * C;
        int t = 0;
        for (int c = 0; c < C; ++c) t += q[c];
        return t;
    };
    const float gx = (float)(sum(y, min(x + 1, W - 1)) - sum(y, max(x - 1, 0)));
    const float gy = (float)(sum(min(y + 1, H - 1), x) - sum(max(y - 1, 0), x));
    const float mag = sqrtf(gx * gx + gy * gy);  // exact integers below 2^24 under the root
    float pos = atan2f(gy, gx) * (float)(4.0 / M_PI);
    if (pos < 0.f) pos += 8.f;
    const float lo = floorf(pos);
    const float frac = pos - lo;
    const int b0 = (int)lo & 7, b1 = (b0 + 1) & 7;
    float* o = O + (size_t)m * kBins * H * W + p;
#pragma unroll
    for (int b = 0; b < kBins; ++b)
        o[(size_t)b * H * W] = b == b0 ? mag * (1.f - frac) : (b == b1 ? mag * frac : 0.f);
}

// Cs[m][Y + 6][X + 6][b] = sum of O[m][b] over the 3 x 3 cell whose top-left
// pixel is (Y, X), coordinates clamped; Y in -6 .. H + 2, X in -6 .. W + 2.
// The 8 bins of a cell are contiguous (32 bytes, two 16-byte loads).
__global__ void __launch_bounds__(256) cellsum_kernel(const float* __restrict__ O,
                                                      float* __restrict__ Cs, int H, int W) {
    const int He = H + kExt, We = W + kExt;
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= He * We) return;
    const int m = blockIdx.y;
    const int Yr = q / We;
    const int Y = Yr - kHalf, X = q - Yr * We - kHalf;
    int ys[kCell], xs[kCell];
#pragma unroll
    for (int a = 0; a < kCell; ++a) {
        ys[a] = clampi(Y + a, 0, H - 1);
        xs[a] = clampi(X + a, 0, W - 1);
    }
    const float* o = O + (size_t)m * kBins * H * W;
    float sum[kBins];
#pragma unroll
    for (int b = 0; b < kBins; ++b) {
        const float* ob = o + (size_t)b * H * W;
        float s = 0.f;
#pragma unroll
        for (int a = 0; a < kCell; ++a)
#pragma unroll
            for (int c = 0; c < kCell; ++c) s += ob[(size_t)ys[a] * W + xs[c]];
        sum[b] = s;
    }
    float4* cs = reinterpret_cast<float4*>(Cs + ((size_t)m * He * We + q) * kBins);
    cs[0] = make_float4(sum[0], sum[1], sum[2], sum[3]);
    cs[1] = make_float4(sum[4], sum[5], sum[6], sum[7]);
}

// Sum over the 4 lanes of a quad (DPP quad permutations).
__device__ __forceinline__ float quad_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
    return v;
}

// Quarter q (cell row q: 4 cells x 8 bins, descriptor entries 32 q .. 32 q + 31)
// of the normalised descriptor of pixel (y, x); the 4 quarters of a pixel sit in
// one quad of lanes, which must all be active.
__device__ __forceinline__ void desc_quarter(const float* __restrict__ cs, int He, int We, int y, int x,
                                             int q, float (&v)[32]) {
    const float4* row = reinterpret_cast<const float4*>(cs + ((size_t)(y + kCell * q) * We + x) * kBins);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float4 lo = row[2 * kCell * j], hi = row[2 * kCell * j + 1];
        v[8 * j + 0] = lo.x;
        v[8 * j + 1] = lo.y;
        v[8 * j + 2] = lo.z;
        v[8 * j + 3] = lo.w;
        v[8 * j + 4] = hi.x;
        v[8 * j + 5] = hi.y;
        v[8 * j + 6] = hi.z;
        v[8 * j + 7] = hi.w;
    }
    float ss = 0.f;
#pragma unroll
    for (int k = 0; k < 32; ++k) ss += v[k] * v[k];
    ss = quad_sum(ss);
    if (ss > 0.f) {
        const float n = sqrtf(ss);
        float s2 = 0.f;
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            v[k] = fminf(v[k] / n, kClampV);
            s2 += v[k] * v[k];
        }
        s2 = quad_sum(s2);
        const float n2 = sqrtf(s2);
#pragma unroll
        for (int k = 0; k < 32; ++k) v[k] = v[k] / n2;
    }
}

// Dense SIFT written out: [nimg][H][W][128], 64 pixels per block.
__global__ void __launch_bounds__(256) sift_out_kernel(const float* __restrict__ Cs, float* __restrict__ out,
                                                       int H, int W, int nimg) {
    const int He = H + kExt, We = W + kExt;
    const int t = threadIdx.x, q = t & 3;
    const long total = (long)nimg * H * W;
    const long g = (long)blockIdx.x * kGramPx + (t >> 2);
    const long ge = g < total ? g : total - 1;  // whole quads stay active
    const int m = (int)(ge / ((long)H * W));
    const int p = (int)(ge - (long)m * H * W);
    const int y = p / W, x = p - y * W;
    float v[32];
    desc_quarter(Cs + (size_t)m * kBins * He * We, He, We, y, x, q, v);
    if (g >= total) return;
    float4* o = reinterpret_cast<float4*>(out + (size_t)ge * kDesc + 32 * q);
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
}

// ------------------------------------------------------------------- PCA --

// Gram matrix and sum of the descriptors of one pair (4 H W of them), FP64:
// each block takes every nblk-th group of 64 descriptors and stages them in
// LDS; the 36 upper-triangle 16 x 16 tiles of the Gram matrix accumulate on
// the FP64 matrix cores (v_mfma_f64_16x16x4f64: A = 16 descriptor entries of 4
// pixels, B = 16 entries of the same pixels).  Wave w owns the tile rows w and
// 7 - w (9 tiles); the operand of tile column J is also the A operand of tile
// row J, so each 4-pixel step loads 8 - w values per lane.  Partials (upper
// tiles only) go to part[pair][block].
struct GramArgs {
    const float* Cs;
    double* part;
    int H, W, nblk;
};

typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int W>
__device__ __forceinline__ void gram_tiles(const float (*D)[kDesc + 4], int lane, f64x4 (&acc)[9]) {
    constexpr int I1 = 7 - W;
    const int li = lane & 15, lk = lane >> 4;
    for (int k0 = 0; k0 < kGramPx; k0 += 4) {
        double b[8];
#pragma unroll
        for (int J = W; J < 8; ++J) b[J] = (double)D[k0 + lk][16 * J + li];
        int n = 0;
#pragma unroll
        for (int J = W; J < 8; ++J, ++n) acc[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[W], b[J], acc[n], 0, 0, 0);
#pragma unroll
        for (int J = I1; J < 8; ++J, ++n)
            if (I1 != W) acc[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[I1], b[J], acc[n], 0, 0, 0);
    }
}

template <int W>
__device__ __forceinline__ void gram_store(double* part, int lane, const f64x4 (&acc)[9]) {
    constexpr int I1 = 7 - W;
    // accumulator element v of lane l: row l / 16 + 4 v, column l % 16 of the
    // tile (the operands: A[l % 16][l / 16], B[l / 16][l % 16])
    const int col = lane & 15, row0 = lane >> 4;
    int n = 0;
#pragma unroll
    for (int J = W; J < 8; ++J, ++n)
#pragma unroll
        for (int v = 0; v < 4; ++v) part[(size_t)(16 * W + row0 + 4 * v) * kDesc + 16 * J + col] = acc[n][v];
#pragma unroll
    for (int J = I1; J < 8; ++J, ++n)
        if (I1 != W)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                part[(size_t)(16 * I1 + row0 + 4 * v) * kDesc + 16 * J + col] = acc[n][v];
}

__global__ void __launch_bounds__(256) gram_kernel(GramArgs a) {
    __shared__ float D[kGramPx][kDesc + 4];
    const int t = threadIdx.x, q = t & 3, px = t >> 2, lane = t & 63, w = wave_id();
    const int H = a.H, W = a.W, He = H + kExt, We = W + kExt;
    const long npx = (long)H * W, total = 4 * npx;
    const int pair = blockIdx.y;
    const float* Cs = a.Cs + (size_t)pair * 4 * kBins * He * We;
    f64x4 acc[9];
#pragma unroll
    for (int n = 0; n < 9; ++n) acc[n] = f64x4{0.0, 0.0, 0.0, 0.0};
    double sacc = 0.0;
    for (long base = (long)blockIdx.x * kGramPx; base < total; base += (long)a.nblk * kGramPx) {
        const long g = base + px;
        const long ge = g < total ? g : total - 1;
        const int m = (int)(ge / npx);
        const int p = (int)(ge - m * npx);
        const int y = p / W, x = p - y * W;
        float v[32];
        desc_quarter(Cs + (size_t)m * kBins * He * We, He, We, y, x, q, v);
#pragma unroll
        for (int k = 0; k < 32; ++k) D[px][32 * q + k] = g < total ? v[k] : 0.f;
        __syncthreads();
        switch (w) {  // wave-uniform
            case 0: gram_tiles<0>(D, lane, acc); break;
            case 1: gram_tiles<1>(D, lane, acc); break;
            case 2: gram_tiles<2>(D, lane, acc); break;
            default: gram_tiles<3>(D, lane, acc); break;
        }
        if (t < kDesc)
            for (int k = 0; k < kGramPx; ++k) sacc += (double)D[k][t];
        __syncthreads();
    }
    double* part = a.part + ((size_t)pair * a.nblk + blockIdx.x) * kPart;
    switch (w) {
        case 0: gram_store<0>(part, lane, acc); break;
        case 1: gram_store<1>(part, lane, acc); break;
        case 2: gram_store<2>(part, lane, acc); break;
        default: gram_store<3>(part, lane, acc); break;
    }
    if (t < kDesc) part[kDesc * kDesc + t] = sacc;
}

// Partials summed per entry (upper tiles of G, then S) with 8 interleaved
// accumulators combined in a fixed order: deterministic.
constexpr int kSumEntries = kDesc * kDesc + kDesc;
__global__ void __launch_bounds__(256) gram_sum_kernel(const double* __restrict__ part, int nblk,
                                                       double* __restrict__ gsum) {
    const int e = blockIdx.x * 256 + threadIdx.x, pair = blockIdx.y;
    if (e >= kSumEntries) return;
    if (e < kDesc * kDesc && ((e / kDesc) >> 4) > ((e % kDesc) >> 4)) return;  // lower tile: not stored
    const double* P = part + (size_t)pair * nblk * kPart + e;
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int b = 0;
    for (; b + 8 <= nblk; b += 8)
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] += P[(size_t)(b + u) * kPart];
    for (; b < nblk; ++b) s[0] += P[(size_t)b * kPart];
    gsum[(size_t)pair * kSumEntries + e] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// mean = S / N, cov = G / N - mean mean^T (G from its upper tiles).
__global__ void __launch_bounds__(kDesc) gram_cov_kernel(const double* __restrict__ gsum, double inv_n,
                                                        double* __restrict__ mean, double* __restrict__ cov) {
    const int r = blockIdx.x, pair = blockIdx.y, c = threadIdx.x;
    const double* g = gsum + (size_t)pair * kSumEntries;
    const bool up = (r >> 4) <= (c >> 4);
    const double grc = g[up ? (size_t)r * kDesc + c : (size_t)c * kDesc + r];
    const double mr = g[kDesc * kDesc + r] * inv_n, mc = g[kDesc * kDesc + c] * inv_n;
    cov[((size_t)pair * kDesc + r) * kDesc + c] = grc * inv_n - mr * mc;
    if (r == 0) mean[(size_t)pair * kDesc + c] = mc;
}

// Small dense linear algebra of one thread, every loop fully unrolled so
// that the arrays stay in registers.

// Rinv = R^-1 for G = R^T R (Cholesky, R upper).  A column that is
// (numerically) in the span of the previous ones keeps a unit diagonal and no
// coupling instead of being scaled up, so a rank-deficient covariance cannot
// make the iteration overflow.
__device__ __forceinline__ void chol_inverse(const double (*Gs)[kSub], double (*Rinv_out)[kSub]) {
    double R[kSub][kSub], Ri[kSub][kSub];
    double gmax = 0.0;
#pragma unroll
    for (int i = 0; i < kSub; ++i) gmax = fmax(gmax, Gs[i][i]);
#pragma unroll
    for (int j = 0; j < kSub; ++j) {
#pragma unroll
        for (int i = 0; i < kSub; ++i) R[i][j] = 0.0;
#pragma unroll
        for (int i = 0; i < j; ++i) {
            double s = Gs[i][j];
#pragma unroll
            for (int k = 0; k < i; ++k) s -= R[k][i] * R[k][j];
            R[i][j] = s / R[i][i];
        }
        double s = Gs[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= R[k][j] * R[k][j];
        if (s > 1e-24 * gmax && gmax > 0.0) {
            R[j][j] = sqrt(s);
        } else {
#pragma unroll
            for (int i = 0; i < j; ++i) R[i][j] = 0.0;
            R[j][j] = 1.0;
        }
    }
#pragma unroll
    for (int j = 0; j < kSub; ++j) {
#pragma unroll
        for (int i = 0; i < kSub; ++i) Ri[i][j] = 0.0;
        Ri[j][j] = 1.0 / R[j][j];
#pragma unroll
        for (int i = j - 1; i >= 0; --i) {
            double s = 0.0;
#pragma unroll
            for (int k = i + 1; k <= j; ++k) s += R[i][k] * Ri[k][j];
            Ri[i][j] = -s / R[i][i];
        }
    }
#pragma unroll
    for (int i = 0; i < kSub; ++i)
#pragma unroll
        for (int j = 0; j < kSub; ++j) Rinv_out[i][j] = Ri[i][j];
}

// Eigenpairs of the symmetric part of Ts by cyclic Jacobi rotations, sorted by
// eigenvalue, largest first: values to th_out, vectors to the columns of S_out.
__device__ __forceinline__ void ritz_small(const double (*Ts)[kSub], double* th_out, double (*S_out)[kSub]) {
    double A[kSub][kSub], V[kSub][kSub];
#pragma unroll
    for (int i = 0; i < kSub; ++i)
#pragma unroll
        for (int j = 0; j < kSub; ++j) {
            A[i][j] = 0.5 * (Ts[i][j] + Ts[j][i]);
            V[i][j] = i == j ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 40; ++sweep) {
        double off = 0.0, tot = 0.0;
#pragma unroll
        for (int i = 0; i < kSub; ++i)
#pragma unroll
            for (int j = 0; j < kSub; ++j) {
                tot += A[i][j] * A[i][j];
                if (i != j) off += A[i][j] * A[i][j];
            }
        if (off <= 1e-32 * tot) break;
#pragma unroll
        for (int p = 0; p < kSub - 1; ++p)
#pragma unroll
            for (int q = p + 1; q < kSub; ++q) {
                const double apq = A[p][q];
                if (apq != 0.0) {
                    const double th = (A[q][q] - A[p][p]) / (2.0 * apq);
                    const double tt = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                    const double c = 1.0 / sqrt(tt * tt + 1.0), s = tt * c;
#pragma unroll
                    for (int k = 0; k < kSub; ++k) {
                        const double akp = A[k][p], akq = A[k][q];
                        A[k][p] = c * akp - s * akq;
                        A[k][q] = s * akp + c * akq;
                    }
#pragma unroll
                    for (int k = 0; k < kSub; ++k) {
                        const double apk = A[p][k], aqk = A[q][k];
                        A[p][k] = c * apk - s * aqk;
                        A[q][k] = s * apk + c * aqk;
                    }
#pragma unroll
                    for (int k = 0; k < kSub; ++k) {
                        const double vkp = V[k][p], vkq = V[k][q];
                        V[k][p] = c * vkp - s * vkq;
                        V[k][q] = s * vkp + c * vkq;
                    }
                }
            }
    }
    double d[kSub];
#pragma unroll
    for (int i = 0; i < kSub; ++i) d[i] = A[i][i];
    // selection order, largest first (columns swapped along)
#pragma unroll
    for (int i = 0; i < kSub; ++i)
#pragma unroll
        for (int j = i + 1; j < kSub; ++j) {
            const bool sw = d[j] > d[i];
            const double di = d[i], dj = d[j];
            d[i] = sw ? dj : di;
            d[j] = sw ? di : dj;
#pragma unroll
            for (int k = 0; k < kSub; ++k) {
                const double vi = V[k][i], vj = V[k][j];
                V[k][i] = sw ? vj : vi;
                V[k][j] = sw ? vi : vj;
            }
        }
#pragma unroll
    for (int i = 0; i < kSub; ++i) {
        th_out[i] = d[i];
#pragma unroll
        for (int j = 0; j < kSub; ++j) S_out[i][j] = V[i][j];
    }
}

// Sum over the block (256 threads) of one double per thread.
__device__ double block_sum(double v, double* red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// The three leading eigenvectors of one pair's covariance A.  The SIFT
// covariance has a flat spectrum (neighbouring eigenvalues within a few
// percent), so plain subspace iteration converges slowly; the iteration runs
// on M = A^(2^kSquare) instead (same eigenvectors, ratios raised to that
// power), formed beforehand by square_kernel (squarings normalised by the
// trace).  Subspace iteration with
// kSub vectors: Z = M Q, Q = orth(Z) (Cholesky QR, twice).  Every kCheck-th
// step multiplies by A itself and does a Rayleigh-Ritz step in span(Q): Ritz
// pairs of A and their residuals ||A y - theta y|| (A y = Z s); it stops when
// the three leading residuals are below 1e-12 theta_1 (or after kMaxIter).
// The matrices are read from global memory (symmetric: row r of M Q is read
// down column r, coalesced).  Each axis is signed so that its component of
// largest magnitude is positive.  Also writes the FP32 axes and mean used by
// the projection.
constexpr int kSquare = 6;  // A^64: KITTI-size pair 1.68 ms of features vs 1.78 with A^32 (A^128: no gain)

// One 16 x 16 tile of C = B B / trace(B B) per block, for a symmetric B:
// trace(B B) = |B|_F^2, summed by every block in the same order (so all tiles
// share one scale), and C[r][c] = sum_k B[k][r] B[k][c] with the two factors
// of a term commuting in fma, so C is exactly symmetric again.
__global__ void __launch_bounds__(256) square_kernel(const double* __restrict__ B_all, size_t b_stride,
                                                     double* __restrict__ C_all, size_t c_stride) {
    __shared__ double colr[kDesc][16], colc[kDesc][16];
    __shared__ double red[256];
    const int t = threadIdx.x, ti = blockIdx.x >> 3, tj = blockIdx.x & 7;
    const double* B = B_all + (size_t)blockIdx.y * b_stride;
    double* C = C_all + (size_t)blockIdx.y * c_stride;
    // four independent partial sums so the 64 loads of a thread are in flight together
    double f4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int e = t; e < kDesc * kDesc; e += 1024)
#pragma unroll
        for (int u = 0; u < 4; ++u) f4[u] = fma(B[e + 256 * u], B[e + 256 * u], f4[u]);
    const double f = block_sum((f4[0] + f4[1]) + (f4[2] + f4[3]), red);
#pragma unroll
    for (int e = t; e < kDesc * 16; e += 256) {
        const int k = e >> 4, c = e & 15;
        colr[k][c] = B[(size_t)k * kDesc + 16 * ti + c];
        colc[k][c] = B[(size_t)k * kDesc + 16 * tj + c];
    }
    __syncthreads();
    const int r = t >> 4, c = t & 15;
    double acc = 0.0;
    for (int k = 0; k < kDesc; ++k) acc = fma(colr[k][r], colc[k][c], acc);
    const double sc = f > 0.0 ? 1.0 / f : 1.0;
    C[(size_t)(16 * ti + r) * kDesc + 16 * tj + c] = acc * sc;
}

__global__ void __launch_bounds__(256) eig_kernel(const double* __restrict__ cov_all,
                                                  const double* __restrict__ mean_all,
                                                  double* __restrict__ sq_all, double* __restrict__ eigval,
                                                  double* __restrict__ axes, float* __restrict__ ax32) {
    __shared__ double Q[kSub][kDesc], Z[kSub][kDesc];
    __shared__ double G[kSub][kSub], Rinv[kSub][kSub], S[kSub][kSub], th[kSub];
    __shared__ double red[256];
    __shared__ int done;
    const int t = threadIdx.x, pair = blockIdx.x;
    const double* A = cov_all + (size_t)pair * kDesc * kDesc;
    double* sq = sq_all + (size_t)pair * 2 * kDesc * kDesc;
    const int r = t & (kDesc - 1), h = t >> 7;  // row and vector half (4 vectors)

    // M = A^(2^kSquare), trace-normalised at each squaring (square_kernel)
    const double* M = sq + (size_t)((kSquare - 1) & 1) * kDesc * kDesc;

    // deterministic pseudo-random start
    for (int i = t; i < kSub * kDesc; i += 256) {
        uint32_t z = (uint32_t)(i + 1) * 2654435761u;
        z ^= z >> 15;
        z *= 2246822519u;
        z ^= z >> 13;
        Z[i / kDesc][i % kDesc] = (double)(z & 0xFFFF) / 32768.0 - 1.0;
    }
    __syncthreads();

    // Q = orth(Z) by Cholesky QR, twice
    auto orth = [&]() {
        for (int pass = 0; pass < 2; ++pass) {
            if (t < kSub * kSub) {
                const int i = t / kSub, j = t % kSub;
                double s = 0.0;
                for (int k = 0; k < kDesc; ++k) s = fma(Z[i][k], Z[j][k], s);
                G[i][j] = s;
            }
            __syncthreads();
            if (t == 0) chol_inverse(G, Rinv);
            __syncthreads();
            double z[kSub];
#pragma unroll
            for (int u = 0; u < kSub; ++u) z[u] = Z[u][r];
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int vv = 4 * h + u;
                double s = 0.0;
#pragma unroll
                for (int w = 0; w < kSub; ++w)
                    if (w <= vv) s = fma(z[w], Rinv[w][vv], s);
                Z[vv][r] = s;
            }
            __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) Q[4 * h + u][r] = Z[4 * h + u][r];
        __syncthreads();
    };
    orth();

    for (int it = 1; it <= kMaxIter; ++it) {
        const bool check = it % kCheck == 0 || it == kMaxIter;
        const double* Mi = check ? A : M;
        {
            double s[4] = {0.0, 0.0, 0.0, 0.0};
            for (int k = 0; k < kDesc; ++k) {
                const double mk = Mi[(size_t)k * kDesc + r];
#pragma unroll
                for (int u = 0; u < 4; ++u) s[u] = fma(mk, Q[4 * h + u][k], s[u]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) Z[4 * h + u][r] = s[u];
        }
        __syncthreads();
        if (check) {
            // Rayleigh-Ritz on A: T = Q^T (A Q)
            if (t < kSub * kSub) {
                const int i = t / kSub, j = t % kSub;
                double s = 0.0;
                for (int k = 0; k < kDesc; ++k) s = fma(Q[i][k], Z[j][k], s);
                G[i][j] = s;
            }
            __syncthreads();
            if (t == 0) ritz_small(G, th, S);
            __syncthreads();
            double res[3];
            for (int k = 0; k < 3; ++k) {
                double az = 0.0, y = 0.0;
                if (t < kDesc) {
#pragma unroll
                    for (int i = 0; i < kSub; ++i) {
                        az = fma(Z[i][t], S[i][k], az);
                        y = fma(Q[i][t], S[i][k], y);
                    }
                }
                const double e = az - th[k] * y;
                res[k] = sqrt(block_sum(t < kDesc ? e * e : 0.0, red));
            }
            if (t == 0) {
                const double tol = 1e-12 * fabs(th[0]);
                done = (res[0] <= tol && res[1] <= tol && res[2] <= tol) || th[0] == 0.0 || it == kMaxIter;
            }
            __syncthreads();
            if (done) break;
        }
        orth();
    }

    // Ritz vectors y_k = Q s_k, signed, written out
    __shared__ double Y[3][kDesc];
    if (t < kDesc)
        for (int k = 0; k < 3; ++k) {
            double y = 0.0;
#pragma unroll
            for (int i = 0; i < kSub; ++i) y = fma(Q[i][t], S[i][k], y);
            Y[k][t] = y;
        }
    __syncthreads();
    if (t < 3) {
        int best = 0;
        for (int i = 1; i < kDesc; ++i)
            if (fabs(Y[t][i]) > fabs(Y[t][best])) best = i;
        red[t] = Y[t][best] < 0.0 ? -1.0 : 1.0;
        eigval[(size_t)pair * 3 + t] = th[t];
    }
    __syncthreads();
    if (t < kDesc) {
        for (int k = 0; k < 3; ++k) {
            const double y = red[k] * Y[k][t];
            axes[((size_t)pair * 3 + k) * kDesc + t] = y;
            ax32[((size_t)pair * 4 + k) * kDesc + t] = (float)y;
        }
        ax32[((size_t)pair * 4 + 3) * kDesc + t] = (float)mean_all[(size_t)pair * kDesc + t];
    }
}

// phi = axes (f - mean) per pixel of the pair's four images, float4 (phi, 0).
__global__ void __launch_bounds__(256) project_kernel(const float* __restrict__ Cs,
                                                      const float* __restrict__ ax32,
                                                      float4* __restrict__ phi, int H, int W) {
    const int He = H + kExt, We = W + kExt;
    const int t = threadIdx.x, q = t & 3;
    const long npx = (long)H * W, total = 4 * npx;
    const int pair = blockIdx.y;
    const long g = (long)blockIdx.x * kGramPx + (t >> 2);
    const long ge = g < total ? g : total - 1;
    const int m = (int)(ge / npx);
    const int p = (int)(ge - m * npx);
    const int y = p / W, x = p - y * W;
    float v[32];
    desc_quarter(Cs + ((size_t)pair * 4 + m) * kBins * He * We, He, We, y, x, q, v);
    const float* ax = ax32 + (size_t)pair * 4 * kDesc + 32 * q;
    float f[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        const float d = v[k] - ax[3 * kDesc + k];
#pragma unroll
        for (int c = 0; c < 3; ++c) f[c] = fmaf(ax[c * kDesc + k], d, f[c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) f[c] = quad_sum(f[c]);
    if (g < total && q == 0) phi[(size_t)pair * total + ge] = make_float4(f[0], f[1], f[2], 0.f);
}

// ------------------------------------------------------------------ cost --

// Euclidean distance of the first three components, every operation rounded
// as written (no contraction), so that sums agree bit for bit with the FP32
// definition: ((e0^2 + e1^2) + e2^2), correctly rounded square root.  sqrtf
// is correctly rounded in this toolchain's default FP32 mode (a committed test
// checks it against the host); __fsqrt_rn is not (15% of 2^20 inputs differ by
// an ulp).  HIP contracts multiply-adds by default (the __f*_rn helpers
// included): switched off here, with plain operators under the pragma.
__device__ __forceinline__ float fdist3(float4 a, float4 b) {
#pragma clang fp contract(off)
    const float e0 = a.x - b.x, e1 = a.y - b.y, e2 = a.z - b.z;
    float q = e0 * e0;
    q = q + e1 * e1;
    q = q + e2 * e2;
    return sqrtf(q);
}

// Views of one field: (R, T, S, X) = (l0, l1, r0, r1) for s = +1 and
// (r1, r0, l1, l0) for s = -1.
struct SiftViews {
    const float4 *R, *T, *S, *X;
    int H, W, s;
};

__device__ __forceinline__ SiftViews sift_views(const float4* phi_pair, int H, int W, int s) {
    const size_t npx = (size_t)H * W;
    SiftViews V;
    V.R = phi_pair + (size_t)(s > 0 ? 0 : 3) * npx;
    V.T = phi_pair + (size_t)(s > 0 ? 1 : 2) * npx;
    V.S = phi_pair + (size_t)(s > 0 ? 2 : 1) * npx;
    V.X = phi_pair + (size_t)(s > 0 ? 3 : 0) * npx;
    V.H = H;
    V.W = W;
    V.s = s;
    return V;
}

// Eq. (1) of (u, v, d0, d1) at (x, y): window rows wy = -3..3, columns wx, and
// for each window pixel the temporal, stereo and cross distances, added in
// that order.  The terms are non-negative, so the partial sum only grows: once
// it reaches `bound` after a window row the remaining rows are skipped and a
// value >= bound is returned; below `bound` the exact sum is returned.
__device__ __forceinline__ float sift_cost_below(const SiftViews& V, int x, int y, int u, int v, int d0,
                                                 int d1, float bound) {
    const int H = V.H, W = V.W, s = V.s;
    float sum = 0.f;
    for (int wy = -kWinR; wy <= kWinR; ++wy) {
        const int py = y + wy;
        const size_t rr = (size_t)clampi(py, 0, H - 1) * W, rv = (size_t)clampi(py + v, 0, H - 1) * W;
#pragma unroll
        for (int wx = -kWinR; wx <= kWinR; ++wx) {
            const int px = x + wx;
            const float4 r = V.R[rr + clampi(px, 0, W - 1)];
            const float4 t = V.T[rv + clampi(px + u, 0, W - 1)];
            const float4 sv = V.S[rr + clampi(px - s * d0, 0, W - 1)];
            const float4 xv = V.X[rv + clampi(px + u - s * d1, 0, W - 1)];
            sum = sum + fdist3(r, t);
            sum = sum + fdist3(r, sv);
            sum = sum + fdist3(r, xv);
        }
        if (sum >= bound) return sum;
    }
    return sum;
}

// Eq. (1) at fixed vectors: one thread per pixel of a 16 x 16 tile.
__global__ void __launch_bounds__(256) cost_sift_kernel(const float4* __restrict__ phi,
                                                        const int16_t* __restrict__ hyp,
                                                        float* __restrict__ cost, int H, int W, int dir) {
    const int b = blockIdx.z;
    const size_t npx = (size_t)H * W;
    const SiftViews V = sift_views(phi + (size_t)b * 4 * npx, H, W, dir);
    const int y = blockIdx.y * kCT + threadIdx.x / kCT, x = blockIdx.x * kCT + threadIdx.x % kCT;
    if (y >= H || x >= W) return;
    const short4 h = reinterpret_cast<const short4*>(hyp)[(size_t)b * npx + (size_t)y * W + x];
    cost[(size_t)b * npx + (size_t)y * W + x] = sift_cost_below(V, x, y, h.x, h.y, h.z, h.w, INFINITY);
}

// Full-resolution matching with eq. (1) (Section 3.1, "Multi-Scale
// Propagation" at the finest scale): one red-black half-step of both fields.
// Per-lane form (SFF_SIFT_EVAL=lane; the wave-shared form follows further
// down): block = 4 image rows x 64 pixels of the half-step's colour; each lane
// scores its own candidates (left, up, right, down, then the random-search
// samples, one at a time, strict improvement).  Random stream: Philox4x32-10
// with the counter's level field 16 and radii R0 >> t.
struct SiftMatchArgs {
    const float4* phi;       // [batch][4][H][W]
    const uint64_t* seeds;   // [batch]
    int16_t* hyp;            // [ndir][batch][H][W][4]
    float* cost;             // [ndir][batch][H][W]
    int H, W, rs_r0, rs_samples, fmax, dmax, batch, ndir, dir0;
};

constexpr uint32_t kSiftLevelTag = 16;

__global__ void __launch_bounds__(256) sift_cost_init_kernel(SiftMatchArgs a) {
    const int z = blockIdx.y, di = z / a.batch, b = z - di * a.batch;
    const int s = a.ndir == 2 ? (di == 0 ? 1 : -1) : a.dir0;
    const size_t npx = (size_t)a.H * a.W;
    const int p = blockIdx.x * 256 + threadIdx.x;
    if ((size_t)p >= npx) return;
    const SiftViews V = sift_views(a.phi + (size_t)b * 4 * npx, a.H, a.W, s);
    const short4 h = reinterpret_cast<const short4*>(a.hyp)[(size_t)z * npx + p];
    a.cost[(size_t)z * npx + p] = sift_cost_below(V, p % a.W, p / a.W, h.x, h.y, h.z, h.w, INFINITY);
}

__global__ void __launch_bounds__(256) sift_half_step_kernel(SiftMatchArgs a, int it, int colour, int tiles_x,
                                                             int tiles_y) {
    const int per_field = tiles_x * tiles_y;
    const int z = blockIdx.x / per_field;
    const int tr = blockIdx.x - z * per_field;
    const int ty = tr / tiles_x, tx = tr - ty * tiles_x;
    const int lane = threadIdx.x & 63;
    const int i = ty * 4 + wave_id();
    if (i >= a.H) return;  // whole wave
    const int j = 2 * (tx * 64 + lane) + ((i + colour) & 1);
    const bool act = j < a.W;
    const int jj = min(j, a.W - 1);
    const int di = z / a.batch, b = z - di * a.batch;
    const int s = a.ndir == 2 ? (di == 0 ? 1 : -1) : a.dir0;
    const size_t npx = (size_t)a.H * a.W;
    const SiftViews V = sift_views(a.phi + (size_t)b * 4 * npx, a.H, a.W, s);
    short4* field = reinterpret_cast<short4*>(a.hyp) + (size_t)z * npx;
    float* cost = a.cost + (size_t)z * npx;
    const size_t o = (size_t)i * a.W + jj;
    short4 best = field[o];
    float bestc = cost[o];
    const short4 own = best;
    const int ni[4] = {i, i - 1, i, i + 1};
    const int nj[4] = {jj - 1, jj, jj + 1, jj};
    short4 nh[4];
    bool in[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        in[q] = act && ni[q] >= 0 && ni[q] < a.H && nj[q] >= 0 && nj[q] < a.W;
        nh[q] = in[q] ? field[(size_t)ni[q] * a.W + nj[q]] : own;
    }
    auto eq = [](short4 p, short4 q) { return p.x == q.x && p.y == q.y && p.z == q.z && p.w == q.w; };
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        // a vector equal to one already scored has the same cost: no strict improvement
        bool dup = eq(nh[q], own);
#pragma unroll
        for (int p = 0; p < q; ++p) dup = dup || (in[p] && eq(nh[q], nh[p]));
        const bool want = in[q] && !dup;
        if (!__any(want)) continue;
        if (want) {
            const float c = sift_cost_below(V, jj, i, nh[q].x, nh[q].y, nh[q].z, nh[q].w, bestc);
            if (c < bestc) {
                bestc = c;
                best = nh[q];
            }
        }
    }
    const short4 centre = best;
    const uint64_t seed = a.seeds[b];
    for (int t = 0; t < a.rs_samples; ++t) {
        const int r = max(1, a.rs_r0 >> t);
        U4 ctr;
        ctr.x = (uint32_t)(i * a.W + jj);
        ctr.y = (uint32_t)it;
        ctr.z = (kSiftLevelTag << 16) | ((uint32_t)t << 8) | (s < 0 ? 1u : 0u);
        ctr.w = 0u;
        const U4 rnd = philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32));
        short4 c;
        c.x = (short)clampi(centre.x + uniform_offset(rnd.x, r), -a.fmax, a.fmax);
        c.y = (short)clampi(centre.y + uniform_offset(rnd.y, r), -a.fmax, a.fmax);
        c.z = (short)clampi(centre.z + uniform_offset(rnd.z, r), 0, a.dmax);
        c.w = (short)clampi(centre.w + uniform_offset(rnd.w, r), 0, a.dmax);
        const bool want = act && !eq(c, centre);
        if (!__any(want)) continue;
        if (want) {
            const float cc = sift_cost_below(V, jj, i, c.x, c.y, c.z, c.w, bestc);
            if (cc < bestc) {
                bestc = cc;
                best = c;
            }
        }
    }
    if (act) {
        field[o] = best;
        cost[o] = bestc;
    }
}

// The same half-step with the window gathers shared by the wave (one wave per
// block, 64 pixels of the colour in one image row).  Per window row, slot
// f = 64 k + lane (k < 7) serves owner f / 7 at window column f % 7 - 3: it
// loads that column's R, T, S and X elements (the 7 columns of one owner are
// consecutive lanes, so a load instruction reads a few contiguous runs instead
// of 64 scattered elements) and writes the three distances to LDS; the owner
// then adds its 21 distances in the per-lane kernel's order (column, then
// temporal, stereo, cross), so every sum is the same FP32 value, and stops
// after the first row whose partial sum reaches the bound.  Tiles are
// numbered column-major and dealt to the XCDs in vertical strips, which keeps
// the window gathers of neighbouring tiles in one L2 (KITTI-size pair: one
// matching iteration 1.72 vs 2.45 ms with tiles dealt in launch order).
constexpr int kSiftSlots = 2 * kWinR + 1;           // slot loads per window row
constexpr int kDistStride = 3 * kSiftSlots + 3;     // 24 floats per owner in LDS

__device__ __forceinline__ void sift_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct SiftCoop {
    SiftViews V;
    float* dist;              // this wave's LDS [64][kDistStride]
    int lane, y;
    int so[kSiftSlots];       // owner of slot k
    int sx[kSiftSlots];       // x of the slot's window column (owner's x + offset)
    int sd[kSiftSlots];       // LDS word of the slot's first distance

    // Eq. (1) of each owner's (u, v, d0, d1) at its pixel (x_o, y), the same
    // value as sift_cost_below (>= bound once a row's partial sum reaches it).
    // want = false: no candidate, result meaningless.  Called by all lanes.
    __device__ __forceinline__ float cost_below(bool want, short4 h, float bound) const {
        const int H = V.H, W = V.W, s = V.s;
        const uint32_t uv = (uint32_t)(uint16_t)h.x | ((uint32_t)(uint16_t)h.y << 16);
        const uint32_t dd = (uint32_t)(uint16_t)h.z | ((uint32_t)(uint16_t)h.w << 16);
        int su[kSiftSlots], svv[kSiftSlots], sd0[kSiftSlots], sd1[kSiftSlots];
#pragma unroll
        for (int k = 0; k < kSiftSlots; ++k) {
            const uint32_t a = (uint32_t)__shfl((int)uv, so[k]), b = (uint32_t)__shfl((int)dd, so[k]);
            su[k] = (int)(int16_t)(a & 0xFFFFu);
            svv[k] = (int)(int16_t)(a >> 16);
            sd0[k] = (int)(int16_t)(b & 0xFFFFu);
            sd1[k] = (int)(int16_t)(b >> 16);
        }
        float sum = 0.f;
        bool alive = want;
        for (int wy = -kWinR; wy <= kWinR; ++wy) {
            if (!__any(alive)) break;
            const int py = clampi(y + wy, 0, H - 1);
#pragma unroll
            for (int k = 0; k < kSiftSlots; ++k) {
                if (__shfl((int)alive, so[k])) {
                    const int pyv = clampi(y + wy + svv[k], 0, H - 1);
                    const int px = sx[k];
                    const float4 r = V.R[py * W + clampi(px, 0, W - 1)];
                    const float4 t = V.T[pyv * W + clampi(px + su[k], 0, W - 1)];
                    const float4 sv = V.S[py * W + clampi(px - s * sd0[k], 0, W - 1)];
                    const float4 xv = V.X[pyv * W + clampi(px + su[k] - s * sd1[k], 0, W - 1)];
                    dist[sd[k] + 0] = fdist3(r, t);
                    dist[sd[k] + 1] = fdist3(r, sv);
                    dist[sd[k] + 2] = fdist3(r, xv);
                }
            }
            sift_wave_sync();
            if (alive) {
                const float* d = dist + lane * kDistStride;
#pragma unroll
                for (int e = 0; e < 3 * kSiftSlots; ++e) sum = sum + d[e];
                alive = sum < bound;
            }
            sift_wave_sync();
        }
        return sum;
    }
};

__global__ void __launch_bounds__(64) sift_half_step_coop_kernel(SiftMatchArgs a, int it, int colour,
                                                                 int tiles_x) {
    __shared__ float dist_lds[64 * kDistStride];
    const int per_field = tiles_x * a.H;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);  // column-major tiles, a strip per XCD
    const int z = tile / per_field;
    const int tr = tile - z * per_field;
    const int tx = tr / a.H, i = tr - tx * a.H;
    const int lane = threadIdx.x;
    const int par = (i + colour) & 1;
    const int j = 2 * (tx * 64 + lane) + par;
    const bool act = j < a.W;
    const int jj = min(j, a.W - 1);
    const int di = z / a.batch, b = z - di * a.batch;
    const int s = a.ndir == 2 ? (di == 0 ? 1 : -1) : a.dir0;
    const size_t npx = (size_t)a.H * a.W;
    SiftCoop E;
    E.V = sift_views(a.phi + (size_t)b * 4 * npx, a.H, a.W, s);
    E.dist = dist_lds;
    E.lane = lane;
    E.y = i;
#pragma unroll
    for (int k = 0; k < kSiftSlots; ++k) {
        const int f = 64 * k + lane, o = f / kSiftSlots, c = f - kSiftSlots * o;
        E.so[k] = o;
        E.sx[k] = min(2 * (tx * 64 + o) + par, a.W - 1) + c - kWinR;
        E.sd[k] = o * kDistStride + 3 * c;
    }
    short4* field = reinterpret_cast<short4*>(a.hyp) + (size_t)z * npx;
    float* cost = a.cost + (size_t)z * npx;
    const size_t o = (size_t)i * a.W + jj;
    short4 best = field[o];
    float bestc = cost[o];
    const short4 own = best;
    const int ni[4] = {i, i - 1, i, i + 1};
    const int nj[4] = {jj - 1, jj, jj + 1, jj};
    short4 nh[4];
    bool in[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        in[q] = act && ni[q] >= 0 && ni[q] < a.H && nj[q] >= 0 && nj[q] < a.W;
        nh[q] = in[q] ? field[(size_t)ni[q] * a.W + nj[q]] : own;
    }
    auto eq = [](short4 p, short4 q) { return p.x == q.x && p.y == q.y && p.z == q.z && p.w == q.w; };
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        bool dup = eq(nh[q], own);
#pragma unroll
        for (int p = 0; p < q; ++p) dup = dup || (in[p] && eq(nh[q], nh[p]));
        const bool want = in[q] && !dup;
        if (!__any(want)) continue;
        const float c = E.cost_below(want, nh[q], bestc);
        if (want && c < bestc) {
            bestc = c;
            best = nh[q];
        }
    }
    const short4 centre = best;
    const uint64_t seed = a.seeds[b];
    for (int t = 0; t < a.rs_samples; ++t) {
        const int r = max(1, a.rs_r0 >> t);
        U4 ctr;
        ctr.x = (uint32_t)(i * a.W + jj);
        ctr.y = (uint32_t)it;
        ctr.z = (kSiftLevelTag << 16) | ((uint32_t)t << 8) | (s < 0 ? 1u : 0u);
        ctr.w = 0u;
        const U4 rnd = philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32));
        short4 c;
        c.x = (short)clampi(centre.x + uniform_offset(rnd.x, r), -a.fmax, a.fmax);
        c.y = (short)clampi(centre.y + uniform_offset(rnd.y, r), -a.fmax, a.fmax);
        c.z = (short)clampi(centre.z + uniform_offset(rnd.z, r), 0, a.dmax);
        c.w = (short)clampi(centre.w + uniform_offset(rnd.w, r), 0, a.dmax);
        const bool want = act && !eq(c, centre);
        if (!__any(want)) continue;
        const float cc = E.cost_below(want, c, bestc);
        if (want && cc < bestc) {
            bestc = cc;
            best = c;
        }
    }
    if (act) {
        field[o] = best;
        cost[o] = bestc;
    }
}

// Eq. (1) at fixed vectors with the wave-shared gathers: 64 consecutive
// pixels of one row per wave (block), every field z of hyp/cost ([ndir][batch]
// or [batch]) in one launch; the same values as sift_cost_below.
__global__ void __launch_bounds__(64) sift_cost_coop_kernel(SiftMatchArgs a, int tiles_x) {
    __shared__ float dist_lds[64 * kDistStride];
    const int per_field = tiles_x * a.H;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);  // column-major tiles, a strip per XCD
    const int z = tile / per_field;
    const int tr = tile - z * per_field;
    const int tx = tr / a.H, i = tr - tx * a.H;
    const int lane = threadIdx.x;
    const int j = tx * 64 + lane;
    const bool act = j < a.W;
    const int jj = min(j, a.W - 1);
    const int di = z / a.batch, b = z - di * a.batch;
    const int s = a.ndir == 2 ? (di == 0 ? 1 : -1) : a.dir0;
    const size_t npx = (size_t)a.H * a.W;
    SiftCoop E;
    E.V = sift_views(a.phi + (size_t)b * 4 * npx, a.H, a.W, s);
    E.dist = dist_lds;
    E.lane = lane;
    E.y = i;
#pragma unroll
    for (int k = 0; k < kSiftSlots; ++k) {
        const int f = 64 * k + lane, o = f / kSiftSlots, c = f - kSiftSlots * o;
        E.so[k] = o;
        E.sx[k] = min(tx * 64 + o, a.W - 1) + c - kWinR;
        E.sd[k] = o * kDistStride + 3 * c;
    }
    const size_t o = (size_t)z * npx + (size_t)i * a.W + jj;
    const short4 h = reinterpret_cast<const short4*>(a.hyp)[o];
    const float c = E.cost_below(act, h, INFINITY);
    if (act) a.cost[o] = c;
}

// The cost's square root (sqrtf) over an array, to check its rounding.
__global__ void __launch_bounds__(256) sift_sqrt_kernel(const float* __restrict__ in, float* __restrict__ out,
                                                        int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = sqrtf(in[i]);
}

bool sift_shape_ok(const sff_params* p, int64_t nimg) {
    if (!params_ok(p) || nimg < 1) return false;
    // flattened indices stay below 2^31 in every kernel
    return nimg * (int64_t)(p->H + kExt) * (p->W + kExt) * kBins < (int64_t(1) << 31);
}

void launch_planes(const SiftGeom& g, int nimg, int C, const uint8_t* img, float* O, float* Cs,
                   hipStream_t st) {
    hipLaunchKernelGGL(orient_kernel, dim3((unsigned)((g.npx + 255) / 256), nimg), dim3(256), 0, st, img, O,
                       g.H, g.W, C);
    hipLaunchKernelGGL(cellsum_kernel, dim3((unsigned)((g.plane_c + 255) / 256), nimg), dim3(256), 0, st, O,
                       Cs, g.H, g.W);
}

}  // namespace
}  // namespace sff

using namespace sff;

extern "C" size_t sff_sift_workspace_bytes(const sff_params* p, int32_t nimg) {
    if (!sift_shape_ok(p, nimg)) return 0;
    return sift_ws(sift_geom(*p), nimg).total;
}

extern "C" sff_status sff_dense_sift(const sff_params* p, int32_t nimg, const uint8_t* img, float* sift,
                                     void* workspace, size_t workspace_bytes, void* stream) {
    if (!sift_shape_ok(p, nimg) || !img || !sift || (reinterpret_cast<uintptr_t>(sift) & 15) != 0)
        return SFF_ERR_INVALID_ARG;
    const SiftGeom g = sift_geom(*p);
    const SiftWs L = sift_ws(g, nimg);
    if (!workspace || workspace_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return SFF_ERR_WORKSPACE;
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    float* O = reinterpret_cast<float*>(ws + L.O);
    float* Cs = reinterpret_cast<float*>(ws + L.Cs);
    hipStream_t st = as_stream(stream);
    launch_planes(g, nimg, p->C, img, O, Cs, st);
    const long total = (long)nimg * g.npx;
    hipLaunchKernelGGL(sift_out_kernel, dim3((unsigned)((total + kGramPx - 1) / kGramPx)), dim3(256), 0, st,
                       Cs, sift, g.H, g.W, nimg);
    return launch_status();
}

extern "C" sff_status sff_sift_pca(const sff_params* p, int32_t batch, const uint8_t* imgs, double* mean,
                                   double* cov, double* eigval, double* axes, float* phi, void* workspace,
                                   size_t workspace_bytes, void* stream) {
    if (batch < 1 || batch > 65535 || !sift_shape_ok(p, 4 * (int64_t)batch) || !imgs || !mean || !cov ||
        !eigval || !axes || !phi)
        return SFF_ERR_INVALID_ARG;
    if (((reinterpret_cast<uintptr_t>(mean) | reinterpret_cast<uintptr_t>(cov) |
          reinterpret_cast<uintptr_t>(eigval) | reinterpret_cast<uintptr_t>(axes)) & 7) != 0 ||
        (reinterpret_cast<uintptr_t>(phi) & 15) != 0)
        return SFF_ERR_INVALID_ARG;
    const SiftGeom g = sift_geom(*p);
    const int nimg = 4 * batch;
    const SiftWs L = sift_ws(g, nimg);
    if (!workspace || workspace_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return SFF_ERR_WORKSPACE;
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    float* O = reinterpret_cast<float*>(ws + L.O);
    float* Cs = reinterpret_cast<float*>(ws + L.Cs);
    double* part = reinterpret_cast<double*>(ws + L.part);
    float* ax32 = reinterpret_cast<float*>(ws + L.ax32);
    hipStream_t st = as_stream(stream);
    launch_planes(g, nimg, p->C, imgs, O, Cs, st);
    const int nblk = gram_blocks(g);
    GramArgs ga{Cs, part, g.H, g.W, nblk};
    hipLaunchKernelGGL(gram_kernel, dim3(nblk, batch), dim3(256), 0, st, ga);
    double* gsum = reinterpret_cast<double*>(ws + L.gsum);
    hipLaunchKernelGGL(gram_sum_kernel, dim3((kSumEntries + 255) / 256, batch), dim3(256), 0, st, part, nblk,
                       gsum);
    hipLaunchKernelGGL(gram_cov_kernel, dim3(kDesc, batch), dim3(kDesc), 0, st, gsum,
                       1.0 / (4.0 * (double)g.npx), mean, cov);
    double* sqm = reinterpret_cast<double*>(ws + L.sq);  // [batch][2][kDesc][kDesc]
    for (int i = 0; i < kSquare; ++i) {
        const double* src = i == 0 ? cov : sqm + (size_t)((i - 1) & 1) * kDesc * kDesc;
        const size_t src_stride = i == 0 ? (size_t)kDesc * kDesc : (size_t)2 * kDesc * kDesc;
        hipLaunchKernelGGL(square_kernel, dim3(64, batch), dim3(256), 0, st, src, src_stride,
                           sqm + (size_t)(i & 1) * kDesc * kDesc, (size_t)2 * kDesc * kDesc);
    }
    hipLaunchKernelGGL(eig_kernel, dim3(batch), dim3(256), 0, st, cov, mean, sqm, eigval, axes, ax32);
    const long total = 4L * (long)g.npx;
    hipLaunchKernelGGL(project_kernel, dim3((unsigned)((total + kGramPx - 1) / kGramPx), batch), dim3(256), 0,
                       st, Cs, ax32, reinterpret_cast<float4*>(phi), g.H, g.W);
    return launch_status();
}

extern "C" sff_status sff_cost_sift(const sff_params* p, int32_t batch, int32_t dir, const float* phi,
                                    const int16_t* hyp, float* cost, void* stream) {
    if (!params_ok(p) || batch < 1 || batch > 65535 || (dir != SFF_DIR_FORWARD && dir != SFF_DIR_INVERSE) ||
        !phi || !hyp || !cost || (int64_t)batch * 4 * p->H * p->W >= (int64_t(1) << 31))
        return SFF_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(phi) & 15) != 0 || (reinterpret_cast<uintptr_t>(hyp) & 7) != 0 ||
        (reinterpret_cast<uintptr_t>(cost) & 3) != 0)
        return SFF_ERR_INVALID_ARG;
    const char* e = std::getenv("SFF_SIFT_EVAL");
    if (e && std::strcmp(e, "lane") == 0) {
        hipLaunchKernelGGL(cost_sift_kernel, dim3((p->W + kCT - 1) / kCT, (p->H + kCT - 1) / kCT, batch),
                           dim3(256), 0, as_stream(stream), reinterpret_cast<const float4*>(phi), hyp, cost,
                           p->H, p->W, dir == SFF_DIR_FORWARD ? 1 : -1);
        return launch_status();
    }
    SiftMatchArgs a{};
    a.phi = reinterpret_cast<const float4*>(phi);
    a.hyp = const_cast<int16_t*>(hyp);  // read only by this kernel
    a.cost = cost;
    a.H = p->H;
    a.W = p->W;
    a.batch = batch;
    a.ndir = 1;
    a.dir0 = dir == SFF_DIR_FORWARD ? 1 : -1;
    const int tiles_x = (p->W + 63) / 64;
    hipLaunchKernelGGL(sift_cost_coop_kernel, dim3(tiles_x * p->H * batch), dim3(64), 0, as_stream(stream), a,
                       tiles_x);
    return launch_status();
}

extern "C" sff_status sff_match_sift(const sff_params* p, int32_t batch, int32_t dir, const float* phi,
                                     const uint64_t* seeds, int32_t iters, int16_t* hyp, float* cost,
                                     void* stream) {
    if (!params_ok(p) || batch < 1 || batch > 32767 || (dir != SFF_DIR_FORWARD && dir != SFF_DIR_INVERSE &&
                                                         dir != SFF_DIR_BOTH) ||
        !phi || !seeds || !hyp || !cost || iters < 0 || iters > 64 ||
        (int64_t)batch * 4 * p->H * p->W >= (int64_t(1) << 31))
        return SFF_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(phi) & 15) != 0 || (reinterpret_cast<uintptr_t>(hyp) & 7) != 0 ||
        (reinterpret_cast<uintptr_t>(cost) & 3) != 0 || (reinterpret_cast<uintptr_t>(seeds) & 7) != 0)
        return SFF_ERR_INVALID_ARG;
    SiftMatchArgs a;
    a.phi = reinterpret_cast<const float4*>(phi);
    a.seeds = seeds;
    a.hyp = hyp;
    a.cost = cost;
    a.H = p->H;
    a.W = p->W;
    a.rs_r0 = p->rs_r0;
    a.rs_samples = p->rs_samples;
    a.fmax = p->fmax;
    a.dmax = p->dmax;
    a.batch = batch;
    a.ndir = dir == SFF_DIR_BOTH ? 2 : 1;
    a.dir0 = dir == SFF_DIR_BOTH ? 1 : dir;
    const int nz = a.ndir * batch;
    hipStream_t st = as_stream(stream);
    const size_t npx = (size_t)p->H * p->W;
    // SFF_SIFT_EVAL=lane forces the per-lane kernels (same results; testing and timing)
    const char* e = std::getenv("SFF_SIFT_EVAL");
    const bool lane = e && std::strcmp(e, "lane") == 0;
    if (lane)
        hipLaunchKernelGGL(sift_cost_init_kernel, dim3((unsigned)((npx + 255) / 256), nz), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(sift_cost_coop_kernel, dim3(((p->W + 63) / 64) * p->H * nz), dim3(64), 0, st, a,
                           (p->W + 63) / 64);
    const int tiles_x = ((p->W + 1) / 2 + 63) / 64, tiles_y = (p->H + 3) / 4;
    for (int it = 0; it < iters; ++it)
        for (int colour = 0; colour < 2; ++colour) {
            if (lane)
                hipLaunchKernelGGL(sift_half_step_kernel, dim3(tiles_x * tiles_y * nz), dim3(256), 0, st, a,
                                   it, colour, tiles_x, tiles_y);
            else
                hipLaunchKernelGGL(sift_half_step_coop_kernel, dim3(tiles_x * p->H * nz), dim3(64), 0, st, a,
                                   it, colour, tiles_x);
        }
    return launch_status();
}

extern "C" sff_status sff_sift_sqrt(const float* in, float* out, int64_t n, void* stream) {
    if (!in || !out || n < 0 || n > (int64_t(1) << 31)) return SFF_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(in) & 3) != 0 || (reinterpret_cast<uintptr_t>(out) & 3) != 0)
        return SFF_ERR_INVALID_ARG;
    if (n == 0) return SFF_OK;
    hipLaunchKernelGGL(sift_sqrt_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, as_stream(stream), in,
                       out, n);
    return launch_status();
}
