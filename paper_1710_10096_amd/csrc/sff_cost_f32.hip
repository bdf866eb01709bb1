// Window form of the matching cost on real-valued feature maps and its
// gradient (SceneFlowFields, Section 3.1, eq. (1): feature distances summed
// over a window around the pixel for the temporal, stereo and cross
// correspondences; replicated borders).
//
//   cost(p) = sum_corr sum_{w in {-3..4}^2} sum_c
//             (F_R(clamp(p + w), c) - F_corr(clamp(t_corr(p) + w), c))^2,
//   t_corr(p) = clamp(p + o_corr(h_p)),  o_T = (u, v), o_S = (-s d0, 0),
//   o_X = (u - s d1, v).
//
// Backward for L = sum_p g_p cost(p): each term with difference delta adds
// 2 g_p delta to the reference entry and subtracts it from the target entry.
//   * reference map: a gather over the preimage {(p, w) : clamp(p + w) = q};
//   * target maps: pixels are grouped by their (clamped) target centre with a
//     stable radix sort (hand-written, 8-bit digits), then every target entry
//     gathers over the centres whose window covers it.
// Both are deterministic (no floating-point atomics).
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "sff_internal.hpp"

namespace sff {
namespace {

constexpr int kWin0 = -3, kWin1 = 4;  // window offsets, the descriptors' 8x8 patch

struct CostArgs {
    const float* feat;      // [batch][4][H][W][CF]
    const int16_t* hyp;     // [batch][H][W][4]
    const float* gcost;     // [batch][H][W] (backward)
    float* out;             // cost [batch][H][W] or gradient [batch][4][H][W][CF]
    int H, W, s, batch;
};

template <int CF>
__device__ __forceinline__ void load_vec(const float* __restrict__ f, float* v) {
    const float4* p = reinterpret_cast<const float4*>(f);
#pragma unroll
    for (int k = 0; k < CF / 4; ++k) {
        const float4 x = p[k];
        v[4 * k] = x.x;
        v[4 * k + 1] = x.y;
        v[4 * k + 2] = x.z;
        v[4 * k + 3] = x.w;
    }
}

__device__ __forceinline__ int view(int s, int role) {  // canonical map of R, T, S, X
    return s > 0 ? role : 3 - role;
}

struct Targets {
    int y[3], x[3];
};

__device__ __forceinline__ Targets targets(const int16_t* hyp, size_t pix, int y, int x, int s,
                                           int H, int W) {
    const uint2 h = reinterpret_cast<const uint2*>(hyp)[pix];
    const int u = (int16_t)(h.x & 0xFFFFu), v = (int16_t)(h.x >> 16);
    const int d0 = (int16_t)(h.y & 0xFFFFu), d1 = (int16_t)(h.y >> 16);
    Targets t;
    t.y[0] = clampi(y + v, 0, H - 1);
    t.x[0] = clampi(x + u, 0, W - 1);
    t.y[1] = y;
    t.x[1] = clampi(x - s * d0, 0, W - 1);
    t.y[2] = t.y[0];
    t.x[2] = clampi(x + u - s * d1, 0, W - 1);
    return t;
}

// One thread per pixel; block = 64 pixels of 4 rows.  Partial sums per window
// position, then per window row, keep the FP32 rounding error near 10^-5.
template <int CF>
__global__ void __launch_bounds__(256) cost_fwd_kernel(CostArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int b = blockIdx.z;
    if (x >= a.W || y >= a.H) return;
    const int H = a.H, W = a.W;
    const size_t HW = (size_t)H * W;
    const float* base = a.feat + (size_t)b * 4 * HW * CF;
    const float* R = base + (size_t)view(a.s, 0) * HW * CF;
    const float* M[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) M[k] = base + (size_t)view(a.s, k + 1) * HW * CF;
    const Targets t = targets(a.hyp, (size_t)b * HW + (size_t)y * W + x, y, x, a.s, H, W);
    float total = 0.f;
    for (int dy = kWin0; dy <= kWin1; ++dy) {
        const int ry = clampi(y + dy, 0, H - 1);
        int ty[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) ty[k] = clampi(t.y[k] + dy, 0, H - 1);
        float rsum = 0.f;
        for (int dx = kWin0; dx <= kWin1; ++dx) {
            float ref[CF];
            load_vec<CF>(R + ((size_t)ry * W + clampi(x + dx, 0, W - 1)) * CF, ref);
            float psum = 0.f;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                float tg[CF];
                load_vec<CF>(M[k] + ((size_t)ty[k] * W + clampi(t.x[k] + dx, 0, W - 1)) * CF, tg);
#pragma unroll
                for (int c = 0; c < CF; ++c) {
                    const float d = ref[c] - tg[c];
                    psum = fmaf(d, d, psum);
                }
            }
            rsum += psum;
        }
        total += rsum;
    }
    a.out[(size_t)b * HW + (size_t)y * W + x] = total;
}

// The same cost with CF / 4 lanes per pixel, four channels each: a gathered
// vector is CF / 4 neighbouring 16-byte loads.  Each lane sums its channels
// in the nested order above; the CF / 4 lane sums are combined by an xor
// butterfly (every lane ends with the same value), so the result is
// deterministic; it rounds differently from cost_fwd_kernel (within the same
// error bound).
template <int CF>
__global__ void __launch_bounds__(256) cost_fwd_coop_kernel(CostArgs a) {
    constexpr int L = CF / 4, QPB = 256 / L;
    const int sub = threadIdx.x % L;
    const int H = a.H, W = a.W, b = blockIdx.y;
    const size_t HW = (size_t)H * W;
    const size_t q = (size_t)xcd_tile(blockIdx.x, gridDim.x) * QPB + threadIdx.x / L;  // a band of rows per XCD
    if (q >= HW) return;  // all L lanes of the pixel together
    const int y = (int)(q / W), x = (int)(q - (size_t)y * W);
    const float* base = a.feat + (size_t)b * 4 * HW * CF;
    const float4* R = reinterpret_cast<const float4*>(base + (size_t)view(a.s, 0) * HW * CF) + sub;
    const float4* M[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) M[k] = reinterpret_cast<const float4*>(base + (size_t)view(a.s, k + 1) * HW * CF) + sub;
    const Targets t = targets(a.hyp, (size_t)b * HW + q, y, x, a.s, H, W);
    float total = 0.f;
    for (int dy = kWin0; dy <= kWin1; ++dy) {
        const int ry = clampi(y + dy, 0, H - 1);
        int ty[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) ty[k] = clampi(t.y[k] + dy, 0, H - 1);
        float rsum = 0.f;
        for (int dx = kWin0; dx <= kWin1; ++dx) {
            const float4 r = R[((size_t)ry * W + clampi(x + dx, 0, W - 1)) * L];
            float psum = 0.f;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float4 tg = M[k][((size_t)ty[k] * W + clampi(t.x[k] + dx, 0, W - 1)) * L];
                const float d0 = r.x - tg.x, d1 = r.y - tg.y, d2 = r.z - tg.z, d3 = r.w - tg.w;
                psum = fmaf(d0, d0, psum);
                psum = fmaf(d1, d1, psum);
                psum = fmaf(d2, d2, psum);
                psum = fmaf(d3, d3, psum);
            }
            rsum += psum;
        }
        total += rsum;
    }
#pragma unroll
    for (int off = L / 2; off >= 1; off >>= 1) total += __shfl_xor(total, off, L);
    if (sub == 0) a.out[(size_t)b * HW + q] = total;
}

// Preimage of the clamped coordinate: {p in [0, n) : clamp(p + w, 0, n - 1) = q}.
__device__ __forceinline__ void preimage(int q, int w, int n, int& lo, int& hi) {
    if (n == 1) {
        lo = hi = 0;
        return;
    }
    if (q == 0) {
        lo = 0;
        hi = min(-w, n - 1);
    } else if (q == n - 1) {
        lo = max(n - 1 - w, 0);
        hi = n - 1;
    } else {
        lo = hi = q - w;
        if (lo < 0 || lo > n - 1) hi = lo - 1;  // empty
    }
}

// The gradient entries gather their terms in row_split(CF) parts of
// consecutive window rows, summed alone and then added in part order: eight
// single rows up to 32 channels, four pairs of rows at 64 (the CF / 4 lanes of
// every part of an entry share one wave).
constexpr int row_split(int cf) { return cf <= 32 ? 8 : 4; }
constexpr int kWinN = kWin1 - kWin0 + 1;  // 8 window rows and columns

// Reference-map gradient, one thread per entry q of R (testing and timing).
// The terms of q are the (p, w) with clamp(p + w) = q, taken by window row wy,
// preimage row py, window column wx, preimage column px and correspondence;
// each part of the window rows is summed alone, then the parts in order.
template <int CF>
__global__ void __launch_bounds__(256) grad_ref_kernel(CostArgs a) {
    const int qx = blockIdx.x * 64 + (threadIdx.x & 63);
    const int qy = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int b = blockIdx.z;
    if (qx >= a.W || qy >= a.H) return;
    const int H = a.H, W = a.W;
    const size_t HW = (size_t)H * W;
    const float* base = a.feat + (size_t)b * 4 * HW * CF;
    const int mR = view(a.s, 0);
    const float* M[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) M[k] = base + (size_t)view(a.s, k + 1) * HW * CF;
    float fq[CF], acc[CF], sum[CF];
    load_vec<CF>(base + ((size_t)mR * HW + (size_t)qy * W + qx) * CF, fq);
    constexpr int kSplit = row_split(CF), kPartRows = kWinN / kSplit;
    for (int part = 0; part < kSplit; ++part) {
#pragma unroll
        for (int c = 0; c < CF; ++c) acc[c] = 0.f;
        for (int wy = kWin0 + part * kPartRows; wy < kWin0 + (part + 1) * kPartRows; ++wy) {
            int ylo, yhi;
            preimage(qy, wy, H, ylo, yhi);
            for (int py = ylo; py <= yhi; ++py)
                for (int wx = kWin0; wx <= kWin1; ++wx) {
                    int xlo, xhi;
                    preimage(qx, wx, W, xlo, xhi);
                    for (int px = xlo; px <= xhi; ++px) {
                        const size_t pix = (size_t)b * HW + (size_t)py * W + px;
                        const float g2 = 2.f * a.gcost[pix];
                        const Targets t = targets(a.hyp, pix, py, px, a.s, H, W);
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            float tg[CF];
                            load_vec<CF>(M[k] + ((size_t)clampi(t.y[k] + wy, 0, H - 1) * W +
                                                 clampi(t.x[k] + wx, 0, W - 1)) * CF, tg);
#pragma unroll
                            for (int c = 0; c < CF; ++c) acc[c] = fmaf(g2, fq[c] - tg[c], acc[c]);
                        }
                    }
                }
        }
#pragma unroll
        for (int c = 0; c < CF; ++c) sum[c] = part ? sum[c] + acc[c] : acc[c];
    }
    float4* o = reinterpret_cast<float4*>(a.out + ((size_t)b * 4 * HW + (size_t)mR * HW +
                                                   (size_t)qy * W + qx) * CF);
#pragma unroll
    for (int k = 0; k < CF / 4; ++k) o[k] = make_float4(sum[4 * k], sum[4 * k + 1], sum[4 * k + 2], sum[4 * k + 3]);
}

// Grouping of the pixels by target centre, all three correspondences in one
// list: element k * n + i (pixel i of the batch, n pixels) has the key
// k * n + (centre cell of correspondence k) and the value i.  After a stable
// sort by key, the pixels of each centre cell are in ascending pixel order.
__global__ void target_keys_kernel(const int16_t* __restrict__ hyp, uint32_t* __restrict__ keys,
                                   uint32_t* __restrict__ vals, int H, int W, int s, uint32_t n) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= 3 * (size_t)n) return;
    const uint32_t k = (uint32_t)(e / n), i = (uint32_t)(e - (size_t)k * n);
    const size_t HW = (size_t)H * W;
    const int b = (int)(i / HW);
    const int pix = (int)(i - (size_t)b * HW);
    const int y = pix / W, x = pix - y * W;
    const Targets t = targets(hyp, i, y, x, s, H, W);
    keys[e] = k * n + (uint32_t)((size_t)b * HW + (size_t)t.y[k] * W + t.x[k]);
    vals[e] = i;
}

// Least-significant-digit radix sort of (key, value) pairs, 8-bit digits, one
// pass = histogram per block, exclusive scan over (digit, block), stable
// scatter.  Blocks of 256 threads take 16 rounds of 256 consecutive elements.
constexpr int kSortTile = 4096;

__global__ void __launch_bounds__(256) sort_hist_kernel(const uint32_t* __restrict__ keys, size_t N,
                                                        int sh, uint32_t* __restrict__ hist,
                                                        uint32_t nblk) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * kSortTile;
    for (int j = 0; j < kSortTile / 256; ++j) {
        const size_t i = base + (size_t)j * 256 + threadIdx.x;
        if (i < N) atomicAdd(&h[(keys[i] >> sh) & 255u], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Exclusive prefix sum of v over the 1024 threads of the block; *total gets
// the sum.
__device__ uint32_t block_scan_1024(uint32_t v, uint32_t* total) {
    __shared__ uint32_t wsum[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(x, off);
        if (lane >= off) x += t;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (w == 0) {
        uint32_t y = lane < 16 ? wsum[lane] : 0u;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const uint32_t t = __shfl_up(y, off);
            if (lane >= off) y += t;
        }
        if (lane < 16) wsum[lane] = y;  // inclusive
    }
    __syncthreads();
    const uint32_t before = w ? wsum[w - 1] : 0u;
    *total = wsum[15];
    __syncthreads();  // wsum is reused by the next call
    return before + x - v;
}

// Exclusive scan of h[0 .. total) in two steps: each block of 1024 threads
// scans its chunk of 1024 entries in place and writes the chunk's sum; one
// block then scans the chunk sums (sort_scan_sums_kernel).  A scanned entry
// is h[i] + sums[i / 1024].
__global__ void __launch_bounds__(1024) sort_scan_chunks_kernel(uint32_t* __restrict__ h, size_t total,
                                                                uint32_t* __restrict__ sums) {
    const size_t i = (size_t)blockIdx.x * 1024 + threadIdx.x;
    const uint32_t v = i < total ? h[i] : 0u;
    uint32_t sum;
    const uint32_t ex = block_scan_1024(v, &sum);
    if (i < total) h[i] = ex;
    if (threadIdx.x == 0) sums[blockIdx.x] = sum;
}

__global__ void __launch_bounds__(1024) sort_scan_sums_kernel(uint32_t* __restrict__ sums, size_t nchunks) {
    uint32_t run = 0;
    for (size_t c = 0; c < nchunks; c += 1024) {
        const size_t i = c + threadIdx.x;
        const uint32_t v = i < nchunks ? sums[i] : 0u;
        uint32_t sum;
        const uint32_t ex = block_scan_1024(v, &sum);
        if (i < nchunks) sums[i] = run + ex;
        run += sum;
    }
}

// Stable scatter of one pass: element order is (round, wave, lane), the input
// order; the rank inside a wave comes from the lanes with the same digit.
__global__ void __launch_bounds__(256) sort_scatter_kernel(const uint32_t* __restrict__ kin,
                                                           const uint32_t* __restrict__ vin,
                                                           uint32_t* __restrict__ kout,
                                                           uint32_t* __restrict__ vout, size_t N,
                                                           int sh, const uint32_t* __restrict__ scan,
                                                           const uint32_t* __restrict__ sums,
                                                           uint32_t nblk) {
    __shared__ uint32_t off[256];
    __shared__ uint32_t wc[4][256];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const size_t hi = (size_t)t * nblk + blockIdx.x;
    off[t] = scan[hi] + sums[hi / 1024];
#pragma unroll
    for (int q = 0; q < 4; ++q) wc[q][t] = 0;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * kSortTile;
    const uint64_t below = (1ull << lane) - 1ull;
    for (int j = 0; j < kSortTile / 256; ++j) {
        const size_t i = base + (size_t)j * 256 + t;
        const bool ok = i < N;
        uint32_t key = 0, val = 0, d = 0;
        if (ok) {
            key = kin[i];
            val = vin[i];
            d = (key >> sh) & 255u;
        }
        uint64_t m = __ballot(ok);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (d >> bit) & 1u;
            const uint64_t bb = __ballot(on);
            m &= on ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(m & below);
        const uint32_t cnt = (uint32_t)__popcll(m);
        if (ok && rank == cnt - 1) wc[w][d] = cnt;  // the group's last lane
        __syncthreads();
        if (ok) {
            uint32_t pos = off[d] + rank;
            for (int q = 0; q < w; ++q) pos += wc[q][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        off[t] += wc[0][t] + wc[1][t] + wc[2][t] + wc[3][t];
#pragma unroll
        for (int q = 0; q < 4; ++q) wc[q][t] = 0;
        __syncthreads();
    }
}

// start[c] = first position of a sorted key >= c, for every cell c in [0, N]
// (binary search; any run of empty cells costs nothing extra).
__global__ void cell_starts_kernel(const uint32_t* __restrict__ keys, uint32_t* __restrict__ start,
                                   size_t N) {
    const size_t c = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (c > N) return;
    size_t lo = 0, hi = N;
    while (lo < hi) {
        const size_t mid = lo + (hi - lo) / 2;
        if ((size_t)keys[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    start[c] = (uint32_t)lo;
}

// Gradient of target map k, one thread per entry q of that map (testing and
// timing).  The terms of q are the (pixel, w) with clamp(centre + w) = q, in
// the canonical order: window row wy ascending, cell row ty of its preimage
// ascending, window column wx descending (cells by ascending x), cell column
// tx of its preimage ascending, the pixels grouped at the cell in sorted
// order.  Term i goes to accumulator i mod row_split(CF); the gradient is the
// sum of the accumulators in order.  (Dealing the terms round-robin keeps the
// tiled kernel's lanes busy however unevenly the pixels crowd the cells.)
template <int CF>
__global__ void __launch_bounds__(256) grad_target_kernel(CostArgs a, int k, size_t n,
                                                          const uint32_t* __restrict__ start,
                                                          const uint32_t* __restrict__ order) {
    const int qx = blockIdx.x * 64 + (threadIdx.x & 63);
    const int qy = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int b = blockIdx.z;
    if (qx >= a.W || qy >= a.H) return;
    const int H = a.H, W = a.W;
    const size_t HW = (size_t)H * W;
    const float* base = a.feat + (size_t)b * 4 * HW * CF;
    const float* R = base + (size_t)view(a.s, 0) * HW * CF;
    const int mk = view(a.s, k + 1);
    constexpr int S = row_split(CF);
    float fq[CF], acc[S][CF];
    load_vec<CF>(base + ((size_t)mk * HW + (size_t)qy * W + qx) * CF, fq);
#pragma unroll
    for (int t = 0; t < S; ++t)
#pragma unroll
        for (int c = 0; c < CF; ++c) acc[t][c] = 0.f;
    uint32_t i = 0;
    for (int wy = kWin0; wy <= kWin1; ++wy) {
        int ylo, yhi;
        preimage(qy, wy, H, ylo, yhi);
        for (int ty = ylo; ty <= yhi; ++ty)
            for (int wx = kWin1; wx >= kWin0; --wx) {
                int xlo, xhi;
                preimage(qx, wx, W, xlo, xhi);
                for (int tx = xlo; tx <= xhi; ++tx) {
                    const size_t cell = (size_t)k * n + (size_t)b * HW + (size_t)ty * W + tx;
                    const uint32_t e0 = start[cell], e1 = start[cell + 1];
                    for (uint32_t e = e0; e < e1; ++e, ++i) {
                        const uint32_t pix = order[e];
                        const int pl = (int)(pix - (size_t)b * HW);
                        const int py = pl / W, px = pl - py * W;
                        const float g2 = 2.f * a.gcost[pix];
                        float r[CF];
                        load_vec<CF>(R + ((size_t)clampi(py + wy, 0, H - 1) * W +
                                          clampi(px + wx, 0, W - 1)) * CF, r);
                        float* ac = acc[i % S];
#pragma unroll
                        for (int c = 0; c < CF; ++c) ac[c] = fmaf(-g2, r[c] - fq[c], ac[c]);
                    }
                }
            }
    }
    float4* o = reinterpret_cast<float4*>(a.out + ((size_t)b * 4 * HW + (size_t)mk * HW +
                                                   (size_t)qy * W + qx) * CF);
#pragma unroll
    for (int kk = 0; kk < CF / 4; ++kk) {
        float4 v = make_float4(acc[0][4 * kk], acc[0][4 * kk + 1], acc[0][4 * kk + 2], acc[0][4 * kk + 3]);
#pragma unroll
        for (int t = 1; t < S; ++t)
            v = make_float4(v.x + acc[t][4 * kk], v.y + acc[t][4 * kk + 1], v.z + acc[t][4 * kk + 2],
                            v.w + acc[t][4 * kk + 3]);
        o[kk] = v;
    }
}

// Tiled gradient kernels: a block takes kTileQ consecutive entries of one row
// of one map and first stages in LDS what all of them read besides the
// gathered feature vectors; then CF / 4 lanes (four channels each) per part
// of the window rows and row_split(CF) parts per entry gather the vectors and
// add the same terms in the same order as the one-thread kernels (each part
// alone, then the parts in order by a shuffle), so the results are identical.
// Tiles are numbered ((map * batch + b) * H + row) * tiles_x + column tile and
// given out by XCD, so an XCD's L2 holds a band of rows.
constexpr int kTileQ = 32;
constexpr int kTileC = kTileQ + kWinN - 1;  // staged columns: the tile's and the window's
constexpr int kStageCap = 2048;             // staged pixels per target-gradient tile

// Add the four-channel part of the terms of one pixel: fma(g, x - y, acc).
__device__ __forceinline__ void fma4(float g, const float4& x, const float4& y, float4& acc) {
    acc.x = fmaf(g, x.x - y.x, acc.x);
    acc.y = fmaf(g, x.y - y.y, acc.y);
    acc.z = fmaf(g, x.z - y.z, acc.z);
    acc.w = fmaf(g, x.w - y.w, acc.w);
}

// One image's feature map read 16 bytes per lane.  BUF: a raw buffer with
// 32-bit offsets (maps below 2 GiB), where a load flagged `skip` reads nothing
// (its value is filled in by the caller); otherwise plain loads, `skip`
// ignored.
constexpr int kSkipOff = 0x7FFFFFF0;
template <bool BUF>
struct Vec4Map {
    const float4* p;
    __amdgpu_buffer_rsrc_t rs;
    __device__ __forceinline__ void init(const float* base, size_t bytes) {
        p = reinterpret_cast<const float4*>(base);
        if constexpr (BUF) {
            const uint64_t a = reinterpret_cast<uint64_t>(base);
            const uint64_t u = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)a) |
                               ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(a >> 32)) << 32);
            rs = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(u), (short)0,
                                                   (int)__builtin_amdgcn_readfirstlane((uint32_t)bytes),
                                                   0x00020000);
        }
    }
    __device__ __forceinline__ float4 ld(uint32_t i, bool skip) const {
        if constexpr (BUF) {
            const uint4 v = __builtin_bit_cast(
                uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, skip ? kSkipOff : (int)(i * 16u), 0, 0));
            return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z),
                               __uint_as_float(v.w));
        } else {
            return p[i];
        }
    }
};

// Sum of the entry's parts, in part order, in the lanes of part 0.
template <int kSplit, int L>
__device__ __forceinline__ float4 sum_parts(const float4& acc) {
    float4 sum = acc;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int g = 1; g < kSplit; ++g) {
        const int src = lane + g * L;  // part g of this entry, for the lanes of part 0
        sum.x += __shfl(acc.x, src);
        sum.y += __shfl(acc.y, src);
        sum.z += __shfl(acc.z, src);
        sum.w += __shfl(acc.w, src);
    }
    return sum;
}

// Reference-map gradient: the tile stages 2 g and the three target centres of
// the pixels its entries' windows reach (8 rows by kTileC columns).
template <int CF, bool BUF>
__global__ void __launch_bounds__(256) grad_ref_tile_kernel(CostArgs a, int tiles_x) {
    constexpr int kSplit = row_split(CF), kPartRows = kWinN / kSplit;
    constexpr int L = CF / 4, G = kSplit * L, EPB = 256 / G;
    static_assert(G <= 64 && 64 % G == 0, "the parts of an entry share one wave");
    __shared__ float s_g[kWinN][kTileC];
    __shared__ uint32_t s_t[3][kWinN][kTileC];  // (ty << 16) | tx
    __shared__ float4 s_fq[kTileQ * L];         // the entries' own vectors
    const int H = a.H, W = a.W;
    const size_t HW = (size_t)H * W;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tq = tile % tiles_x, rest = tile / tiles_x;
    const int qy = rest % H, b = rest / H;
    const int qx0 = tq * kTileQ;
    const int py0 = qy - kWin1, px0 = qx0 - kWin1;  // staged pixel (0, 0)
    for (int idx = threadIdx.x; idx < kWinN * kTileC; idx += 256) {
        const int r = idx / kTileC, c = idx - r * kTileC;
        const int py = py0 + r, px = px0 + c;
        if (py < 0 || py >= H || px < 0 || px >= W) continue;
        const size_t pix = (size_t)b * HW + (size_t)py * W + px;
        s_g[r][c] = 2.f * a.gcost[pix];
        const Targets t = targets(a.hyp, pix, py, px, a.s, H, W);
#pragma unroll
        for (int k = 0; k < 3; ++k) s_t[k][r][c] = ((uint32_t)t.y[k] << 16) | (uint32_t)t.x[k];
    }
    const float* base = a.feat + (size_t)b * 4 * HW * CF;
    const int mR = view(a.s, 0);
    for (int idx = threadIdx.x; idx < kTileQ * L; idx += 256) {
        const int qx = qx0 + idx / L;
        if (qx < W)
            s_fq[idx] = reinterpret_cast<const float4*>(base + ((size_t)mR * HW + (size_t)qy * W + qx) * CF)[idx % L];
    }
    __syncthreads();
    Vec4Map<BUF> M[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) M[k].init(base + (size_t)view(a.s, k + 1) * HW * CF, HW * CF * 4);
    const int sub = threadIdx.x % L, part = (threadIdx.x / L) % kSplit;
    const int wy0 = kWin0 + part * kPartRows;
    for (int e0 = 0; e0 < kTileQ; e0 += EPB) {
        const int qx = qx0 + e0 + (int)threadIdx.x / G;
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        const bool live = qx < W && qx < qx0 + kTileQ;
        const size_t q = (size_t)qy * W + qx;
        float4 fq = make_float4(0.f, 0.f, 0.f, 0.f);
        if (live) fq = s_fq[(qx - qx0) * L + sub];
        if (live && qy >= kWin1 && qy <= H - 1 + kWin0 && qx >= kWin1 && qx <= W - 1 + kWin0) {
            // interior: the preimage of q under w is the one pixel q - w.  A
            // gathered vector equal to the previous one of the same map (a
            // locally constant field reads one vector for the whole row) is not
            // loaded again but copied once all loads are back; the arithmetic
            // is unchanged.
            // (half a window row, 12 gathers, at a time: fewer registers, more waves)
            constexpr int JH = kWinN / 2;
            int pidx[3] = {-1, -1, -1};
            float4 pv[3];
            for (int wy = wy0; wy < wy0 + kPartRows; ++wy) {
                const int r = qy - wy - py0;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    float4 tg[JH][3];
                    float g2[JH];
                    int idx[JH][3];
#pragma unroll
                    for (int jj = 0; jj < JH; ++jj) {  // wx = kWin0 + j
                        const int j = h * JH + jj, wx = kWin0 + j, c = qx - wx - px0;
                        g2[jj] = s_g[r][c];
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            const uint32_t t = s_t[k][r][c];
                            idx[jj][k] = clampi((int)(t >> 16) + wy, 0, H - 1) * W +
                                         clampi((int)(t & 0xFFFFu) + wx, 0, W - 1);
                        }
                    }
#pragma unroll
                    for (int jj = 0; jj < JH; ++jj)
#pragma unroll
                        for (int k = 0; k < 3; ++k)
                            tg[jj][k] = M[k].ld((uint32_t)idx[jj][k] * L + sub,
                                                idx[jj][k] == (jj ? idx[jj - 1][k] : pidx[k]));
                    if constexpr (BUF) {
#pragma unroll
                        for (int jj = 0; jj < JH; ++jj)
#pragma unroll
                            for (int k = 0; k < 3; ++k)
                                if (idx[jj][k] == (jj ? idx[jj - 1][k] : pidx[k])) tg[jj][k] = jj ? tg[jj - 1][k] : pv[k];
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            pidx[k] = idx[JH - 1][k];
                            pv[k] = tg[JH - 1][k];
                        }
                    }
#pragma unroll
                    for (int jj = 0; jj < JH; ++jj)
#pragma unroll
                        for (int k = 0; k < 3; ++k) fma4(g2[jj], fq, tg[jj][k], acc);
                }
            }
        } else if (live) {
            for (int wy = wy0; wy < wy0 + kPartRows; ++wy) {
                int ylo, yhi;
                preimage(qy, wy, H, ylo, yhi);
                for (int py = ylo; py <= yhi; ++py)
                    for (int wx = kWin0; wx <= kWin1; ++wx) {
                        int xlo, xhi;
                        preimage(qx, wx, W, xlo, xhi);
                        for (int px = xlo; px <= xhi; ++px) {
                            const int r = py - py0, c = px - px0;
                            const float g2 = s_g[r][c];
#pragma unroll
                            for (int k = 0; k < 3; ++k) {
                                const uint32_t t = s_t[k][r][c];
                                const int ty = (int)(t >> 16), tx = (int)(t & 0xFFFFu);
                                const float4 tg = M[k].ld((uint32_t)(clampi(ty + wy, 0, H - 1) * W + clampi(tx + wx, 0, W - 1)) * L + sub, false);
                                fma4(g2, fq, tg, acc);
                            }
                        }
                    }
            }
        }
        const float4 sum = sum_parts<kSplit, L>(acc);
        if (live && part == 0)
            reinterpret_cast<float4*>(a.out + ((size_t)b * 4 * HW + (size_t)mR * HW + q) * CF)[sub] = sum;
    }
}

// Target-map gradients (all three maps in one launch): the tile stages the
// pixels grouped at the centre cells its entries' windows reach (8 rows of
// kTileC cells; position, 2 g and cell column of each, and the run bounds of
// every cell).  A tile whose cells hold more than kStageCap pixels reads them
// from the sorted lists in global memory instead, in the same order.  The
// row_split(CF) groups of CF / 4 lanes of an entry are its accumulators (terms
// dealt round-robin, as in grad_target_kernel).
template <int CF, bool BUF>
__global__ void __launch_bounds__(256) grad_target_tile_kernel(CostArgs a, int tiles_x, size_t n,
                                                               const uint32_t* __restrict__ start,
                                                               const uint32_t* __restrict__ skeys,
                                                               const uint32_t* __restrict__ svals) {
    constexpr int kSplit = row_split(CF);
    constexpr int L = CF / 4, G = kSplit * L, EPB = 256 / G;
    static_assert(G <= 64 && 64 % G == 0, "the parts of an entry share one wave");
    __shared__ uint32_t s_st[kWinN][kTileC + 1];  // staged run start of each cell, and the row's end
    __shared__ uint32_t s_row[kWinN + 1];         // staged offset of each row's run
    __shared__ uint32_t s_gb[kWinN];              // sorted position of each row's run
    __shared__ uint32_t s_pos[kStageCap];         // (py << 16) | px
    __shared__ float s_g[kStageCap];
    __shared__ uint8_t s_cx[kStageCap];           // cell column - tx_lo
    __shared__ float4 s_fq[kTileQ * L];           // the entries' own vectors
    const int H = a.H, W = a.W;
    const size_t HW = (size_t)H * W;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tq = tile % tiles_x, rest = tile / tiles_x;
    const int qy = rest % H, kb = rest / H;
    const int b = kb % a.batch, k = kb / a.batch;
    const int qx0 = tq * kTileQ;
    const int ty0 = qy - kWin1;                                    // staged row 0
    const int tx_lo = max(qx0 - kWin1, 0), tx_hi = min(qx0 + kTileQ - 1 - kWin0, W - 1);
    const int ncol = tx_hi - tx_lo + 1;
    const size_t cbase = (size_t)k * n + (size_t)b * HW;          // cell (0, 0) of map k, image b
    if (threadIdx.x < kWinN) {
        const int r = threadIdx.x, ty = ty0 + r;
        uint32_t g0 = 0, len = 0;
        if (ty >= 0 && ty < H) {
            const size_t c0 = cbase + (size_t)ty * W + tx_lo;
            g0 = start[c0];
            len = start[c0 + ncol] - g0;
        }
        s_gb[r] = g0;
        s_row[r + 1] = len;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s_row[0] = 0;
        for (int r = 0; r < kWinN; ++r) s_row[r + 1] += s_row[r];
    }
    __syncthreads();
    const uint32_t total = s_row[kWinN];
    const bool staged = total <= (uint32_t)kStageCap;
    if (staged) {
        for (int idx = threadIdx.x; idx < kWinN * (kTileC + 1); idx += 256) {
            const int r = idx / (kTileC + 1), j = idx - r * (kTileC + 1), ty = ty0 + r;
            if (j > ncol) continue;
            uint32_t v = s_row[r];
            if (ty >= 0 && ty < H) v += start[cbase + (size_t)ty * W + tx_lo + j] - s_gb[r];
            s_st[r][j] = v;
        }
        for (uint32_t e = threadIdx.x; e < total; e += 256) {
            int r = 0;
#pragma unroll
            for (int rr = 1; rr < kWinN; ++rr) r += e >= s_row[rr] ? 1 : 0;
            const uint32_t ge = s_gb[r] + (e - s_row[r]);
            const uint32_t pix = svals[ge];
            const int cc = (int)((size_t)skeys[ge] - cbase - (size_t)(ty0 + r) * W);
            const int pl = (int)(pix - (size_t)b * HW);
            const int py = pl / W, px = pl - py * W;
            s_pos[e] = ((uint32_t)py << 16) | (uint32_t)px;
            s_g[e] = 2.f * a.gcost[pix];
            s_cx[e] = (uint8_t)(cc - tx_lo);
        }
    }
    const float* base = a.feat + (size_t)b * 4 * HW * CF;
    for (int idx = threadIdx.x; idx < kTileQ * L; idx += 256) {
        const int qx = qx0 + idx / L;
        if (qx < W)
            s_fq[idx] = reinterpret_cast<const float4*>(
                base + ((size_t)view(a.s, k + 1) * HW + (size_t)qy * W + qx) * CF)[idx % L];
    }
    __syncthreads();
    Vec4Map<BUF> R;
    R.init(base + (size_t)view(a.s, 0) * HW * CF, HW * CF * 4);
    const int mk = view(a.s, k + 1);
    const int sub = threadIdx.x % L, part = (threadIdx.x / L) % kSplit;  // part = accumulator
    auto rvec = [&](int py, int px, int wy, int wx) {
        return R.ld((uint32_t)(clampi(py + wy, 0, H - 1) * W + clampi(px + wx, 0, W - 1)) * L + sub, false);
    };
    for (int e0 = 0; e0 < kTileQ; e0 += EPB) {
        const int qx = qx0 + e0 + (int)threadIdx.x / G;
        const bool live = qx < W;
        const size_t q = (size_t)qy * W + qx;
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        float4 fq = make_float4(0.f, 0.f, 0.f, 0.f);
        if (live) fq = s_fq[(qx - qx0) * L + sub];
        const bool interior = qy >= kWin1 && qy <= H - 1 + kWin0 && qx >= kWin1 && qx <= W - 1 + kWin0;
        // the whole wave takes the interior path or none of it does (shuffles); a tile too
        // crowded to stage reads the same terms from the sorted lists in global memory
        if (__all(!live || interior)) {
            // the terms are the runs of the window rows wy = -3 .. 4 (cells (qy - wy, qx - 4 ..
            // qx + 3)), one after the other, in blocks of G: lane lg of the entry's G lanes
            // finds term i0 + lg (row, staged pixel, gathered vector, 2 g) once, and the lanes of
            // accumulator `part` take terms i0 + part, i0 + part + kSplit, ... from them by
            // shuffles, all their loads in flight together.  A vector equal to the accumulator's
            // previous one (a locally constant field reads one vector for the whole window) is not
            // loaded again but copied once all loads are back; the arithmetic is unchanged.
            constexpr int U = G / kSplit;  // terms per accumulator and block
            const int lg = (int)threadIdx.x % G, gbase = ((int)threadIdx.x & 63) - lg;
            const int j0 = qx - kWin1 - tx_lo;
            uint32_t rb[kWinN], rend[kWinN];
            uint32_t m = 0;
#pragma unroll
            for (int t = 0; t < kWinN; ++t) {
                const int r = qy - (kWin0 + t) - ty0;
                uint32_t b0 = 0, b1 = 0;
                if (live && staged) {
                    b0 = s_st[r][j0];
                    b1 = s_st[r][j0 + kWinN];
                } else if (live) {
                    const size_t c0 = cbase + (size_t)(ty0 + r) * W + (qx - kWin1);
                    b0 = start[c0];
                    b1 = start[c0 + kWinN];
                }
                rb[t] = b0 - m;  // staged (or sorted) index of term i of this row: rb[t] + i
                m += b1 - b0;
                rend[t] = m;
            }
            int pidx = -1;
            float4 pv = make_float4(0.f, 0.f, 0.f, 0.f);
            const uint32_t mmax = (uint32_t)__reduce_max_sync(~0ull, m);
            for (uint32_t i0 = 0; i0 < mmax; i0 += G) {
                const uint32_t it = i0 + (uint32_t)lg;
                int tidx = 0;
                float tg2 = 0.f;
                if (it < m) {
                    int t = 0;
#pragma unroll
                    for (int tt = 0; tt < kWinN - 1; ++tt) t += it >= rend[tt] ? 1 : 0;
                    const uint32_t e = rb[t] + it;
                    const int wy = kWin0 + t;
                    int py, px, wx;
                    if (staged) {
                        const uint32_t pos = s_pos[e];
                        tg2 = s_g[e];
                        py = (int)(pos >> 16);
                        px = (int)(pos & 0xFFFFu);
                        wx = qx - tx_lo - (int)s_cx[e];
                    } else {
                        const uint32_t pix = svals[e];
                        const int cc = (int)((size_t)skeys[e] - cbase - (size_t)(qy - wy) * W);
                        const int pl = (int)(pix - (size_t)b * HW);
                        py = pl / W;
                        px = pl - py * W;
                        tg2 = 2.f * a.gcost[pix];
                        wx = qx - cc;
                    }
                    tidx = clampi(py + wy, 0, H - 1) * W + clampi(px + wx, 0, W - 1);
                }
                float4 rv[U];
                float gv[U];
                int idx[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int src = gbase + u * kSplit + part;
                    idx[u] = __shfl(tidx, src);
                    gv[u] = __shfl(tg2, src);
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    rv[u] = R.ld((uint32_t)idx[u] * L + sub, idx[u] == (u ? idx[u - 1] : pidx));
                if constexpr (BUF) {
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (idx[u] == (u ? idx[u - 1] : pidx)) rv[u] = u ? rv[u - 1] : pv;
                    pidx = idx[U - 1];
                    pv = rv[U - 1];
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (i0 + (uint32_t)(u * kSplit + part) < m) fma4(-gv[u], rv[u], fq, acc);
            }
        } else if (live) {
            // the canonical order term by term; this lane adds terms part, part + kSplit, ...
            uint32_t i = 0;
            for (int wy = kWin0; wy <= kWin1; ++wy) {
                int ylo, yhi;
                preimage(qy, wy, H, ylo, yhi);
                for (int ty = ylo; ty <= yhi; ++ty)
                    for (int wx = kWin1; wx >= kWin0; --wx) {  // target cells in ascending x
                        int xlo, xhi;
                        preimage(qx, wx, W, xlo, xhi);
                        for (int tx = xlo; tx <= xhi; ++tx) {
                            if (staged) {
                                const int r = ty - ty0, j = tx - tx_lo;
                                const uint32_t e0 = s_st[r][j], e1 = s_st[r][j + 1];
                                for (uint32_t e = e0 + (part + kSplit - i % kSplit) % kSplit; e < e1; e += kSplit) {
                                    const uint32_t pos = s_pos[e];
                                    fma4(-s_g[e], rvec((int)(pos >> 16), (int)(pos & 0xFFFFu), wy, wx), fq, acc);
                                }
                                i += e1 - e0;
                            } else {
                                const size_t cell = cbase + (size_t)ty * W + tx;
                                const uint32_t e0 = start[cell], e1 = start[cell + 1];
                                for (uint32_t e = e0 + (part + kSplit - i % kSplit) % kSplit; e < e1; e += kSplit) {
                                    const uint32_t pix = svals[e];
                                    const int pl = (int)(pix - (size_t)b * HW);
                                    const int py = pl / W, px = pl - py * W;
                                    fma4(-2.f * a.gcost[pix], rvec(py, px, wy, wx), fq, acc);
                                }
                                i += e1 - e0;
                            }
                        }
                    }
            }
        }
        const float4 sum = sum_parts<kSplit, L>(acc);
        if (live && part == 0)
            reinterpret_cast<float4*>(a.out + ((size_t)b * 4 * HW + (size_t)mk * HW + q) * CF)[sub] = sum;
    }
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace of the backward: the key/value lists (two buffers each for the
// sort passes), the cell starts and the per-block digit counts.
struct BwdWs {
    size_t N, nblk, keys_a, vals_a, keys_b, vals_b, start, hist, sums, total;
};

BwdWs bwd_ws(size_t n) {
    BwdWs L;
    L.N = 3 * n;
    L.nblk = (L.N + kSortTile - 1) / kSortTile;
    L.keys_a = 0;
    L.vals_a = L.keys_a + align256(L.N * 4);
    L.keys_b = L.vals_a + align256(L.N * 4);
    L.vals_b = L.keys_b + align256(L.N * 4);
    L.start = L.vals_b + align256(L.N * 4);
    L.hist = L.start + align256((L.N + 1) * 4);
    L.sums = L.hist + align256(256 * L.nblk * 4);
    L.total = L.sums + align256((256 * L.nblk + 1023) / 1024 * 4);
    return L;
}

// Largest batch * H * W the backward takes: its lists hold 3 entries per pixel
// with 32-bit positions.
constexpr size_t kBwdMaxPixels = (size_t)1 << 30;

bool shape_ok(int batch, int H, int W, int cf, int dir) {
    if (batch < 1 || H < 1 || W < 1 || H > 16384 || W > 16384) return false;
    if ((size_t)batch * H * W >= (1ull << 31)) return false;
    if (cf != 4 && cf != 8 && cf != 16 && cf != 32 && cf != 64) return false;
    return dir == 1 || dir == -1;
}

template <template <int> class K, typename... Args>
void launch_cf(int cf, dim3 g, hipStream_t st, Args... args) {
    switch (cf) {
        case 4: hipLaunchKernelGGL(K<4>::fn, g, dim3(256), 0, st, args...); break;
        case 8: hipLaunchKernelGGL(K<8>::fn, g, dim3(256), 0, st, args...); break;
        case 16: hipLaunchKernelGGL(K<16>::fn, g, dim3(256), 0, st, args...); break;
        case 32: hipLaunchKernelGGL(K<32>::fn, g, dim3(256), 0, st, args...); break;
        default: hipLaunchKernelGGL(K<64>::fn, g, dim3(256), 0, st, args...); break;
    }
}

template <int CF>
struct FwdK {
    static constexpr auto fn = cost_fwd_kernel<CF>;
};

template <int CF>
struct FwdCoopK {
    static constexpr auto fn = cost_fwd_coop_kernel<CF>;
};
template <int CF>
struct RefK {
    static constexpr auto fn = grad_ref_kernel<CF>;
};
template <int CF>
struct TgtK {
    static constexpr auto fn = grad_target_kernel<CF>;
};

template <int CF>
struct RefTileK {
    static constexpr auto fn = grad_ref_tile_kernel<CF, true>;
};

template <int CF>
struct TgtTileK {
    static constexpr auto fn = grad_target_tile_kernel<CF, true>;
};

template <int CF>
struct RefTileWideK {
    static constexpr auto fn = grad_ref_tile_kernel<CF, false>;
};

template <int CF>
struct TgtTileWideK {
    static constexpr auto fn = grad_target_tile_kernel<CF, false>;
};

}  // namespace
}  // namespace sff

using namespace sff;

extern "C" sff_status sff_cost_f32_fwd(int32_t batch, int32_t H, int32_t W, int32_t cf, int32_t dir,
                                       const float* feat, const int16_t* hyp, float* cost_px,
                                       void* stream) {
    if (!shape_ok(batch, H, W, cf, dir) || !feat || !hyp || !cost_px) return SFF_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(feat) & 15) != 0 || (reinterpret_cast<uintptr_t>(hyp) & 7) != 0 ||
        (reinterpret_cast<uintptr_t>(cost_px) & 3) != 0)
        return SFF_ERR_INVALID_ARG;
    CostArgs a{feat, hyp, nullptr, cost_px, H, W, dir, batch};
    // SFF_COST_F32_EVAL=lane: one lane per pixel (testing and timing)
    const char* ev = std::getenv("SFF_COST_F32_EVAL");
    if (ev && std::strcmp(ev, "lane") == 0)
        launch_cf<FwdK>(cf, dim3((W + 63) / 64, (H + 3) / 4, batch), as_stream(stream), a);
    else
        launch_cf<FwdCoopK>(cf, dim3((unsigned)(((size_t)H * W * (cf / 4) + 255) / 256), batch), as_stream(stream),
                            a);
    return launch_status();
}

extern "C" size_t sff_cost_f32_bwd_workspace_bytes(int32_t batch, int32_t H, int32_t W) {
    if (batch < 1 || H < 1 || W < 1 || (size_t)batch * H * W > kBwdMaxPixels) return 0;
    return bwd_ws((size_t)batch * H * W).total;
}

extern "C" sff_status sff_cost_f32_bwd(int32_t batch, int32_t H, int32_t W, int32_t cf,
                                       int32_t dir, const float* feat, const int16_t* hyp,
                                       const float* grad_cost, float* grad_feat, void* workspace,
                                       size_t workspace_bytes, void* stream) {
    if (!shape_ok(batch, H, W, cf, dir) || !feat || !hyp || !grad_cost || !grad_feat)
        return SFF_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(feat) & 15) != 0 || (reinterpret_cast<uintptr_t>(hyp) & 7) != 0 ||
        (reinterpret_cast<uintptr_t>(grad_cost) & 3) != 0 ||
        (reinterpret_cast<uintptr_t>(grad_feat) & 15) != 0)
        return SFF_ERR_INVALID_ARG;
    const size_t n = (size_t)batch * H * W;
    if (n > kBwdMaxPixels) return SFF_ERR_UNSUPPORTED;
    const BwdWs L = bwd_ws(n);
    if (!workspace || workspace_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return SFF_ERR_WORKSPACE;
    hipStream_t st = as_stream(stream);
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    uint32_t* ka = reinterpret_cast<uint32_t*>(ws + L.keys_a);
    uint32_t* va = reinterpret_cast<uint32_t*>(ws + L.vals_a);
    uint32_t* kb = reinterpret_cast<uint32_t*>(ws + L.keys_b);
    uint32_t* vb = reinterpret_cast<uint32_t*>(ws + L.vals_b);
    uint32_t* start = reinterpret_cast<uint32_t*>(ws + L.start);
    uint32_t* hist = reinterpret_cast<uint32_t*>(ws + L.hist);
    uint32_t* sums = reinterpret_cast<uint32_t*>(ws + L.sums);
    const size_t nhist = 256 * L.nblk, nchunks = (nhist + 1023) / 1024;
    CostArgs a{feat, hyp, grad_cost, grad_feat, H, W, dir, batch};
    // SFF_COST_F32_EVAL=lane: one lane per gradient entry (same results; testing and timing)
    const char* ev = std::getenv("SFF_COST_F32_EVAL");
    const bool lane_grad = ev && std::strcmp(ev, "lane") == 0;
    const int tiles_x = (W + kTileQ - 1) / kTileQ;
    const dim3 grid((W + 63) / 64, (H + 3) / 4, batch);
    // maps below 2 GiB are read through 32-bit buffer offsets
    const bool buf = (size_t)H * W * cf * 4 <= (size_t)kSkipOff;
    // The reference-map gradient and the target-map gradients (with the
    // grouping they need) read the same inputs and write different maps, so
    // the reference gradient runs on the library's helper stream beside them
    // (SFF_COST_F32_SPLIT=0: one stream; identical results either way).
    const char* sp = std::getenv("SFF_COST_F32_SPLIT");
    std::unique_lock<std::mutex> lock(helper_lock(), std::defer_lock);
    HelperStream* hs = nullptr;
    if (!(sp && std::strcmp(sp, "0") == 0)) {
        lock.lock();
        hs = helper_for_current_device();
        if (hs && !helper_fork(hs, st)) return SFF_ERR_HIP;
    }
    hipStream_t sr = hs ? hs->stream : st;
    if (lane_grad)
        launch_cf<RefK>(cf, grid, sr, a);
    else if (buf)
        launch_cf<RefTileK>(cf, dim3((unsigned)((size_t)batch * H * tiles_x)), sr, a, tiles_x);
    else
        launch_cf<RefTileWideK>(cf, dim3((unsigned)((size_t)batch * H * tiles_x)), sr, a, tiles_x);
    // group the pixels by target centre: keys, then a stable radix sort
    const size_t N = L.N;
    hipLaunchKernelGGL(target_keys_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, hyp,
                       ka, va, H, W, dir, (uint32_t)n);
    int bits = 1;
    while (bits < 32 && (1ull << bits) < N) ++bits;
    uint32_t *kin = ka, *vin = va, *kout = kb, *vout = vb;
    for (int sh = 0; sh < bits; sh += 8) {
        hipLaunchKernelGGL(sort_hist_kernel, dim3((unsigned)L.nblk), dim3(256), 0, st,
                           (const uint32_t*)kin, N, sh, hist, (uint32_t)L.nblk);
        hipLaunchKernelGGL(sort_scan_chunks_kernel, dim3((unsigned)nchunks), dim3(1024), 0, st, hist,
                           nhist, sums);
        hipLaunchKernelGGL(sort_scan_sums_kernel, dim3(1), dim3(1024), 0, st, sums, nchunks);
        hipLaunchKernelGGL(sort_scatter_kernel, dim3((unsigned)L.nblk), dim3(256), 0, st,
                           (const uint32_t*)kin, (const uint32_t*)vin, kout, vout, N, sh,
                           (const uint32_t*)hist, (const uint32_t*)sums, (uint32_t)L.nblk);
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    hipLaunchKernelGGL(cell_starts_kernel, dim3((unsigned)((N + 1 + 255) / 256)), dim3(256), 0, st,
                       (const uint32_t*)kin, start, N);
    if (lane_grad) {
        for (int k = 0; k < 3; ++k)
            launch_cf<TgtK>(cf, grid, st, a, k, n, (const uint32_t*)start, (const uint32_t*)vin);
    } else if (buf) {
        launch_cf<TgtTileK>(cf, dim3((unsigned)((size_t)3 * batch * H * tiles_x)), st, a, tiles_x, n,
                            (const uint32_t*)start, (const uint32_t*)kin, (const uint32_t*)vin);
    } else {
        launch_cf<TgtTileWideK>(cf, dim3((unsigned)((size_t)3 * batch * H * tiles_x)), st, a, tiles_x, n,
                                (const uint32_t*)start, (const uint32_t*)kin, (const uint32_t*)vin);
    }
    const sff_status r = launch_status();
    if (hs && !helper_join(hs, st)) return SFF_ERR_HIP;
    return r;
}
