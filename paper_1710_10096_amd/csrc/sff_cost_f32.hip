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
//     stable radix sort, then every target entry gathers over the centres
//     whose window covers it.
// Both are deterministic (no floating-point atomics).
#include <rocprim/device/device_radix_sort.hpp>

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

// Reference-map gradient: one thread per entry q of R.
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
    float fq[CF], acc[CF];
    load_vec<CF>(base + ((size_t)mR * HW + (size_t)qy * W + qx) * CF, fq);
#pragma unroll
    for (int c = 0; c < CF; ++c) acc[c] = 0.f;
    for (int wy = kWin0; wy <= kWin1; ++wy) {
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
    float4* o = reinterpret_cast<float4*>(a.out + ((size_t)b * 4 * HW + (size_t)mR * HW +
                                                   (size_t)qy * W + qx) * CF);
#pragma unroll
    for (int k = 0; k < CF / 4; ++k) o[k] = make_float4(acc[4 * k], acc[4 * k + 1], acc[4 * k + 2], acc[4 * k + 3]);
}

// The same gradient with CF / 4 lanes per entry, four channels each (see
// grad_target_coop_kernel); every channel adds the same terms in the same
// order as grad_ref_kernel, so the results are identical.
template <int CF>
__global__ void __launch_bounds__(256) grad_ref_coop_kernel(CostArgs a) {
    constexpr int L = CF / 4, QPB = 256 / L;
    const int sub = threadIdx.x % L;
    const int H = a.H, W = a.W, b = blockIdx.y;
    const size_t HW = (size_t)H * W;
    const size_t q = (size_t)xcd_tile(blockIdx.x, gridDim.x) * QPB + threadIdx.x / L;  // a band of rows per XCD
    if (q >= HW) return;  // all L lanes of the entry together
    const int qy = (int)(q / W), qx = (int)(q - (size_t)qy * W);
    const float* base = a.feat + (size_t)b * 4 * HW * CF;
    const int mR = view(a.s, 0);
    const float4* M[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) M[k] = reinterpret_cast<const float4*>(base + (size_t)view(a.s, k + 1) * HW * CF) + sub;
    const float4 fq = reinterpret_cast<const float4*>(base + ((size_t)mR * HW + q) * CF)[sub];
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int wy = kWin0; wy <= kWin1; ++wy) {
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
                        const float4 tg = M[k][((size_t)clampi(t.y[k] + wy, 0, H - 1) * W +
                                                clampi(t.x[k] + wx, 0, W - 1)) * L];
                        acc.x = fmaf(g2, fq.x - tg.x, acc.x);
                        acc.y = fmaf(g2, fq.y - tg.y, acc.y);
                        acc.z = fmaf(g2, fq.z - tg.z, acc.z);
                        acc.w = fmaf(g2, fq.w - tg.w, acc.w);
                    }
                }
            }
    }
    reinterpret_cast<float4*>(a.out + ((size_t)b * 4 * HW + (size_t)mR * HW + q) * CF)[sub] = acc;
}

// Keys for grouping pixels by the target centre of correspondence k.
__global__ void target_keys_kernel(const int16_t* __restrict__ hyp, uint32_t* keys, uint32_t* vals,
                                   int H, int W, int s, int k, int batch) {
    const size_t HW = (size_t)H * W;
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= HW * batch) return;
    const int b = (int)(i / HW);
    const int pix = (int)(i - (size_t)b * HW);
    const int y = pix / W, x = pix - y * W;
    const Targets t = targets(hyp, i, y, x, s, H, W);
    keys[i] = (uint32_t)((size_t)b * HW + (size_t)t.y[k] * W + t.x[k]);
    vals[i] = (uint32_t)i;
}

// start[c] = first position of sorted key >= c, for every cell c in [0, n].
__global__ void cell_starts_kernel(const uint32_t* __restrict__ keys, uint32_t* start, size_t n) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i > n) return;
    const int64_t k = i < n ? (int64_t)keys[i] : (int64_t)n;
    const int64_t kp = i == 0 ? -1 : (int64_t)keys[i - 1];
    for (int64_t c = kp + 1; c <= k; ++c) start[c] = (uint32_t)i;
}

// The target gradients gather the window rows in row_split(CF) parts of
// consecutive rows, summed in part order: eight single rows up to 32 channels,
// four pairs of rows at 64 (the CF / 4 lanes of every part of an entry share
// one wave).
constexpr int row_split(int cf) { return cf <= 32 ? 8 : 4; }

// Gradient of target map k: one thread per entry q of that map; gathers over
// the centres t with clamp(t + w) = q and the pixels grouped at each centre.
template <int CF>
__global__ void __launch_bounds__(256) grad_target_kernel(CostArgs a, int k,
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
    float fq[CF], acc[CF];
    load_vec<CF>(base + ((size_t)mk * HW + (size_t)qy * W + qx) * CF, fq);
    float4* o = reinterpret_cast<float4*>(a.out + ((size_t)b * 4 * HW + (size_t)mk * HW +
                                                   (size_t)qy * W + qx) * CF);
    // the window rows in kSplit parts of consecutive rows; the gradient is
    // ((part 0 + part 1) + part 2) + ...
    constexpr int kSplit = row_split(CF), kPartRows = (kWin1 - kWin0 + 1) / kSplit;
    static_assert(kPartRows * kSplit == kWin1 - kWin0 + 1, "rows split evenly");
    for (int part = 0; part < kSplit; ++part) {
#pragma unroll
        for (int c = 0; c < CF; ++c) acc[c] = 0.f;
        for (int wy = kWin0 + part * kPartRows; wy < kWin0 + (part + 1) * kPartRows; ++wy) {
            int ylo, yhi;
            preimage(qy, wy, H, ylo, yhi);
            for (int ty = ylo; ty <= yhi; ++ty)
                for (int wx = kWin1; wx >= kWin0; --wx) {  // target cells in ascending x
                    int xlo, xhi;
                    preimage(qx, wx, W, xlo, xhi);
                    for (int tx = xlo; tx <= xhi; ++tx) {
                        const size_t cell = (size_t)b * HW + (size_t)ty * W + tx;
                        const uint32_t e0 = start[cell], e1 = start[cell + 1];
                        for (uint32_t e = e0; e < e1; ++e) {
                            const uint32_t pix = order[e];
                            const int pl = (int)(pix - (size_t)b * HW);
                            const int py = pl / W, px = pl - py * W;
                            const float g2 = 2.f * a.gcost[pix];
                            float r[CF];
                            load_vec<CF>(R + ((size_t)clampi(py + wy, 0, H - 1) * W +
                                              clampi(px + wx, 0, W - 1)) * CF, r);
#pragma unroll
                            for (int c = 0; c < CF; ++c) acc[c] = fmaf(-g2, r[c] - fq[c], acc[c]);
                        }
                    }
                }
        }
#pragma unroll
        for (int kk = 0; kk < CF / 4; ++kk) {
            float4 v = make_float4(acc[4 * kk], acc[4 * kk + 1], acc[4 * kk + 2], acc[4 * kk + 3]);
            if (part) {
                const float4 lo = o[kk];
                v = make_float4(lo.x + v.x, lo.y + v.y, lo.z + v.z, lo.w + v.w);
            }
            o[kk] = v;
        }
    }
}

// Blocks of the target-gradient launch (a multiple of 8): 32 per compute unit,
// four times what is resident at once (8 per unit measured 7% slower, 16 to 64
// the same).
constexpr size_t kTgtBlocks = 256 * 32;

// The same gradient with CF / 4 lanes per target entry, each owning four
// channels: a gathered vector is CF / 4 consecutive 16-byte loads of
// neighbouring lanes (a few cache lines per load instruction instead of one per
// lane), a lane holds a float4 accumulator instead of CF, and a wave covers
// 256 / (CF / 4) / 4 entries, so far fewer lanes wait on the slowest entry of
// their wave.  row_split(CF) groups of CF / 4 lanes share an entry, each taking
// one part of the window rows, which shortens the serial chain of each; every
// channel adds the same terms in the same order as grad_target_kernel (each
// part in turn, then their sum in part order), so the results are identical.
template <int CF>
__global__ void __launch_bounds__(256) grad_target_coop_kernel(CostArgs a, int k,
                                                               const uint32_t* __restrict__ start,
                                                               const uint32_t* __restrict__ order) {
    constexpr int kSplit = row_split(CF), kPartRows = (kWin1 - kWin0 + 1) / kSplit;
    constexpr int L = CF / 4, G = kSplit * L, QPB = 256 / G;
    static_assert(G <= 64, "the parts of an entry share one wave");
    const int sub = threadIdx.x % L, part = (threadIdx.x / L) % kSplit;
    const int wy0 = kWin0 + part * kPartRows, wy1 = wy0 + kPartRows - 1;  // this part's window rows
    const int H = a.H, W = a.W, b = blockIdx.y;
    const size_t HW = (size_t)H * W;
    const float* base = a.feat + (size_t)b * 4 * HW * CF;
    const float4* R = reinterpret_cast<const float4*>(base + (size_t)view(a.s, 0) * HW * CF) + sub;
    const int mk = view(a.s, k + 1);
    // A fixed grid (a multiple of 8 blocks) walks the tiles of QPB entries: the
    // blocks of one XCD take that XCD's band of image rows in turn, so a wave
    // handles many entries instead of one short entry each.
    const int ntiles = (int)((HW + QPB - 1) / QPB);
    const int xcd = blockIdx.x & 7, per = gridDim.x >> 3, nq = ntiles >> 3, rem = ntiles & 7;
    const int t0 = xcd * nq + min(xcd, rem), t1 = t0 + nq + (xcd < rem ? 1 : 0);
    for (int tile = t0 + (int)(blockIdx.x >> 3); tile < t1; tile += per) {
        const size_t q = (size_t)tile * QPB + threadIdx.x / G;
        if (q >= HW) continue;  // all G lanes of the entry together; only in the last tile
        const int qy = (int)(q / W), qx = (int)(q - (size_t)qy * W);
        const float4 fq = reinterpret_cast<const float4*>(base + ((size_t)mk * HW + q) * CF)[sub];
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        auto add = [&](uint32_t pix, int wy, int wx) {
            const int pl = (int)(pix - (size_t)b * HW);
            const int py = pl / W, px = pl - py * W;
            const float g2 = 2.f * a.gcost[pix];
            const float4 r = R[((size_t)clampi(py + wy, 0, H - 1) * W + clampi(px + wx, 0, W - 1)) * L];
            acc.x = fmaf(-g2, r.x - fq.x, acc.x);
            acc.y = fmaf(-g2, r.y - fq.y, acc.y);
            acc.z = fmaf(-g2, r.z - fq.z, acc.z);
            acc.w = fmaf(-g2, r.w - fq.w, acc.w);
        };
        constexpr int kN = kWin1 - kWin0 + 1;  // 8 window columns
        if (qy >= kWin1 && qy <= H - 1 + kWin0 && qx >= kWin1 && qx <= W - 1 + kWin0) {
            // interior: window row wy covers the centre cells (qy - wy, qx - 4 .. qx + 3), consecutive,
            // so their pixels are one run [st[0], st[8]) of the sorted order; it is walked in that
            // order (cells by ascending x, the order of the generic loop below) four at a time
            for (int wy = wy0; wy <= wy1; ++wy) {
                const size_t c0 = (size_t)b * HW + (size_t)(qy - wy) * W + (qx - kWin1);
                uint32_t st[kN + 1];
#pragma unroll
                for (int j = 0; j <= kN; ++j) st[j] = start[c0 + j];
                for (uint32_t e = st[0]; e < st[kN]; e += 4) {
                    uint32_t pv[4];
                    int wxv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const uint32_t eu = min(e + u, st[kN] - 1);
                        pv[u] = order[eu];
                        int j = 0;
#pragma unroll
                        for (int jj = 1; jj < kN; ++jj) j += eu >= st[jj] ? 1 : 0;
                        wxv[u] = kWin1 - j;
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (e + u < st[kN]) add(pv[u], wy, wxv[u]);
                }
            }
        } else {
            for (int wy = wy0; wy <= wy1; ++wy) {
                int ylo, yhi;
                preimage(qy, wy, H, ylo, yhi);
                for (int ty = ylo; ty <= yhi; ++ty)
                    for (int wx = kWin1; wx >= kWin0; --wx) {  // target cells in ascending x
                        int xlo, xhi;
                        preimage(qx, wx, W, xlo, xhi);
                        for (int tx = xlo; tx <= xhi; ++tx) {
                            const size_t cell = (size_t)b * HW + (size_t)ty * W + tx;
                            const uint32_t e0 = start[cell], e1 = start[cell + 1];
                            for (uint32_t e = e0; e < e1; ++e) add(order[e], wy, wx);
                        }
                    }
            }
        }
        // ((part 0 + part 1) + part 2) + ..., as the one-lane kernel adds them
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
        if (part == 0)
            reinterpret_cast<float4*>(a.out + ((size_t)b * 4 * HW + (size_t)mk * HW + q) * CF)[sub] = sum;
    }
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct BwdWs {
    size_t keys_in, vals_in, keys_out, order, start, temp, temp_bytes, total;
};

bool bwd_ws(size_t n, BwdWs* L) {
    size_t temp = 0;
    if (rocprim::radix_sort_pairs(nullptr, temp, (uint32_t*)nullptr, (uint32_t*)nullptr,
                                  (uint32_t*)nullptr, (uint32_t*)nullptr, n) != hipSuccess)
        return false;
    L->keys_in = 0;
    L->vals_in = L->keys_in + align256(n * 4);
    L->keys_out = L->vals_in + align256(n * 4);
    L->order = L->keys_out + align256(n * 4);
    L->start = L->order + align256(n * 4);
    L->temp = L->start + align256((n + 1) * 4);
    L->temp_bytes = temp;
    L->total = L->temp + align256(temp);
    return true;
}

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
struct RefCoopK {
    static constexpr auto fn = grad_ref_coop_kernel<CF>;
};

template <int CF>
struct TgtCoopK {
    static constexpr auto fn = grad_target_coop_kernel<CF>;
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
    if (batch < 1 || H < 1 || W < 1 || (size_t)batch * H * W >= (1ull << 31)) return 0;
    BwdWs L;
    if (!bwd_ws((size_t)batch * H * W, &L)) return 0;
    return L.total;
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
    BwdWs L;
    if (!bwd_ws(n, &L)) return SFF_ERR_HIP;
    if (!workspace || workspace_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return SFF_ERR_WORKSPACE;
    hipStream_t st = as_stream(stream);
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    uint32_t* keys_in = reinterpret_cast<uint32_t*>(ws + L.keys_in);
    uint32_t* vals_in = reinterpret_cast<uint32_t*>(ws + L.vals_in);
    uint32_t* keys_out = reinterpret_cast<uint32_t*>(ws + L.keys_out);
    uint32_t* order = reinterpret_cast<uint32_t*>(ws + L.order);
    uint32_t* start = reinterpret_cast<uint32_t*>(ws + L.start);
    CostArgs a{feat, hyp, grad_cost, grad_feat, H, W, dir, batch};
    const dim3 grid((W + 63) / 64, (H + 3) / 4, batch);
    // SFF_COST_F32_EVAL=lane: one lane per gradient entry (same results; testing and timing)
    const char* ev = std::getenv("SFF_COST_F32_EVAL");
    const bool lane_grad = ev && std::strcmp(ev, "lane") == 0;
    const dim3 cgrid((unsigned)(((size_t)H * W * (cf / 4) + 255) / 256), batch);
    if (lane_grad)
        launch_cf<RefK>(cf, grid, st, a);
    else
        launch_cf<RefCoopK>(cf, cgrid, st, a);
    unsigned int bits = 1;
    while (bits < 32 && (1ull << bits) < n) ++bits;
    for (int k = 0; k < 3; ++k) {
        hipLaunchKernelGGL(target_keys_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                           hyp, keys_in, vals_in, H, W, dir, k, batch);
        size_t temp = L.temp_bytes;
        if (rocprim::radix_sort_pairs(ws + L.temp, temp, keys_in, keys_out, vals_in, order, n, 0,
                                      bits, st) != hipSuccess)
            return SFF_ERR_HIP;
        hipLaunchKernelGGL(cell_starts_kernel, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0,
                           st, keys_out, start, n);
        if (lane_grad)
            launch_cf<TgtK>(cf, grid, st, a, k, (const uint32_t*)start, (const uint32_t*)order);
        else
            launch_cf<TgtCoopK>(cf, dim3((unsigned)std::min<size_t>(((((size_t)H * W * (cf / 4) * row_split(cf) + 255) / 256) + 7) & ~(size_t)7, kTgtBlocks), batch),
                                st, a, k, (const uint32_t*)start, (const uint32_t*)order);
    }
    return launch_status();
}
