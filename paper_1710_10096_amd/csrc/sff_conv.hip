// Learned feature extractor: 3x3 convolutions on BF16 NHWC tensors with FP32
// accumulation on the matrix cores (v_mfma_f32_16x16x32_bf16), used in place
// of the WHT features of the matching cost (Section 3.1).  Zero padding,
// dilation d; weights [Cout][3][3][Cin] (tap (ky, kx) reads offset
// ((ky - 1) d, (kx - 1) d)), bias FP32.
//
//   forward:  y = act(b + sum_tap W_tap x_shift)            implicit GEMM, K = 9 Cin
//   dgrad:    dx = conv(dz, W') with W'[i][ky][kx][o] = W[o][2-ky][2-kx][i],
//             dz = dy * (relu_out > 0) when the layer had a ReLU
//   wgrad:    dW_tap = sum_p dz[p] x[p + tap]^T,  db = sum_p dz[p]
//
// MFMA lane layout (16 x 16 x 32): lane l supplies row (A) / column (B) l % 16
// and eight K values for lane group l / 16; it receives C[4 (l / 16) + e][l % 16].
#include <hip/hip_bfloat16.h>

#include <cstdlib>
#include <cstring>

#include "sff_internal.hpp"

namespace sff {
namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef uint16_t bf16_t;  // raw bfloat16 bits in memory

__device__ __forceinline__ float bf2f(bf16_t v) { return __uint_as_float((uint32_t)v << 16); }

// Two values rounded to nearest even by the conversion instruction of gfx950
// (v_cvt_pk_bf16_f32; infinities kept, NaNs quiet), packed (lo, hi).
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t f2bf2(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((v2f){lo, hi}, v2bf));
}

constexpr int kTilePx = 64;  // output pixels per block (one row segment)
constexpr int kMaxDil = 16;  // largest dilation

// ---------------------------------------------------------------- forward --
// Block: 64 consecutive pixels of one row, 4 waves of 16 pixels, all COUT
// channels.  LDS: weights [COUT][KP] and the im2col tile [64][KP] (KP = 9 CIN
// rounded up to 32, zero padded).  `mask` (optional) multiplies each input
// value by (mask > 0), which folds a ReLU derivative into the gradient path.
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) conv_fwd_kernel(const bf16_t* __restrict__ x,
                                                       const bf16_t* __restrict__ mask,
                                                       const bf16_t* __restrict__ w,
                                                       const float* __restrict__ bias,
                                                       bf16_t* __restrict__ y, int H, int W, int dil,
                                                       int relu) {
    constexpr int K = 9 * CIN, KP = (K + 31) / 32 * 32;
    __shared__ __align__(16) bf16_t wl[COUT * KP];
    __shared__ __align__(16) bf16_t col[kTilePx * KP];
    const int x0 = blockIdx.x * kTilePx, row = blockIdx.y, n = blockIdx.z;
    const size_t img = (size_t)n * H * W;
    for (int e = threadIdx.x; e < COUT * KP; e += 256) {
        const int o = e / KP, k = e - o * KP;
        wl[e] = k < K ? w[(size_t)o * K + k] : (bf16_t)0;
    }
    for (int e = threadIdx.x; e < kTilePx * KP; e += 256) {
        const int p = e / KP, k = e - p * KP;
        bf16_t v = 0;
        if (k < K) {
            const int tap = k / CIN, i = k - tap * CIN;
            const int yy = row + (tap / 3 - 1) * dil, xx = x0 + p + (tap % 3 - 1) * dil;
            if (yy >= 0 && yy < H && xx >= 0 && xx < W && x0 + p < W) {
                const size_t o = (img + (size_t)yy * W + xx) * CIN + i;
                v = x[o];
                if (mask && !(bf2f(mask[o]) > 0.f)) v = 0;
            }
        }
        col[e] = v;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ln = lane & 15, g = lane >> 4;
    v4f acc[COUT / 16];
#pragma unroll
    for (int t = 0; t < COUT / 16; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
    const bf16_t* bcol = col + (wv * 16 + ln) * KP + 8 * g;
#pragma unroll
    for (int ks = 0; ks < KP / 32; ++ks) {
        const v8bf bv = *reinterpret_cast<const v8bf*>(bcol + ks * 32);
#pragma unroll
        for (int t = 0; t < COUT / 16; ++t) {
            const v8bf av = *reinterpret_cast<const v8bf*>(wl + (t * 16 + ln) * KP + ks * 32 + 8 * g);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[t], 0, 0, 0);
        }
    }
    const int px = x0 + wv * 16 + ln;
    if (px >= W) return;
    bf16_t* out = y + (img + (size_t)row * W + px) * COUT;
#pragma unroll
    for (int t = 0; t < COUT / 16; ++t) {
        uint32_t packed[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            float v0 = acc[t][2 * h] + (bias ? bias[t * 16 + 4 * g + 2 * h] : 0.f);
            float v1 = acc[t][2 * h + 1] + (bias ? bias[t * 16 + 4 * g + 2 * h + 1] : 0.f);
            if (relu) {
                v0 = fmaxf(v0, 0.f);
                v1 = fmaxf(v1, 0.f);
            }
            packed[h] = f2bf2(v0, v1);
        }
        *reinterpret_cast<uint2*>(out + t * 16 + 4 * g) = make_uint2(packed[0], packed[1]);
    }
}

// The same convolution for Cin = Cout = 32 without an im2col tile: with K
// ordered (tap, channel), the 32 K values of one MFMA step are the 32 channels
// of one input pixel, so lane (pixel l % 16, group l / 16) reads its B
// operand, 8 channels = 16 bytes, straight from the staged input rows.  Block:
// kTile32 consecutive pixels of one row, 4 waves of 64 (4 groups of 16); LDS
// holds the three input rows the taps read (kTile32 + 2 dil pixels each, 80-byte
// pixel stride so the 16 lanes of a read hit distinct banks), filled with
// 16-byte loads; each lane keeps its 18 weight fragments (9 taps x 2 output
// tiles) in registers.  Same MFMAs in the same order on the same values as
// conv_fwd_kernel<32, 32>, so the results are identical.  x (and mask) must be
// 16-byte aligned.
constexpr int kTile32 = 256;
constexpr int kPxStride = 40;  // bf16 per staged pixel (32 used)
constexpr int kStageW = kTile32 + 2 * kMaxDil;
constexpr int kRows32 = 4;  // output rows per block (the weight fragments are loaded once)

__global__ void __launch_bounds__(256) conv32_fwd_kernel(const bf16_t* __restrict__ x,
                                                         const bf16_t* __restrict__ mask,
                                                         const bf16_t* __restrict__ w,
                                                         const float* __restrict__ bias,
                                                         bf16_t* __restrict__ y, int H, int W, int dil,
                                                         int relu) {
    __shared__ __align__(16) bf16_t rows[3][kStageW * kPxStride];
    const int x0 = blockIdx.x * kTile32, n = blockIdx.z;
    const size_t img = (size_t)n * H * W;
    const int nx = kTile32 + 2 * dil;  // staged pixels per row
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ln = lane & 15, g = lane >> 4;
    // weight fragments: output 16 t + ln, tap, channels 8 g .. 8 g + 7 (kept for all rows)
    v8bf a[2][9];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
            a[t][tap] = *reinterpret_cast<const v8bf*>(w + ((size_t)(t * 16 + ln) * 9 + tap) * 32 + 8 * g);
    for (int rr = 0; rr < kRows32; ++rr) {
        const int row = blockIdx.y * kRows32 + rr;
        if (row >= H) break;  // block-uniform
        __syncthreads();      // the previous row's reads of the staged rows are done
        // stage: 4 x 16 bytes per pixel, zero outside the image
        for (int e = threadIdx.x; e < 3 * nx * 4; e += 256) {
            const int ky = e / (nx * 4), r = e - ky * nx * 4, px = r >> 2, q = r & 3;
            const int yy = row + (ky - 1) * dil, xx = x0 - dil + px;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (yy >= 0 && yy < H && xx >= 0 && xx < W) {
                const size_t o = (img + (size_t)yy * W + xx) * 32 + 8 * q;
                v = *reinterpret_cast<const uint4*>(x + o);
                if (mask) {
                    const uint4 m = *reinterpret_cast<const uint4*>(mask + o);
                    const uint32_t mw[4] = {m.x, m.y, m.z, m.w};
                    uint32_t vw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        const uint32_t lo = bf2f((bf16_t)(mw[h] & 0xFFFFu)) > 0.f ? 0x0000FFFFu : 0u;
                        const uint32_t hi = bf2f((bf16_t)(mw[h] >> 16)) > 0.f ? 0xFFFF0000u : 0u;
                        vw[h] &= lo | hi;
                    }
                    v = make_uint4(vw[0], vw[1], vw[2], vw[3]);
                }
            }
            *reinterpret_cast<uint4*>(&rows[ky][px * kPxStride + 8 * q]) = v;
        }
        __syncthreads();
#pragma unroll 1
        for (int grp = 0; grp < 4; ++grp) {
            const int p = wv * 64 + grp * 16 + ln;  // pixel of this lane's B column within the tile
            v4f acc[2] = {v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int ky = tap / 3, kx = tap - 3 * ky;
                const v8bf bv = *reinterpret_cast<const v8bf*>(&rows[ky][(p + kx * dil) * kPxStride + 8 * g]);
                acc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][tap], bv, acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][tap], bv, acc[1], 0, 0, 0);
            }
            const int px = x0 + p;
            if (px < W) {
                bf16_t* out = y + (img + (size_t)row * W + px) * 32;
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    uint32_t packed[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        float v0 = acc[t][2 * h] + (bias ? bias[t * 16 + 4 * g + 2 * h] : 0.f);
                        float v1 = acc[t][2 * h + 1] + (bias ? bias[t * 16 + 4 * g + 2 * h + 1] : 0.f);
                        if (relu) {
                            v0 = fmaxf(v0, 0.f);
                            v1 = fmaxf(v1, 0.f);
                        }
                        packed[h] = f2bf2(v0, v1);
                    }
                    *reinterpret_cast<uint2*>(out + t * 16 + 4 * g) = make_uint2(packed[0], packed[1]);
                }
            }
        }
    }
}

// The first layer (Cin = 3: K = 27, one MFMA step) without an im2col tile:
// the three input rows of a 256-pixel tile are staged in LDS and each lane
// reads its 8 (tap, channel) K values straight from them; the two weight
// fragments stay in registers for the block's rows.  Same operands as
// conv_fwd_kernel<3, 32>, so the same results.
__global__ void __launch_bounds__(256) conv3_fwd_kernel(const bf16_t* __restrict__ x,
                                                        const bf16_t* __restrict__ w,
                                                        const float* __restrict__ bias,
                                                        bf16_t* __restrict__ y, int H, int W, int dil,
                                                        int relu) {
    __shared__ bf16_t rows[3][kStageW * 3];
    const int x0 = blockIdx.x * kTile32, n = blockIdx.z;
    const size_t img = (size_t)n * H * W;
    const int nx = kTile32 + 2 * dil;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ln = lane & 15, g = lane >> 4;
    v8bf a[2];
    int koff[8];  // LDS offset of K value 8 g + e relative to the lane's pixel (-1: zero padding)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = 8 * g + e;
#pragma unroll
        for (int t = 0; t < 2; ++t)
            a[t][e] = __builtin_bit_cast(__bf16, k < 27 ? w[(size_t)(t * 16 + ln) * 27 + k] : (bf16_t)0);
        const int tap = k / 3, ci = k - 3 * tap, ky = tap / 3, kx = tap - 3 * ky;
        koff[e] = k < 27 ? ky * kStageW * 3 + kx * dil * 3 + ci : -1;
    }
    for (int rr = 0; rr < kRows32; ++rr) {
        const int row = blockIdx.y * kRows32 + rr;
        if (row >= H) break;  // block-uniform
        __syncthreads();
        for (int e = threadIdx.x; e < 3 * nx * 3; e += 256) {
            const int ky = e / (nx * 3), r = e - ky * nx * 3, px = r / 3, ci = r - 3 * px;
            const int yy = row + (ky - 1) * dil, xx = x0 - dil + px;
            bf16_t v = 0;
            if (yy >= 0 && yy < H && xx >= 0 && xx < W) v = x[(img + (size_t)yy * W + xx) * 3 + ci];
            rows[ky][px * 3 + ci] = v;
        }
        __syncthreads();
#pragma unroll 1
        for (int grp = 0; grp < 4; ++grp) {
            const int p = wv * 64 + grp * 16 + ln;
            const bf16_t* src = &rows[0][p * 3];
            v8bf bv;
#pragma unroll
            for (int e = 0; e < 8; ++e) bv[e] = __builtin_bit_cast(__bf16, koff[e] >= 0 ? src[koff[e]] : (bf16_t)0);
            v4f acc[2];
#pragma unroll
            for (int t = 0; t < 2; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], bv, v4f{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            const int px = x0 + p;
            if (px < W) {
                bf16_t* out = y + (img + (size_t)row * W + px) * 32;
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    uint32_t packed[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        float v0 = acc[t][2 * h] + (bias ? bias[t * 16 + 4 * g + 2 * h] : 0.f);
                        float v1 = acc[t][2 * h + 1] + (bias ? bias[t * 16 + 4 * g + 2 * h + 1] : 0.f);
                        if (relu) {
                            v0 = fmaxf(v0, 0.f);
                            v1 = fmaxf(v1, 0.f);
                        }
                        packed[h] = f2bf2(v0, v1);
                    }
                    *reinterpret_cast<uint2*>(out + t * 16 + 4 * g) = make_uint2(packed[0], packed[1]);
                }
            }
        }
    }
}

// W'[i][ky][kx][o] = W[o][2 - ky][2 - kx][i]
__global__ void flip_weights_kernel(const bf16_t* __restrict__ w, bf16_t* __restrict__ wt, int cin,
                                    int cout) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= cin * 9 * cout) return;
    const int i = e / (9 * cout), r = e - i * 9 * cout;
    const int tap = r / cout, o = r - tap * cout;
    wt[e] = w[((size_t)o * 9 + (8 - tap)) * cin + i];
}

// ------------------------------------------------------------ weight grad --
// Block: a 64-pixel-wide band of kWgRows rows.  For every row segment the
// block stages dz^T [COUT][64] and, for each kernel row, the input row
// transposed [CIN][64 + 2 d] in LDS; wave t accumulates the (o-tile, i-tile)
// pair t for all 9 taps (K = pixels).  Partial results per block are reduced
// in a fixed order by a second kernel.
constexpr int kWgRows = 32;  // 960 blocks on four KITTI-size images: 1.3% faster per training step than 16; 8 and 64 slower

template <int CIN, int COUT>
__global__ void __launch_bounds__(256) conv_wgrad_kernel(const bf16_t* __restrict__ x,
                                                         const bf16_t* __restrict__ dy,
                                                         const bf16_t* __restrict__ mask,
                                                         float* __restrict__ part, int H, int W,
                                                         int dil, int vec) {
    constexpr int IT = (CIN + 15) / 16, OT = COUT / 16, XW = kTilePx + 2 * kMaxDil;
    __shared__ __align__(16) bf16_t dzT[COUT][kTilePx];
    __shared__ __align__(16) bf16_t xT[3][IT * 16][XW];
    __shared__ float dbs[4][COUT];
    const int x0 = blockIdx.x * kTilePx, r0 = blockIdx.y * kWgRows, n = blockIdx.z;
    const size_t img = (size_t)n * H * W;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ln = lane & 15, g = lane >> 4;
    // wave wv handles pairs wv, wv + 4, ... of the OT x IT (o-tile, i-tile) grid
    constexpr int NP = OT * IT, PPW = (NP + 3) / 4;
    v4f acc[PPW][9];
#pragma unroll
    for (int q = 0; q < PPW; ++q)
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[q][t] = v4f{0.f, 0.f, 0.f, 0.f};
    float db = 0.f;  // thread (wv, lane < COUT) sums dz of channel lane over its pixels
    for (int rr = 0; rr < kWgRows; ++rr) {
        const int row = r0 + rr;
        if (row >= H) break;
        __syncthreads();
        bool staged = false;
        if constexpr (CIN == 32 && COUT == 32) {
            if (vec) {
                // 16-byte loads (8 channels of one pixel), scattered transposed into LDS
                {
                    const int p = threadIdx.x >> 2, q = threadIdx.x & 3;  // 64 pixels x 4 pieces
                    uint4 v = make_uint4(0u, 0u, 0u, 0u);
                    if (x0 + p < W) {
                        const size_t off = (img + (size_t)row * W + x0 + p) * 32 + 8 * q;
                        v = *reinterpret_cast<const uint4*>(dy + off);
                        if (mask) {
                            const uint4 m = *reinterpret_cast<const uint4*>(mask + off);
                            const uint32_t mw[4] = {m.x, m.y, m.z, m.w};
                            uint32_t vw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                            for (int h = 0; h < 4; ++h) {
                                const uint32_t lo = bf2f((bf16_t)(mw[h] & 0xFFFFu)) > 0.f ? 0x0000FFFFu : 0u;
                                const uint32_t hi = bf2f((bf16_t)(mw[h] >> 16)) > 0.f ? 0xFFFF0000u : 0u;
                                vw[h] &= lo | hi;
                            }
                            v = make_uint4(vw[0], vw[1], vw[2], vw[3]);
                        }
                    }
                    const uint32_t vw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int t = 0; t < 8; ++t) dzT[8 * q + t][p] = (bf16_t)(vw[t >> 1] >> (16 * (t & 1)));
                }
                for (int e = threadIdx.x; e < 3 * XW * 4; e += 256) {
                    const int ky = e / (XW * 4), r = e - ky * XW * 4, j = r >> 2, q = r & 3;
                    const int yy = row + (ky - 1) * dil, xx = x0 - kMaxDil + j;
                    uint4 v = make_uint4(0u, 0u, 0u, 0u);
                    if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                        v = *reinterpret_cast<const uint4*>(x + (img + (size_t)yy * W + xx) * 32 + 8 * q);
                    const uint32_t vw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int t = 0; t < 8; ++t) xT[ky][8 * q + t][j] = (bf16_t)(vw[t >> 1] >> (16 * (t & 1)));
                }
                staged = true;
            }
        }
        if (!staged) {
            for (int e = threadIdx.x; e < COUT * kTilePx; e += 256) {
                const int p = e / COUT, o = e - p * COUT;
                bf16_t v = 0;
                if (x0 + p < W) {
                    const size_t off = (img + (size_t)row * W + x0 + p) * COUT + o;
                    v = dy[off];
                    if (mask && !(bf2f(mask[off]) > 0.f)) v = 0;
                }
                dzT[o][p] = v;
            }
            for (int e = threadIdx.x; e < 3 * IT * 16 * XW; e += 256) {
                const int ky = e / (IT * 16 * XW), r = e - ky * IT * 16 * XW;
                const int c = r / XW, j = r - c * XW;
                const int yy = row + (ky - 1) * dil, xx = x0 - kMaxDil + j;
                bf16_t v = 0;
                if (c < CIN && yy >= 0 && yy < H && xx >= 0 && xx < W)
                    v = x[(img + (size_t)yy * W + xx) * CIN + c];
                xT[ky][c][j] = v;
            }
        }
        __syncthreads();
        if (lane < COUT) {
            float s = 0.f;
            for (int p = wv * 16; p < wv * 16 + 16; ++p) s += bf2f(dzT[lane][p]);
            db += s;
        }
#pragma unroll
        for (int q = 0; q < PPW; ++q) {
            const int pair = wv + 4 * q;
            if (pair >= NP) break;
            const int ot = pair / IT, it = pair - ot * IT;
#pragma unroll
            for (int ks = 0; ks < kTilePx / 32; ++ks) {
                const v8bf av = *reinterpret_cast<const v8bf*>(&dzT[ot * 16 + ln][ks * 32 + 8 * g]);
#pragma unroll
                for (int tap = 0; tap < 9; ++tap) {
                    const int ky = tap / 3, kx = tap % 3;
                    const bf16_t* src = &xT[ky][it * 16 + ln][kMaxDil + (kx - 1) * dil + ks * 32 + 8 * g];
                    v8bf bv;
#pragma unroll
                    for (int e = 0; e < 8; ++e) bv[e] = __builtin_bit_cast(__bf16, src[e]);
                    acc[q][tap] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[q][tap], 0, 0, 0);
                }
            }
        }
    }
    // partial layout: [block][COUT][9][IT*16] + db [block][COUT] (after all blocks)
    const size_t blk = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    float* pw = part + blk * COUT * 9 * IT * 16;
#pragma unroll
    for (int q = 0; q < PPW; ++q) {
        const int pair = wv + 4 * q;
        if (pair >= NP) break;
        const int ot = pair / IT, it = pair - ot * IT;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                pw[((size_t)(ot * 16 + 4 * g + e) * 9 + tap) * IT * 16 + it * 16 + ln] = acc[q][tap][e];
    }
    if (lane < COUT) dbs[wv][lane] = db;
    __syncthreads();
    if (threadIdx.x < COUT) {
        const size_t nblk = (size_t)gridDim.x * gridDim.y * gridDim.z;
        part[nblk * COUT * 9 * IT * 16 + blk * COUT + threadIdx.x] =
            dbs[0][threadIdx.x] + dbs[1][threadIdx.x] + dbs[2][threadIdx.x] + dbs[3][threadIdx.x];
    }
}

// Fixed-order sum of the per-block partials: dw [COUT][3][3][CIN], db [COUT].
// Sum of the per-block partials, in a fixed order: 16 outputs per block, 16
// threads per output; thread s sums blocks s, s + 16, s + 32, ... with four
// independent accumulators (their loads in flight together), and the 16
// segment sums of an output are added in order through LDS.
constexpr int kRedOut = 16, kRedSeg = 16;

__global__ void __launch_bounds__(256) wgrad_reduce_kernel(const float* __restrict__ part, float* __restrict__ dw,
                                                           float* __restrict__ db, int nblk, int cin, int cout,
                                                           int cpad) {
    __shared__ float seg[kRedSeg][kRedOut];
    const int lo = threadIdx.x % kRedOut, sg = threadIdx.x / kRedOut;
    const int e = blockIdx.x * kRedOut + lo;
    const int nw = cout * 9 * cin;
    const bool valid = e < nw + cout;
    const float* src = part;
    size_t stride = 0;
    if (e < nw) {
        const int o = e / (9 * cin), r = e - o * 9 * cin;
        const int tap = r / cin, i = r - tap * cin;
        stride = (size_t)cout * 9 * cpad;
        src = part + ((size_t)o * 9 + tap) * cpad + i;
    } else if (valid) {
        stride = (size_t)cout;
        src = part + (size_t)nblk * cout * 9 * cpad + (e - nw);
    }
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    if (valid) {
        int b = sg;
        for (; b + 3 * kRedSeg < nblk; b += 4 * kRedSeg) {
            a0 += src[(size_t)b * stride];
            a1 += src[(size_t)(b + kRedSeg) * stride];
            a2 += src[(size_t)(b + 2 * kRedSeg) * stride];
            a3 += src[(size_t)(b + 3 * kRedSeg) * stride];
        }
        for (; b < nblk; b += kRedSeg) a0 += src[(size_t)b * stride];
    }
    seg[sg][lo] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (sg == 0 && valid) {
        float t = 0.f;
#pragma unroll
        for (int k = 0; k < kRedSeg; ++k) t += seg[k][lo];
        if (e < nw)
            dw[e] = t;
        else
            db[e - nw] = t;
    }
}

bool conv_shape_ok(int n, int H, int W, int cin, int cout, int dil) {
    if (n < 1 || H < 1 || W < 1 || H > 16384 || W > 16384 || n > 65535) return false;
    if (dil < 1 || dil > kMaxDil) return false;
    return (cin == 3 || cin == 32) && cout == 32;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// conv32_fwd_kernel and the 32-channel weight gradient read x (and mask, dy)
// in 16-byte pieces; unaligned tensors and SFF_CONV_IM2COL=1 (testing and
// timing) take the element-wise kernels (the im2col forward, element-wise
// staging of the gradient tiles), which give the same results.
bool staged_conv_enabled() {
    const char* e = std::getenv("SFF_CONV_IM2COL");
    return !(e && std::strcmp(e, "1") == 0);
}

// ------------------------------------------------------- fused 4 layers --
// The whole network (3 -> 32 -> 32 -> 32 -> 32, ReLU after the first three,
// dilation 1) for one kFusedY x kFusedX output tile per block, the layers'
// activations kept in LDS: layer l is computed on the tile grown by 3 - l
// pixels on every side (its inputs' halo), from the LDS region the layer
// before it left there; only the three-channel input is read from and the
// 32-channel output written to HBM.  Positions outside the image are stored
// as zeros (the zero padding the next layer reads), every layer's output is
// rounded to BF16 as the per-layer kernels store it, and each output element
// is the same MFMAs in the same order on the same values as conv3_fwd_kernel
// and conv32_fwd_kernel, so the results are identical (tested).
// Tiles are 26 wide so that every layer's region is at most two 16-pixel
// groups wide (32, 30, 28 and 26 pixels: 15 % of the computed groups fall
// outside a region, against 22 % for 64-wide tiles) and 24 tall, the most that
// fits 150 KB of LDS with that width (four KITTI-size images: 0.35 ms with
// 64 x 8 tiles, 0.31 with 58 x 10, 0.28 with 42 x 15, 0.27 with 26 x 24).
constexpr int kFusedX = 26, kFusedY = 24;
constexpr int kFIn[2] = {kFusedY + 8, kFusedX + 8};   // input region (3 channels, packed)
constexpr int kF1[2] = {kFusedY + 6, kFusedX + 6};    // layer-1 output (and layer 3's, in place later)
constexpr int kF2[2] = {kFusedY + 4, kFusedX + 4};    // layer-2 output
constexpr int kFPx = 40;                              // bf16 per staged pixel (32 used): 80-byte stride

// This lane's biases: output channels 16 t + 4 (l / 16) + e (zero without bias).
__device__ __forceinline__ void fused_bias(const float* __restrict__ bias, float (&bz)[2][4]) {
    const int g = (threadIdx.x & 63) >> 4;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) bz[t][e] = bias ? bias[t * 16 + 4 * g + e] : 0.f;
}

// Round acc + bias, ReLU, to BF16 pairs for output channels 16 t + 4 g .. + 3.
__device__ __forceinline__ uint2 fused_pack(const v4f& acc, const float (&bz)[4], bool relu) {
    uint32_t packed[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        float v0 = acc[2 * h] + bz[2 * h];
        float v1 = acc[2 * h + 1] + bz[2 * h + 1];
        if (relu) {
            v0 = fmaxf(v0, 0.f);
            v1 = fmaxf(v1, 0.f);
        }
        packed[h] = f2bf2(v0, v1);
    }
    return make_uint2(packed[0], packed[1]);
}

// The 18 weight fragments of a 32 -> 32 layer for this lane: output channel
// 16 t + l % 16, tap, input channels 8 (l / 16) .. + 7.
__device__ __forceinline__ void fused_weights(const bf16_t* __restrict__ w, v8bf (&a)[2][9]) {
    const int lane = threadIdx.x & 63, ln = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
            a[t][tap] = *reinterpret_cast<const v8bf*>(w + ((size_t)(t * 16 + ln) * 9 + tap) * 32 + 8 * g);
}

// One 32 -> 32 layer from LDS region `in` (OH + 2) x (OW + 2) to region `out`
// OH x OW (or, for the last layer, to y), the region's pixel (0, 0) at image
// (oy, ox).  Work items are (row, 16-pixel group), dealt to the 8 waves, two
// at a time per wave (four independent accumulator chains in flight).
template <int OH, int OW, bool LAST>
__device__ __forceinline__ void fused_layer32(const bf16_t* in, bf16_t* out, const v8bf (&a)[2][9],
                                              const float (&bz)[2][4], bool relu, int oy, int ox,
                                              int H, int W, bf16_t* __restrict__ y, size_t img) {
    constexpr int IW = OW + 2, NG = (OW + 15) / 16, NI = OH * NG;
    typedef const v8bf __attribute__((address_space(3)))* lds_v8;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ln = lane & 15, g = lane >> 4;
    for (int i0 = wv; i0 < NI; i0 += 16) {
        int r[2], p[2];
        lds_v8 src[2];
        v4f acc[2][2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int item = min(i0 + 8 * h, NI - 1);  // a missing second item repeats the last
            r[h] = item / NG;
            p[h] = (item - r[h] * NG) * 16 + ln;
            const int pr = min(p[h], OW - 1);  // lanes past the row read a valid pixel
            // 32-bit LDS addresses; the taps are constant offsets from the lane's first one
            src[h] = (lds_v8)((const __attribute__((address_space(3))) bf16_t*)in + (r[h] * IW + pr) * kFPx + 8 * g);
            acc[h][0] = v4f{0.f, 0.f, 0.f, 0.f};
            acc[h][1] = v4f{0.f, 0.f, 0.f, 0.f};
        }
        // the B operands of tap t + kAhead are read from LDS while tap t's
        // products run (a ring of kAhead + 1 taps), so the LDS latency is not
        // waited on at every tap
        constexpr int kAhead = 3;
        v8bf bv[kAhead + 1][2];
        auto read_tap = [&](int tap, v8bf (&b)[2]) {
            const int ky = tap / 3, kx = tap - 3 * ky;
#pragma unroll
            for (int h = 0; h < 2; ++h) b[h] = src[h][(ky * IW + kx) * kFPx / 8];
        };
#pragma unroll
        for (int tap = 0; tap < kAhead; ++tap) read_tap(tap, bv[tap]);
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            if (tap + kAhead < 9) read_tap(tap + kAhead, bv[(tap + kAhead) % (kAhead + 1)]);
            __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the products
            const v8bf (&b)[2] = bv[tap % (kAhead + 1)];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                acc[h][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][tap], b[h], acc[h][0], 0, 0, 0);
                acc[h][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][tap], b[h], acc[h][1], 0, 0, 0);
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (p[h] >= OW || (h == 1 && i0 + 8 >= NI)) continue;
            const int iy = oy + r[h], ix = ox + p[h];
            const bool inside = iy >= 0 && iy < H && ix >= 0 && ix < W;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const uint2 v = inside ? fused_pack(acc[h][t], bz[t], relu) : make_uint2(0u, 0u);
                if constexpr (LAST) {
                    if (inside) *reinterpret_cast<uint2*>(y + (img + (size_t)iy * W + ix) * 32 + t * 16 + 4 * g) = v;
                } else {
                    *reinterpret_cast<uint2*>(out + (r[h] * OW + p[h]) * kFPx + t * 16 + 4 * g) = v;
                }
            }
        }
    }
}

__global__ void __launch_bounds__(512) featnet_fwd_kernel(const bf16_t* __restrict__ x,
                                                          const bf16_t* __restrict__ w0, const float* __restrict__ b0,
                                                          const bf16_t* __restrict__ w1, const float* __restrict__ b1,
                                                          const bf16_t* __restrict__ w2, const float* __restrict__ b2,
                                                          const bf16_t* __restrict__ w3, const float* __restrict__ b3,
                                                          bf16_t* __restrict__ y, int H, int W) {
    __shared__ __align__(16) bf16_t xin[kFIn[0] * kFIn[1] * 3];
    __shared__ __align__(16) bf16_t bufA[kF1[0] * kF1[1] * kFPx];
    __shared__ __align__(16) bf16_t bufB[kF2[0] * kF2[1] * kFPx];
    const int x0 = blockIdx.x * kFusedX, y0 = blockIdx.y * kFusedY, n = blockIdx.z;
    const size_t img = (size_t)n * H * W;
    v8bf wa[2][9];
    float bz0[2][4], bz[2][4];
    fused_weights(w1, wa);  // layer 2's, in flight during the staging and layer 1
    fused_bias(b0, bz0);
    fused_bias(b1, bz);
    // input region: image rows y0 - 4 .., columns x0 - 4 .., zero outside
    for (int e = threadIdx.x; e < kFIn[0] * kFIn[1] * 3; e += 512) {
        const int px = e / 3, ci = e - 3 * px, r = px / kFIn[1], c = px - r * kFIn[1];
        const int iy = y0 - 4 + r, ix = x0 - 4 + c;
        xin[e] = (iy >= 0 && iy < H && ix >= 0 && ix < W) ? x[(img + (size_t)iy * W + ix) * 3 + ci] : (bf16_t)0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ln = lane & 15, g = lane >> 4;
    // layer 1 (3 -> 32, K = 27 in one MFMA step) into bufA: kF1 region at image (y0 - 3, x0 - 3)
    {
        v8bf a[2];
        int koff[8];  // offset of K value 8 g + e from the lane's pixel in xin (-1: zero padding)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 8 * g + e;
#pragma unroll
            for (int t = 0; t < 2; ++t)
                a[t][e] = __builtin_bit_cast(__bf16, k < 27 ? w0[(size_t)(t * 16 + ln) * 27 + k] : (bf16_t)0);
            const int tap = k / 3, ci = k - 3 * tap, ky = tap / 3, kx = tap - 3 * ky;
            koff[e] = k < 27 ? (ky * kFIn[1] + kx) * 3 + ci : -1;
        }
        constexpr int NG = (kF1[1] + 15) / 16;
        for (int item = wv; item < kF1[0] * NG; item += 8) {
            const int r = item / NG, p = (item - r * NG) * 16 + ln;
            const int pr = min(p, kF1[1] - 1);
            const bf16_t* src = xin + (r * kFIn[1] + pr) * 3;
            v8bf bv;
#pragma unroll
            for (int e = 0; e < 8; ++e) bv[e] = __builtin_bit_cast(__bf16, koff[e] >= 0 ? src[koff[e]] : (bf16_t)0);
            v4f acc[2];
#pragma unroll
            for (int t = 0; t < 2; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], bv, v4f{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            if (p >= kF1[1]) continue;
            const int iy = y0 - 3 + r, ix = x0 - 3 + p;
            const bool inside = iy >= 0 && iy < H && ix >= 0 && ix < W;
#pragma unroll
            for (int t = 0; t < 2; ++t)
                *reinterpret_cast<uint2*>(bufA + (r * kF1[1] + p) * kFPx + t * 16 + 4 * g) =
                    inside ? fused_pack(acc[t], bz0[t], true) : make_uint2(0u, 0u);
        }
    }
    __syncthreads();
    // the next layer's weight fragments are loaded while this one computes
    v8bf wb[2][9];
    float bz2[2][4];
    fused_weights(w2, wb);
    fused_bias(b2, bz2);
    fused_layer32<kF2[0], kF2[1], false>(bufA, bufB, wa, bz, true, y0 - 2, x0 - 2, H, W, nullptr, img);
    __syncthreads();
    fused_weights(w3, wa);
    fused_bias(b3, bz);
    fused_layer32<kFusedY + 2, kFusedX + 2, false>(bufB, bufA, wb, bz2, true, y0 - 1, x0 - 1, H, W, nullptr, img);
    __syncthreads();
    fused_layer32<kFusedY, kFusedX, true>(bufA, nullptr, wa, bz, false, y0, x0, H, W, y, img);
}

bool use_conv32(const void* x, const void* mask) {
    if ((reinterpret_cast<uintptr_t>(x) & 15) != 0 || (reinterpret_cast<uintptr_t>(mask) & 15) != 0) return false;
    return staged_conv_enabled();
}

size_t wgrad_part_bytes(int n, int H, int W, int cin, int cout) {
    const size_t nblk = (size_t)((W + kTilePx - 1) / kTilePx) * ((H + kWgRows - 1) / kWgRows) * n;
    const int cpad = (cin + 15) / 16 * 16;
    return align256(nblk * ((size_t)cout * 9 * cpad + cout) * sizeof(float));
}

}  // namespace
}  // namespace sff

using namespace sff;

extern "C" sff_status sff_conv3x3_bf16_fwd(int32_t n, int32_t H, int32_t W, int32_t cin,
                                           int32_t cout, int32_t dil, int32_t relu,
                                           const uint16_t* x, const uint16_t* w, const float* bias,
                                           uint16_t* y, void* stream) {
    if (!conv_shape_ok(n, H, W, cin, cout, dil) || !x || !w || !y) return SFF_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(y) & 7) != 0) return SFF_ERR_INVALID_ARG;
    const dim3 grid((W + kTilePx - 1) / kTilePx, H, n);
    hipStream_t st = as_stream(stream);
    if (cin == 3 && staged_conv_enabled())
        hipLaunchKernelGGL(conv3_fwd_kernel, dim3((W + kTile32 - 1) / kTile32, (H + kRows32 - 1) / kRows32, n),
                           dim3(256), 0, st, x, w, bias, y, H, W, dil, relu);
    else if (cin == 3)
        hipLaunchKernelGGL((conv_fwd_kernel<3, 32>), grid, dim3(256), 0, st, x, nullptr, w, bias, y,
                           H, W, dil, relu);
    else if (use_conv32(x, nullptr))
        hipLaunchKernelGGL(conv32_fwd_kernel, dim3((W + kTile32 - 1) / kTile32, (H + kRows32 - 1) / kRows32, n), dim3(256), 0, st, x,
                           nullptr, w, bias, y, H, W, dil, relu);
    else
        hipLaunchKernelGGL((conv_fwd_kernel<32, 32>), grid, dim3(256), 0, st, x, nullptr, w, bias,
                           y, H, W, dil, relu);
    return launch_status();
}

extern "C" size_t sff_conv3x3_bf16_bwd_workspace_bytes(int32_t n, int32_t H, int32_t W,
                                                       int32_t cin, int32_t cout) {
    if (!conv_shape_ok(n, H, W, cin, cout, 1)) return 0;
    return align256((size_t)cin * 9 * cout * sizeof(uint16_t)) +
           wgrad_part_bytes(n, H, W, cin, cout);
}

extern "C" sff_status sff_conv3x3_bf16_dgrad(int32_t n, int32_t H, int32_t W, int32_t cin,
                                             int32_t cout, int32_t dil, const uint16_t* dy,
                                             const uint16_t* relu_out, const uint16_t* w,
                                             uint16_t* dx, void* workspace,
                                             size_t workspace_bytes, void* stream) {
    if (!conv_shape_ok(n, H, W, cin, cout, dil) || cin != 32 || !dy || !w || !dx)
        return SFF_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(dx) & 7) != 0) return SFF_ERR_INVALID_ARG;
    const size_t need = align256((size_t)cin * 9 * cout * sizeof(uint16_t));
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return SFF_ERR_WORKSPACE;
    hipStream_t st = as_stream(stream);
    uint16_t* wt = static_cast<uint16_t*>(workspace);
    hipLaunchKernelGGL(flip_weights_kernel, dim3((cin * 9 * cout + 255) / 256), dim3(256), 0, st, w,
                       wt, cin, cout);
    if (use_conv32(dy, relu_out))
        hipLaunchKernelGGL(conv32_fwd_kernel, dim3((W + kTile32 - 1) / kTile32, (H + kRows32 - 1) / kRows32, n), dim3(256), 0, st, dy,
                           relu_out, wt, nullptr, dx, H, W, dil, 0);
    else
        hipLaunchKernelGGL((conv_fwd_kernel<32, 32>), dim3((W + kTilePx - 1) / kTilePx, H, n), dim3(256),
                           0, st, dy, relu_out, wt, nullptr, dx, H, W, dil, 0);
    return launch_status();
}

extern "C" sff_status sff_conv3x3_bf16_wgrad(int32_t n, int32_t H, int32_t W, int32_t cin,
                                             int32_t cout, int32_t dil, const uint16_t* x,
                                             const uint16_t* dy, const uint16_t* relu_out,
                                             float* dw, float* db, void* workspace,
                                             size_t workspace_bytes, void* stream) {
    if (!conv_shape_ok(n, H, W, cin, cout, dil) || !x || !dy || !dw || !db)
        return SFF_ERR_INVALID_ARG;
    const size_t off = align256((size_t)cin * 9 * cout * sizeof(uint16_t));
    const size_t need = off + wgrad_part_bytes(n, H, W, cin, cout);
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return SFF_ERR_WORKSPACE;
    hipStream_t st = as_stream(stream);
    float* part = reinterpret_cast<float*>(static_cast<uint8_t*>(workspace) + off);
    const dim3 grid((W + kTilePx - 1) / kTilePx, (H + kWgRows - 1) / kWgRows, n);
    const int nblk = grid.x * grid.y * grid.z;
    if (cin == 3)
        hipLaunchKernelGGL((conv_wgrad_kernel<3, 32>), grid, dim3(256), 0, st, x, dy, relu_out, part,
                           H, W, dil, 0);
    else
        hipLaunchKernelGGL((conv_wgrad_kernel<32, 32>), grid, dim3(256), 0, st, x, dy, relu_out,
                           part, H, W, dil, use_conv32(x, relu_out) && use_conv32(dy, nullptr) ? 1 : 0);
    const int cpad = (cin + 15) / 16 * 16;
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((cout * 9 * cin + cout + kRedOut - 1) / kRedOut), dim3(256), 0,
                       st, part, dw, db, nblk, cin, cout, cpad);
    return launch_status();
}

extern "C" sff_status sff_featnet_fwd_bf16(int32_t n, int32_t H, int32_t W, int32_t dil,
                                           const uint16_t* x, const uint16_t* w0, const float* b0,
                                           const uint16_t* w1, const float* b1, const uint16_t* w2,
                                           const float* b2, const uint16_t* w3, const float* b3,
                                           uint16_t* y, void* stream) {
    if (!conv_shape_ok(n, H, W, 3, 32, dil) || !x || !w0 || !w1 || !w2 || !w3 || !y)
        return SFF_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(y) & 7) != 0 || (reinterpret_cast<uintptr_t>(w1) & 15) != 0 ||
        (reinterpret_cast<uintptr_t>(w2) & 15) != 0 || (reinterpret_cast<uintptr_t>(w3) & 15) != 0)
        return SFF_ERR_INVALID_ARG;
    if (dil != 1) return SFF_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(featnet_fwd_kernel, dim3((W + kFusedX - 1) / kFusedX, (H + kFusedY - 1) / kFusedY, n),
                       dim3(512), 0, as_stream(stream), x, w0, b0, w1, b1, w2, b2, w3, b3, y, H, W);
    return launch_status();
}
