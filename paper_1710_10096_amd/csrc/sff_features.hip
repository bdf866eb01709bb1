// WHT feature vectors and scale simulation (SceneFlowFields, Section 3.1:
// "Initialization" for the WHT features, "Multi-Scale Propagation" for the
// smoothing by area-based downsampling and Lanczos upsampling).
//
// Level k, pyramid factor n = 2^k:
//   A  = rounded n x n block means (replicated border)          [Hk][Wk][C] u8
//   h  = horizontal Lanczos-3 pass of A to full width, rounded  [Hk][W][C]  i16
//   S  = vertical Lanczos-3 pass of h to full height, clamped   [H][W][C]   u8
//   desc(q, c) = 4x4 lowest-sequency block of the 2-D WHT of the 8x8 patch of S
//                sampled every n-th pixel at offsets -3..+4 around q.
// The four lowest-sequency length-8 Walsh functions are constant on pixel
// pairs, so the block equals the length-4 sequency-ordered WHT of the 4x4
// matrix of 2x2-bin sums; the kernel computes it that way (exact integers).
#include <cmath>
#include <cstring>

#include "sff_internal.hpp"

namespace sff {
namespace {

constexpr int kMaxN = 1 << (kMaxLevels - 1);

struct LanczosTable {
    int32_t w[kMaxN][6];
    int32_t base[kMaxN];  // floor((p + 0.5) / n - 0.5) - 2, tap 0 offset of phase p
};

double lanczos3(double t) {
    if (t <= -3.0 || t >= 3.0) return 0.0;
    if (t == 0.0) return 1.0;
    const double pi = 3.14159265358979323846;
    const double a = pi * t, b = pi * t / 3.0;
    return (std::sin(a) / a) * (std::sin(b) / b);
}

void build_table(int n, LanczosTable* T) {
    std::memset(T, 0, sizeof(*T));
    for (int p = 0; p < n; ++p) {
        const double s = (p + 0.5) / n - 0.5;
        const double fl = std::floor(s);
        const double f = s - fl;
        T->base[p] = (int)fl - 2;
        double raw[6], sum = 0.0;
        for (int t = 0; t < 6; ++t) {
            raw[t] = lanczos3(f + 2.0 - t);
            sum += raw[t];
        }
        int32_t tot = 0;
        for (int t = 0; t < 6; ++t) {
            const double q = raw[t] / sum * 16384.0;
            const double r = q < 0 ? -std::floor(-q + 0.5) : std::floor(q + 0.5);
            T->w[p][t] = (int32_t)r;
            tot += T->w[p][t];
        }
        T->w[p][f < 0.5 ? 2 : 3] += 16384 - tot;  // residual to the tap nearest s
    }
}

__device__ __forceinline__ int floor_shift14(int v) { return v >> 14; }  // arithmetic shift

// A: one thread per (img, i, j); loops over channels.
__global__ void area_kernel(const uint8_t* __restrict__ img, uint8_t* __restrict__ A, int H,
                            int W, int C, int n, int Hk, int Wk) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    const int m = blockIdx.z;
    if (j >= Wk) return;
    const uint8_t* src = img + (size_t)m * H * W * C;
    for (int c = 0; c < C; ++c) {
        int s = 0;
        for (int a = 0; a < n; ++a) {
            const int y = min(n * i + a, H - 1);
            for (int b = 0; b < n; ++b) {
                const int x = min(n * j + b, W - 1);
                s += src[((size_t)y * W + x) * C + c];
            }
        }
        const int nn = n * n;
        A[(((size_t)m * Hk + i) * Wk + j) * C + c] = (uint8_t)((s + nn / 2) / nn);
    }
}

// h: one thread per (img, i, x, c).
__global__ void lanczos_h_kernel(const uint8_t* __restrict__ A, int16_t* __restrict__ h, int W,
                                 int C, int n, int Hk, int Wk, LanczosTable T) {
    const int xc = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    const int m = blockIdx.z;
    if (xc >= W * C) return;
    const int x = xc / C, c = xc - x * C;
    const int p = x % n, j = x / n;
    const uint8_t* row = A + ((size_t)m * Hk + i) * Wk * C;
    int acc = 8192;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        const int jj = clampi(j + T.base[p] + t, 0, Wk - 1);
        acc += T.w[p][t] * (int)row[jj * C + c];
    }
    h[(((size_t)m * Hk + i) * W) * C + xc] = (int16_t)floor_shift14(acc);
}

// S: one thread per (img, y, x, c).
__global__ void lanczos_v_kernel(const int16_t* __restrict__ h, uint8_t* __restrict__ S, int H,
                                 int W, int C, int n, int Hk, LanczosTable T) {
    const int xc = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    const int m = blockIdx.z;
    if (xc >= W * C) return;
    const int p = y % n, i = y / n;
    const int16_t* plane = h + (size_t)m * Hk * W * C;
    int acc = 8192;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        const int ii = clampi(i + T.base[p] + t, 0, Hk - 1);
        acc += T.w[p][t] * (int)plane[(size_t)ii * W * C + xc];
    }
    S[((size_t)m * H + y) * W * C + xc] = (uint8_t)clampi(floor_shift14(acc), 0, 255);
}

// 4-point sequency-ordered WHT: rows (1,1,1,1), (1,1,-1,-1), (1,-1,-1,1), (1,-1,1,-1).
__device__ __forceinline__ void wht4(int& x0, int& x1, int& x2, int& x3) {
    const int a = x0 + x1, b = x2 + x3, c = x0 - x1, d = x2 - x3;
    x0 = a + b;
    x1 = a - b;
    x2 = c - d;
    x3 = c + d;
}

// One thread per output pixel (all channels).  Block 64 x 4 pixels.
__global__ void __launch_bounds__(256) wht_kernel(const uint8_t* __restrict__ S,
                                                  int16_t* __restrict__ desc, int H, int W, int C,
                                                  int n) {
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int m = blockIdx.z;
    if (x >= W || y >= H) return;
    const uint8_t* src = S + (size_t)m * H * W * C;
    int rows[8], cols[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        rows[t] = clampi(y + n * (t - 3), 0, H - 1) * W;
        cols[t] = clampi(x + n * (t - 3), 0, W - 1);
    }
    int16_t* out = desc + (((size_t)m * H + y) * W + x) * C * 16;
    for (int c = 0; c < C; ++c) {
        int B[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int r0 = rows[2 * a], r1 = rows[2 * a + 1];
                const int c0 = cols[2 * b], c1 = cols[2 * b + 1];
                B[a][b] = (int)src[(size_t)(r0 + c0) * C + c] + (int)src[(size_t)(r0 + c1) * C + c] +
                          (int)src[(size_t)(r1 + c0) * C + c] + (int)src[(size_t)(r1 + c1) * C + c];
            }
#pragma unroll
        for (int a = 0; a < 4; ++a) wht4(B[a][0], B[a][1], B[a][2], B[a][3]);
#pragma unroll
        for (int b = 0; b < 4; ++b) wht4(B[0][b], B[1][b], B[2][b], B[3][b]);
        uint32_t w[8];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            w[2 * a] = (uint32_t)(uint16_t)(int16_t)B[a][0] | ((uint32_t)(uint16_t)(int16_t)B[a][1] << 16);
            w[2 * a + 1] = (uint32_t)(uint16_t)(int16_t)B[a][2] | ((uint32_t)(uint16_t)(int16_t)B[a][3] << 16);
        }
        uint4* o = reinterpret_cast<uint4*>(out + c * 16);
        o[0] = make_uint4(w[0], w[1], w[2], w[3]);
        o[1] = make_uint4(w[4], w[5], w[6], w[7]);
    }
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct WsLayout {
    size_t a_off, h_off, s_off, total;
};

WsLayout ws_layout(const sff_params& p, int nimg, int level) {
    WsLayout L{0, 0, 0, 0};
    if (level == 0) return L;
    const LevelGeom g = level_geom(p, level);
    const size_t C = (size_t)p.C;
    L.a_off = 0;
    L.h_off = align256((size_t)nimg * g.Hk * g.Wk * C);
    L.s_off = L.h_off + align256((size_t)nimg * g.Hk * p.W * C * sizeof(int16_t));
    L.total = L.s_off + align256((size_t)nimg * p.H * p.W * C);
    return L;
}

}  // namespace
}  // namespace sff

using namespace sff;

extern "C" sff_status sff_lanczos_q14(int32_t n, int32_t* table) {
    if (!table || n < 2 || n > kMaxN) return SFF_ERR_INVALID_ARG;
    LanczosTable T;
    build_table(n, &T);
    for (int p = 0; p < n; ++p)
        for (int t = 0; t < 6; ++t) table[p * 6 + t] = T.w[p][t];
    return SFF_OK;
}

extern "C" size_t sff_wht_workspace_bytes(const sff_params* p, int32_t nimg, int32_t level) {
    if (!params_ok(p) || nimg < 1 || level < 0 || level >= p->levels) return 0;
    return ws_layout(*p, nimg, level).total;
}

extern "C" sff_status sff_wht_features(const sff_params* p, int32_t nimg, int32_t level,
                                       const uint8_t* img, int16_t* desc, void* workspace,
                                       size_t workspace_bytes, void* stream) {
    if (!params_ok(p) || nimg < 1 || nimg > 65535 || level < 0 || level >= p->levels || !img ||
        !desc)
        return SFF_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(desc) & 15) != 0) return SFF_ERR_INVALID_ARG;
    const WsLayout L = ws_layout(*p, nimg, level);
    if (level > 0 && (!workspace || workspace_bytes < L.total)) return SFF_ERR_WORKSPACE;
    hipStream_t st = as_stream(stream);
    const int H = p->H, W = p->W, C = p->C;
    const LevelGeom g = level_geom(*p, level);
    const uint8_t* src = img;
    if (level > 0) {
        uint8_t* ws = static_cast<uint8_t*>(workspace);
        uint8_t* A = ws + L.a_off;
        int16_t* h = reinterpret_cast<int16_t*>(ws + L.h_off);
        uint8_t* S = ws + L.s_off;
        LanczosTable T;
        build_table(g.n, &T);
        hipLaunchKernelGGL(area_kernel, dim3((g.Wk + 63) / 64, g.Hk, nimg), dim3(64), 0, st, img,
                           A, H, W, C, g.n, g.Hk, g.Wk);
        hipLaunchKernelGGL(lanczos_h_kernel, dim3((W * C + 255) / 256, g.Hk, nimg), dim3(256), 0,
                           st, A, h, W, C, g.n, g.Hk, g.Wk, T);
        hipLaunchKernelGGL(lanczos_v_kernel, dim3((W * C + 255) / 256, H, nimg), dim3(256), 0, st,
                           h, S, H, W, C, g.n, g.Hk, T);
        src = S;
    }
    hipLaunchKernelGGL(wht_kernel, dim3((W + 63) / 64, (H + 3) / 4, nimg), dim3(64, 4), 0, st, src,
                       desc, H, W, C, g.n);
    return launch_status();
}
