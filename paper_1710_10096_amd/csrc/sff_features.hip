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
#include <mutex>

#include "sff_device.hpp"

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
        const int nn = n * n;  // a power of two: the rounded mean by a shift
        A[(((size_t)m * Hk + i) * Wk + j) * C + c] = (uint8_t)((s + nn / 2) >> (2 * __builtin_ctz(n)));
    }
}

// Both Lanczos passes in one kernel.  Block = 256 consecutive (x, c) columns
// of kBandRows output rows of one image: the horizontal pass is computed for
// the block-mean rows the band needs (at most kBandRows / n + 7) into LDS, then
// each thread forms its column's vertical pass.  Both passes round exactly as
// in the separate definition: h = (sum + 8192) >> 14 unclamped, then
// S = clamp((sum + 8192) >> 14, 0, 255).
constexpr int kBandRows = 32;
constexpr int kBandH = kBandRows + 7;  // h rows for n = 1 (the largest count)

__global__ void __launch_bounds__(256) lanczos_hv_kernel(const uint8_t* __restrict__ A,
                                                         uint8_t* __restrict__ S, int H, int W,
                                                         int C, int n, int Hk, int Wk,
                                                         LanczosTable T) {
    __shared__ int hb[kBandH][256];
    const int xc = blockIdx.x * 256 + threadIdx.x;
    const int y0 = blockIdx.y * kBandRows, m = blockIdx.z;
    const int y1 = min(y0 + kBandRows, H);
    // vertical taps of rows y0..y1-1 reach block-mean rows y/n - 3 .. y/n + 3
    const int ln = __builtin_ctz(n);  // n is a power of two: phases and blocks by masks and shifts
    const int ilo = (y0 >> ln) - 3, ihi = ((y1 - 1) >> ln) + 3;
    const bool live = xc < W * C;
    const int x = live ? xc / C : 0, c = xc - x * C;
    const int ph = x & (n - 1), jh = (x >> ln) + T.base[ph];
    const uint8_t* Am = A + (size_t)m * Hk * Wk * C;
    for (int r = 0; r <= ihi - ilo; ++r) {
        const uint8_t* row = Am + (size_t)clampi(ilo + r, 0, Hk - 1) * Wk * C;
        int acc = 8192;
#pragma unroll
        for (int t = 0; t < 6; ++t) acc += T.w[ph][t] * (int)row[clampi(jh + t, 0, Wk - 1) * C + c];
        hb[r][threadIdx.x] = floor_shift14(acc);
    }
    if (!live) return;  // no barrier follows: each thread reads only its own column
    for (int y = y0; y < y1; ++y) {
        const int pv = y & (n - 1), ib = (y >> ln) + T.base[pv] - ilo;
        int acc = 8192;
#pragma unroll
        for (int t = 0; t < 6; ++t) acc += T.w[pv][t] * hb[ib + t][threadIdx.x];
        S[((size_t)m * H + y) * W * C + xc] = (uint8_t)clampi(floor_shift14(acc), 0, 255);
    }
}

// 4-point sequency-ordered WHT: rows (1,1,1,1), (1,1,-1,-1), (1,-1,-1,1), (1,-1,1,-1).
__device__ __forceinline__ void wht4(int& x0, int& x1, int& x2, int& x3) {
    const int a = x0 + x1, b = x2 + x3, c = x0 - x1, d = x2 - x3;
    x0 = a + b;
    x1 = a - b;
    x2 = c - d;
    x3 = c + d;
}

// Block = 64 x 4 output pixels of one image.  The source region the tile's
// patches sample, rows y0 - 3n .. y0 + 3 + 4n and columns x0 - 3n .. x0 + 63 + 4n
// (replicated border), is staged in LDS with coalesced loads; each thread
// forms its pixel's bin sums from LDS; the coefficients are staged in LDS
// again so every wave stores its row of 64 descriptors as one contiguous run.
constexpr int kTW = 64;
// Output rows per block: 16 for n <= 4, so that the 7n-pixel halo of the
// staged source region is shared by more rows; 4 beyond (the region would not
// fit in LDS).
template <int n>
constexpr int wht_rows() { return n <= 4 ? 16 : 4; }
inline int wht_rows_rt(int n) { return n <= 4 ? 16 : 4; }

// Order LDS accesses of different lanes of one wave.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// n (the pyramid factor) is a template parameter so that every LDS offset
// of the bin sums is an immediate.
template <int C, int n>
__global__ void __launch_bounds__(256) wht_kernel(const uint8_t* __restrict__ S,
                                                  int16_t* __restrict__ desc, int H, int W) {
    constexpr int TH = wht_rows<n>();
    extern __shared__ uint8_t smem[];
    const int RW = kTW + 7 * n, RH = TH + 7 * n;
    const int wv = wave_id(), ln = threadIdx.x & 63;
    uint8_t* reg = smem;  // [RH][RW][C]
    // this wave's row of 64 descriptors [kTW][16C]
    int16_t* outw = reinterpret_cast<int16_t*>(smem + ((RH * RW * C + 15) & ~15)) + wv * kTW * 16 * C;
    const int x0 = blockIdx.x * kTW, y0 = blockIdx.y * TH, m = blockIdx.z;
    const uint8_t* src = S + (size_t)m * H * W * C;
    const int gx0 = x0 - 3 * n, gy0 = y0 - 3 * n;
    const int rowb = RW * C;
    // wave w stages region rows w, w + 4, ...; lanes walk the row's bytes
    // (only divisions by the compile-time channel count)
    {
        const bool inner = gx0 >= 0 && gx0 + RW <= W;  // no column clamping (block-uniform)
        for (int ry = wv; ry < RH; ry += 4) {
            const uint8_t* srow = src + (size_t)clampi(gy0 + ry, 0, H - 1) * W * C;
            uint8_t* drow = reg + ry * rowb;
            if (inner) {
                const uint8_t* seg = srow + gx0 * C;
                for (int rr = ln; rr < rowb; rr += 64) drow[rr] = seg[rr];
            } else {
                for (int rr = ln; rr < rowb; rr += 64) {
                    const int rx = rr / C, c = rr - rx * C;
                    drow[rr] = srow[clampi(gx0 + rx, 0, W - 1) * C + c];
                }
            }
        }
    }
    __syncthreads();
    constexpr int P = 2 * C, RS = 2 * kRecC<C>;
    const int tx = ln;
    const int npx = min(kTW, W - x0);
    int16_t* o = outw + tx * 16 * C;
    // wave w computes rows w, w + 4, ...: one descriptor per lane, staged in
    // the wave's LDS row so that the wave stores a contiguous row
    for (int ty = wv; ty < TH; ty += 4) {
        const int y = y0 + ty;
        if (y >= H) break;  // whole wave
#pragma unroll
        for (int c = 0; c < C; ++c) {
            int B[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const uint8_t* r0 = reg + ((ty + 2 * a * n) * RW + tx) * C + c;
                const uint8_t* r1 = r0 + n * RW * C;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int c0 = 2 * b * n * C, c1 = c0 + n * C;
                    B[a][b] = (int)r0[c0] + (int)r0[c1] + (int)r1[c0] + (int)r1[c1];
                }
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) wht4(B[a][0], B[a][1], B[a][2], B[a][3]);
#pragma unroll
            for (int b = 0; b < 4; ++b) wht4(B[0][b], B[1][b], B[2][b], B[3][b]);
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) o[c * 16 + a * 4 + b] = (int16_t)B[a][b];
        }
        wave_lds_sync();
        // 64 descriptors, 2 C 16-byte chunks each, at a record stride of 2 Cp
        // chunks (padding chunks are not written)
        const int chunks = npx * P;
        const uint4* srow = reinterpret_cast<const uint4*>(outw);
        uint4* drow = reinterpret_cast<uint4*>(desc) + (((size_t)m * H + y) * W + x0) * RS;
        for (int k = tx; k < chunks; k += 64) {
            const int px = k / P;
            drow[px * RS + (k - px * P)] = srow[k];
        }
        wave_lds_sync();
    }
}

template <int C>
void launch_wht(int n, dim3 grid, size_t smem, hipStream_t st, const uint8_t* src, int16_t* desc,
                int H, int W) {
    switch (n) {
        case 1: hipLaunchKernelGGL((wht_kernel<C, 1>), grid, dim3(256), smem, st, src, desc, H, W); break;
        case 2: hipLaunchKernelGGL((wht_kernel<C, 2>), grid, dim3(256), smem, st, src, desc, H, W); break;
        case 4: hipLaunchKernelGGL((wht_kernel<C, 4>), grid, dim3(256), smem, st, src, desc, H, W); break;
        case 8: hipLaunchKernelGGL((wht_kernel<C, 8>), grid, dim3(256), smem, st, src, desc, H, W); break;
        default: hipLaunchKernelGGL((wht_kernel<C, 16>), grid, dim3(256), smem, st, src, desc, H, W); break;
    }
}

inline size_t wht_smem(int n, int C) {
    const int RW = kTW + 7 * n, RH = wht_rows_rt(n) + 7 * n;
    return ((size_t)(RH * RW * C + 15) & ~(size_t)15) + (size_t)4 * kTW * 16 * C * sizeof(int16_t);
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct WsLayout {
    size_t a_off, s_off, total;
};

WsLayout ws_layout(const sff_params& p, int nimg, int level) {
    WsLayout L{0, 0, 0};
    if (level == 0) return L;
    const LevelGeom g = level_geom(p, level);
    const size_t C = (size_t)p.C;
    L.a_off = 0;
    L.s_off = align256((size_t)nimg * g.Hk * g.Wk * C);
    L.total = L.s_off + align256((size_t)nimg * p.H * p.W * C);
    return L;
}

void launch_smooth(const sff_params& p, int nimg, int level, const uint8_t* img, uint8_t* A,
                   uint8_t* S, hipStream_t st) {
    const int H = p.H, W = p.W, C = p.C;
    const LevelGeom g = level_geom(p, level);
    LanczosTable T;
    build_table(g.n, &T);
    hipLaunchKernelGGL(area_kernel, dim3((g.Wk + 63) / 64, g.Hk, nimg), dim3(64), 0, st, img, A, H, W,
                       C, g.n, g.Hk, g.Wk);
    hipLaunchKernelGGL(lanczos_hv_kernel, dim3((W * C + 255) / 256, (H + kBandRows - 1) / kBandRows, nimg),
                       dim3(256), 0, st, A, S, H, W, C, g.n, g.Hk, g.Wk, T);
}

// Bin-sum planes (layout in BinGeom), by tiles: a block takes the entries of
// entry rows r0 .. r0 + R - 1 and entry columns q0 .. q0 + Q - 1 of every plane.
// It first forms in LDS the bins of the extended rows those entries span,
// (R + 3) P of them, over the tile's kQP = Q P extended columns (each bin the
// 2x2 sum of samples n apart, clamped to the image), then writes the entries
// as the contiguous runs they are in memory (plane, row r: Q entries), 8 bytes
// per lane: consecutive lanes write consecutive words, so the stores are whole
// lines instead of the 2-byte pieces of every entry's four slots.
constexpr int kBinTileBins = 4864;  // bins staged per block: (R + 3) P kQP
__host__ __device__ constexpr int bin_tile_qp(int P) { return P * P >= 256 ? P : 256 / P; }
__host__ __device__ constexpr int bin_tile_rows(int P) { return kBinTileBins / (P * bin_tile_qp(P)) - 3; }

template <int C>
__global__ void __launch_bounds__(256) bins_tile_kernel(const uint8_t* __restrict__ S,
                                                        uint16_t* __restrict__ bins, int H, int W,
                                                        int n, int sh, int Hq, int Wq) {
    __shared__ uint16_t lb[kBinTileBins * C];
    const int P = 1 << sh, QP = bin_tile_qp(P), R = bin_tile_rows(P), Q = QP / P;
    const int lqp = __builtin_ctz(QP);  // QP is a power of two
    const int q0 = blockIdx.x * Q, r0 = blockIdx.y * R, m = blockIdx.z;
    const uint8_t* src = S + (size_t)m * H * W * C;
    // bins of extended rows r0 P .. (r0 + R + 3) P - 1, columns q0 P .. q0 P + QP - 1
    const int nb = (R + 3) * P * QP;
#pragma unroll 4
    for (int b = threadIdx.x; b < nb; b += 256) {
        const int ly = b >> lqp, lx = b & (QP - 1);
        const int X0 = q0 * P + lx - 3 * n, Y0 = r0 * P + ly - 3 * n;
        const int x0 = clampi(X0, 0, W - 1), x1 = clampi(X0 + n, 0, W - 1);
        const int y0 = clampi(Y0, 0, H - 1), y1 = clampi(Y0 + n, 0, H - 1);
        const uint8_t* s0 = src + (size_t)y0 * W * C;
        const uint8_t* s1 = src + (size_t)y1 * W * C;
#pragma unroll
        for (int c = 0; c < C; ++c)
            lb[b * C + c] = (uint16_t)((int)s0[x0 * C + c] + (int)s0[x1 * C + c] + (int)s1[x0 * C + c] +
                                       (int)s1[x1 * C + c]);
    }
    __syncthreads();
    // entry (r, q) of plane (py, px): slot t holds the bins of extended row
    // (r + t) P + py at extended column q P + px; an entry is WPE words of 8
    // bytes (four uint16 each, slot-major then channel; for C = 3 the packed
    // entry of the matcher's unpacking, two of its words each).  A run (plane, row) is nq WPE
    // consecutive words; the block's threads take runs_per_pass runs at a time.
    constexpr int WPE = bin_entry_bytes(C) / 8;
    const int nq = min(Q, Wq - q0), nr = min(R, Hq - r0);
    const int words_run = nq * WPE;
    const int runs_per_pass = max(1, 256 / words_run);
    const int k = (int)threadIdx.x % words_run, rsub = (int)threadIdx.x / words_run;
    const int e = k / WPE, j = k - e * WPE;  // entry within the run, word within the entry
    const int nruns = P * P * nr;
    uint2* out = reinterpret_cast<uint2*>(bins);
    if (rsub < runs_per_pass && k < words_run) {
        int plane = 0, rr = rsub;  // run = plane * nr + rr, advanced by runs_per_pass
        while (rr >= nr) {
            rr -= nr;
            ++plane;
        }
        for (int run = rsub; run < nruns; run += runs_per_pass) {
            const int py = plane >> sh, px = plane & (P - 1);
            const size_t o = ((((size_t)m * P * P + plane) * Hq + (r0 + rr)) * Wq + q0 + e) * WPE + j;
            if constexpr (C == 3) {
                // word j holds words 2 j and 2 j + 1 of the packed entry: channel j
                // of bins (0, 1) and (2, 3) in the halves' low 10 bits, and channel 2
                // of bins (2 j, 2 j + 1) split low 6 / high 4 bits over their spare
                // bits 10..15
                uint32_t ch[4], c2[2];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint16_t* b = lb + ((((rr + u) * P + py) << lqp) + e * P + px) * 3;
                    ch[u] = b[j];
                    if (u >> 1 == j) c2[u & 1] = b[2];
                }
                const uint32_t lo = ((c2[0] & 0x3Fu) << 10) | ((c2[1] & 0x3Fu) << 26);
                const uint32_t hi = ((c2[0] >> 6) << 10) | ((c2[1] >> 6) << 26);
                out[o] = make_uint2(ch[0] | (ch[1] << 16) | lo, ch[2] | (ch[3] << 16) | hi);
            } else {
                uint32_t v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int t = 4 * j + u, slot = t / C, c = t - slot * C;
                    v[u] = lb[((((rr + slot) * P + py) << lqp) + e * P + px) * C + c];
                }
                out[o] = make_uint2(v[0] | (v[1] << 16), v[2] | (v[3] << 16));
            }
            rr += runs_per_pass;
            while (rr >= nr) {
                rr -= nr;
                ++plane;
            }
        }
    }
}

void launch_bins(const sff_params& p, int nimg, int level, const uint8_t* S, uint16_t* bins,
                 hipStream_t st) {
    const BinGeom g = bin_geom(p, level);
    const int QP = bin_tile_qp(g.P), R = bin_tile_rows(g.P), Q = QP / g.P;
    const dim3 grid((g.Wq + Q - 1) / Q, (g.Hq + R - 1) / R, nimg);
    switch (p.C) {
        case 1: hipLaunchKernelGGL(bins_tile_kernel<1>, grid, dim3(256), 0, st, S, bins, p.H, p.W, g.n, g.sh, g.Hq, g.Wq); break;
        case 2: hipLaunchKernelGGL(bins_tile_kernel<2>, grid, dim3(256), 0, st, S, bins, p.H, p.W, g.n, g.sh, g.Hq, g.Wq); break;
        case 3: hipLaunchKernelGGL(bins_tile_kernel<3>, grid, dim3(256), 0, st, S, bins, p.H, p.W, g.n, g.sh, g.Hq, g.Wq); break;
        default: hipLaunchKernelGGL(bins_tile_kernel<4>, grid, dim3(256), 0, st, S, bins, p.H, p.W, g.n, g.sh, g.Hq, g.Wq); break;
    }
}

}  // namespace
}  // namespace sff

using namespace sff;

extern "C" size_t sff_bin_bytes(const sff_params* p, int32_t level) {
    if (!params_ok(p) || level < 0 || level >= p->levels) return 0;
    return bin_image_bytes(*p, level);
}

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

namespace sff {
namespace {

sff_status wht_features(const sff_params* p, int32_t nimg, int32_t level, const uint8_t* img,
                        int16_t* desc, uint16_t* bins, uint8_t* ws, hipStream_t st) {
    const int H = p->H, W = p->W, C = p->C;
    const LevelGeom g = level_geom(*p, level);
    const size_t smem = wht_smem(g.n, C);
    if (desc && smem > 65536) return SFF_ERR_UNSUPPORTED;  // levels = 5 with C >= 3
    const WsLayout L = ws_layout(*p, nimg, level);
    const uint8_t* src = img;
    if (level > 0) {
        launch_smooth(*p, nimg, level, img, ws + L.a_off, ws + L.s_off, st);
        src = ws + L.s_off;
    }
    if (desc) {
        const dim3 grid((W + kTW - 1) / kTW, (H + wht_rows_rt(g.n) - 1) / wht_rows_rt(g.n), nimg);
        switch (C) {
            case 1: launch_wht<1>(g.n, grid, smem, st, src, desc, H, W); break;
            case 2: launch_wht<2>(g.n, grid, smem, st, src, desc, H, W); break;
            case 3: launch_wht<3>(g.n, grid, smem, st, src, desc, H, W); break;
            default: launch_wht<4>(g.n, grid, smem, st, src, desc, H, W); break;
        }
    }
    if (bins) launch_bins(*p, nimg, level, src, bins, st);
    return launch_status();
}

bool wht_args_ok(const sff_params* p, int32_t nimg, int32_t level, const uint8_t* img,
                 const int16_t* desc, const uint16_t* bins) {
    if (!params_ok(p) || nimg < 1 || nimg > 65535 || level < 0 || level >= p->levels || !img ||
        (!desc && !bins))
        return false;
    return (reinterpret_cast<uintptr_t>(desc) & 15) == 0 && (reinterpret_cast<uintptr_t>(bins) & 15) == 0;
}

// Fixed device scratch of the allocation-free variant: the block means and
// smoothed images of one call.  Each GPU the library runs on holds its own
// copy until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in, not a device address).
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
uint8_t* scratch_ptr[kMaxDevices];

// Device address of the current device's scratch, looked up once per device
// (on the first call with that device current); NULL on a runtime error.
uint8_t* scratch_for_current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        scratch_ptr[dev] = static_cast<uint8_t*>(ptr);
    }
    return scratch_ptr[dev];
}

}  // namespace
}  // namespace sff

extern "C" sff_status sff_wht_features(const sff_params* p, int32_t nimg, int32_t level,
                                       const uint8_t* img, int16_t* desc, uint16_t* bins,
                                       void* workspace, size_t workspace_bytes, void* stream) {
    if (!wht_args_ok(p, nimg, level, img, desc, bins)) return SFF_ERR_INVALID_ARG;
    const WsLayout L = ws_layout(*p, nimg, level);
    if (level > 0 && (!workspace || workspace_bytes < L.total)) return SFF_ERR_WORKSPACE;
    return wht_features(p, nimg, level, img, desc, bins, static_cast<uint8_t*>(workspace),
                        as_stream(stream));
}

extern "C" size_t sff_wht_scratch_bytes(void) { return kScratchBytes; }

extern "C" sff_status sff_wht_features_noalloc(const sff_params* p, int32_t nimg, int32_t level,
                                               const uint8_t* img, int16_t* desc, uint16_t* bins,
                                               void* stream) {
    if (!wht_args_ok(p, nimg, level, img, desc, bins)) return SFF_ERR_INVALID_ARG;
    const WsLayout L = ws_layout(*p, nimg, level);
    if (L.total > kScratchBytes) return SFF_ERR_WORKSPACE;
    uint8_t* ws = nullptr;
    if (level > 0) {
        ws = scratch_for_current_device();
        if (!ws) return SFF_ERR_HIP;
    }
    return wht_features(p, nimg, level, img, desc, bins, ws, as_stream(stream));
}

extern "C" sff_status sff_smooth_level(const sff_params* p, int32_t nimg, int32_t level,
                                       const uint8_t* img, uint8_t* out, void* workspace,
                                       size_t workspace_bytes, void* stream) {
    if (!params_ok(p) || nimg < 1 || nimg > 65535 || level < 0 || level >= p->levels || !img || !out)
        return SFF_ERR_INVALID_ARG;
    const WsLayout L = ws_layout(*p, nimg, level);
    if (level > 0 && (!workspace || workspace_bytes < L.s_off)) return SFF_ERR_WORKSPACE;
    hipStream_t st = as_stream(stream);
    if (level == 0) {
        if (hipMemcpyAsync(out, img, (size_t)nimg * p->H * p->W * p->C, hipMemcpyDeviceToDevice, st) !=
            hipSuccess)
            return SFF_ERR_HIP;
        return SFF_OK;
    }
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    launch_smooth(*p, nimg, level, img, ws + L.a_off, out, st);
    return launch_status();
}
