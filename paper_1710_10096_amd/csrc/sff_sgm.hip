// Disparity fill (SceneFlowFields, Section 3.1, last paragraph of "Consistency
// Check"): a second disparity map by semi-global matching (Hirschmueller,
// TPAMI 2008) and the check of the disparity matches alone against it.
//
// Cost: Hamming distance of 5 x 5 census words of the channel-mean images,
// right pixel x - d clamped to the image.  Aggregation along 8 paths,
//   L(p, d) = C(p, d) + min(L(q, d), L(q, d +- 1) + P1, min_k L(q, k) + P2)
//             - min_k L(q, k),   q = p - r,
// summed over the paths; the disparity minimises the sum (smallest d on ties).
// One wave per path line, four disparities per lane: the line is walked
// sequentially, neighbouring disparities exchanged by DPP lane moves and the
// minimum over d by a DPP reduction; the cost of a pixel is recomputed from
// the census words, so no cost volume is stored; each direction's costs (at
// most 24 + P2 <= 255) are written as uint8 and summed per pixel at the end.
#include <climits>

#include "sff_internal.hpp"

namespace sff {
namespace {

constexpr int kMaxD = 256;
constexpr int kPad = kMaxD;  // left pad of the right census rows

__global__ void __launch_bounds__(256) grey_kernel(const uint8_t* __restrict__ img, uint8_t* __restrict__ g,
                                                   int npx, int C, size_t pair_stride) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= npx) return;
    const uint8_t* src = img + (size_t)blockIdx.y * pair_stride + (size_t)p * C;
    int s = 0;
    for (int c = 0; c < C; ++c) s += src[c];
    g[(size_t)blockIdx.y * npx + p] = (uint8_t)((s + C / 2) / C);
}

// bit k set when neighbour k (row-major over the 5 x 5 window without the
// centre) is darker than the centre; replicated border
// Census words of one image, rows of kPad + W words when pad = kPad (the pad
// words repeat column 0, so x - d reads the clamped pixel without a clamp).
__global__ void __launch_bounds__(256) census_kernel(const uint8_t* __restrict__ g,
                                                     uint32_t* __restrict__ cw, int H, int W, int pad) {
    const int Wo = W + pad;
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= H * Wo) return;
    const uint8_t* gi = g + (size_t)blockIdx.y * H * W;
    const int y = p / Wo, x = max(p - y * Wo - pad, 0);
    const int c = gi[y * W + x];
    uint32_t w = 0;
    int k = 0;
#pragma unroll
    for (int dy = -2; dy <= 2; ++dy)
#pragma unroll
        for (int dx = -2; dx <= 2; ++dx) {
            if (dx == 0 && dy == 0) continue;
            const int v = gi[clampi(y + dy, 0, H - 1) * W + clampi(x + dx, 0, W - 1)];
            w |= (uint32_t)(v < c) << k;
            ++k;
        }
    cw[(size_t)blockIdx.y * H * Wo + p] = w;
}

struct PathArgs {
    const uint32_t* cl;  // [batch][H][W] census of the left images
    const uint32_t* cr;  // [batch][H][kPad + W] census of the right images, padded rows
    uint8_t* L;          // [8][batch][H][W][Dp] path costs per direction, Dp = D rounded to 4
    int H, W, D, Dp, P1, P2, batch;
};

__constant__ int kDirs[8][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, -1}, {1, -1}, {-1, 1}};

// Lane moves by DPP: the value of lane l - 1 (wave_shr:1) or l + 1 (wave_shl:1),
// and the minimum over the wave (quad, half-row and row mirrors, then the four
// rows by readlane), so the per-step chain never goes through the LDS crossbar.
__device__ __forceinline__ int from_lane_below(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ int from_lane_above(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ int wave_min_uniform(int m) {
    m = min(m, __builtin_amdgcn_update_dpp(0, m, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
    m = min(m, __builtin_amdgcn_update_dpp(0, m, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
    m = min(m, __builtin_amdgcn_update_dpp(0, m, 0x141, 0xF, 0xF, false));  // row_half_mirror
    m = min(m, __builtin_amdgcn_update_dpp(0, m, 0x140, 0xF, 0xF, false));  // row_mirror
    return min(min(__builtin_amdgcn_readlane(m, 0), __builtin_amdgcn_readlane(m, 16)),
               min(__builtin_amdgcn_readlane(m, 32), __builtin_amdgcn_readlane(m, 48)));
}

// One wave per path line (4 lines per block; blockIdx.y = batch element,
// blockIdx.z = direction); lane l holds disparities 4l .. 4l + 3, so the
// neighbours d - 1 and d + 1 across lanes come from DPP lane moves and the
// minimum over d from a DPP reduction: no block barrier.  The census words are
// loaded kAhead - 1 steps ahead into a register ring.  The walk starts from
// zero costs, which makes the first step L = C (P1, P2 >= 0).
__global__ void __launch_bounds__(256) sgm_path_kernel(PathArgs a) {
    const int lane = threadIdx.x & 63;
    const int H = a.H, W = a.W, D = a.D;
    const int r = blockIdx.z, dx = kDirs[r][0], dy = kDirs[r][1];
    // the horizontal lines are the longest chains (W steps): they get the
    // issue slots first, the shorter lines fill the gaps
    if (dy == 0) __builtin_amdgcn_s_setprio(2);
    const int ncol = dx != 0 ? H : 0;
    const int lines = ncol + (dy != 0 ? W - (dx != 0 ? 1 : 0) : 0);
    const int line = blockIdx.x * 4 + wave_id();
    if (line >= lines) return;  // whole wave
    int x0, y0;
    if (line < ncol) {
        x0 = dx > 0 ? 0 : W - 1;
        y0 = line;
    } else {
        const int k = line - ncol;
        x0 = dx != 0 ? (dx > 0 ? 1 + k : W - 2 - k) : k;
        y0 = dy > 0 ? 0 : H - 1;
    }
    const int nx = dx > 0 ? W - x0 : (dx < 0 ? x0 + 1 : INT_MAX);
    const int ny = dy > 0 ? H - y0 : (dy < 0 ? y0 + 1 : INT_MAX);
    const int len = min(nx, ny);
    const size_t base = (size_t)blockIdx.y * H * W;
    const uint32_t* cl = a.cl + base;
    const uint32_t* cr = a.cr + (size_t)blockIdx.y * H * (W + kPad) + kPad;
    uint8_t* L8 = a.L + ((size_t)r * a.batch + blockIdx.y) * H * W * a.Dp;
    constexpr int kBig = 1 << 28;
    constexpr int kAhead = 4;  // 8 measured no faster
    const int d0 = 4 * lane, lane_off = 252 - d0;
    // right word for disparity d0 + k: row[x - d0 - k] = (row + x - 255)[lane_off + 3 - k],
    // a uniform base plus a fixed lane offset
    auto load = [&](int t, uint32_t& wl, uint32_t (&wr)[4]) {
        const int x = x0 + t * dx, y = y0 + t * dy;
        const uint32_t* rb = cr + (size_t)y * (W + kPad) + x - 255;
        wl = cl[(size_t)y * W + x];
#pragma unroll
        for (int k = 0; k < 4; ++k) wr[k] = rb[lane_off + 3 - k];
    };
    int Lp[4] = {0, 0, 0, 0}, prev_min = 0;
    auto step = [&](int t, uint32_t wl, const uint32_t (&wr)[4]) {
        int up = from_lane_below(Lp[3]), dn = from_lane_above(Lp[0]);
        up = lane == 0 ? kBig : up;
        dn = lane == 63 ? kBig : dn;
        int L[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int c = __popc(wl ^ wr[k]);
            const int lm = k == 0 ? up : Lp[k - 1];
            const int lp = k == 3 ? dn : Lp[k + 1];
            int m = min(Lp[k], min(lm, lp) + a.P1);
            m = min(m, prev_min + a.P2);
            L[k] = d0 + k < D ? c + m - prev_min : kBig;  // kBig never wins a minimum
        }
        if (d0 < D) {
            const size_t p = (size_t)(y0 + t * dy) * W + x0 + t * dx;
            uint32_t packed = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) packed |= (uint32_t)(L[k] & 0xFF) << (8 * k);
            *reinterpret_cast<uint32_t*>(L8 + p * a.Dp + d0) = packed;
        }
        prev_min = wave_min_uniform(min(min(L[0], L[1]), min(L[2], L[3])));
#pragma unroll
        for (int k = 0; k < 4; ++k) Lp[k] = L[k];
    };
    // ring slot i holds step t + i at the top of each group of kAhead steps;
    // the loads never depend on a branch (steps past the end reload the last
    // pixel), so their waits stay kAhead - 1 steps behind the issue
    uint32_t ql[kAhead], qr[kAhead][4];
#pragma unroll
    for (int j = 0; j < kAhead - 1; ++j) load(min(j, len - 1), ql[j], qr[j]);
    int t = 0;
    for (; t + kAhead <= len; t += kAhead) {
#pragma unroll
        for (int j = 0; j < kAhead; ++j) {
            const int jn = (j + kAhead - 1) % kAhead;
            load(min(t + j + kAhead - 1, len - 1), ql[jn], qr[jn]);
            step(t + j, ql[j], qr[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < kAhead - 1; ++j)
        if (t + j < len) step(t + j, ql[j], qr[j]);
}

// Winner-take-all over the summed path costs: one wave per pixel, lane l
// holds disparities 4l .. 4l + 3 (one dword of each direction's plane), the
// 8 planes are summed two bytes at a time in 16-bit fields (at most 8 * 255),
// and the minimum of (sum, d) over the wave gives the smallest d on ties.
// Each wave takes kWtaPix consecutive pixels with all their loads in flight.
constexpr int kWtaPix = 4;
__global__ void __launch_bounds__(256) wta_kernel(const uint32_t* __restrict__ L4,
                                                  int16_t* __restrict__ disp, int npx, int D, int nd,
                                                  int batch) {
    const int lane = threadIdx.x & 63;
    const int p0 = (blockIdx.x * 4 + wave_id()) * kWtaPix;
    if (p0 >= npx) return;  // whole wave
    const size_t plane = (size_t)batch * npx * nd;
    const uint32_t* s = L4 + ((size_t)blockIdx.y * npx + p0) * nd + lane;
    const int np = min(kWtaPix, npx - p0);
    const bool on = lane < nd;
    uint32_t w[kWtaPix][8];
#pragma unroll
    for (int j = 0; j < kWtaPix; ++j)
#pragma unroll
        for (int r = 0; r < 8; ++r) w[j][r] = on && j < np ? s[r * plane + (size_t)j * nd] : 0u;
#pragma unroll
    for (int j = 0; j < kWtaPix; ++j) {
        uint32_t lo = 0, hi = 0;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            lo += w[j][r] & 0x00FF00FFu;
            hi += (w[j][r] >> 8) & 0x00FF00FFu;
        }
        const uint32_t sum[4] = {lo & 0xFFFFu, hi & 0xFFFFu, lo >> 16, hi >> 16};
        int best = 0x7FFFFFFF;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int d = 4 * lane + k;
            if (d < D) best = min(best, (int)(sum[k] << 8) | d);
        }
        best = wave_min_uniform(best);
        if (lane == 0 && j < np) disp[(size_t)blockIdx.y * npx + p0 + j] = (int16_t)(best & 0xFF);
    }
}

__global__ void __launch_bounds__(256) fill_kernel(const int16_t* __restrict__ hyp,
                                                   const uint8_t* __restrict__ valid,
                                                   const int16_t* __restrict__ disp,
                                                   uint8_t* __restrict__ fill, int H, int W, int tau) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= H * W) return;
    const size_t o = (size_t)blockIdx.y * H * W + p;
    const int x = p % W;
    const int d0 = hyp[o * 4 + 2];
    const int e = d0 - disp[o];
    fill[o] = (valid[o] || (x - d0 >= 0 && e <= tau && e >= -tau)) ? 1 : 0;
}

struct SgmWs {
    size_t grey, census, census_r, S, total;
};

SgmWs sgm_ws(const sff_params& p, int batch) {
    const size_t npx = (size_t)p.H * p.W, n = (size_t)batch;
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    SgmWs L;
    L.grey = 0;
    L.census = al(2 * n * npx);
    L.census_r = L.census + al(n * npx * sizeof(uint32_t));
    L.S = L.census_r + al(n * p.H * (p.W + (size_t)kPad) * sizeof(uint32_t));
    L.total = L.S + al(8 * n * npx * (size_t)((p.dmax + 4) & ~3));
    return L;
}

}  // namespace
}  // namespace sff

using namespace sff;

extern "C" size_t sff_sgm_workspace_bytes(const sff_params* p, int32_t batch) {
    if (!params_ok(p) || batch < 1 || batch > 32767) return 0;
    return sgm_ws(*p, batch).total;
}

extern "C" sff_status sff_sgm_disparity(const sff_params* p, int32_t batch, const uint8_t* left,
                                        const uint8_t* right, size_t pair_stride, int32_t P1,
                                        int32_t P2, int16_t* disp, void* workspace,
                                        size_t workspace_bytes, void* stream) {
    if (!params_ok(p) || batch < 1 || batch > 32767 || !left || !right || !disp || P1 < 0 ||
        P2 < P1 || P2 > 231 || (reinterpret_cast<uintptr_t>(disp) & 1) != 0)
        return SFF_ERR_INVALID_ARG;
    const size_t img_bytes = (size_t)p->H * p->W * p->C;
    if (batch > 1 && pair_stride < img_bytes) return SFF_ERR_INVALID_ARG;
    const int D = p->dmax + 1;
    if (D > kMaxD) return SFF_ERR_UNSUPPORTED;
    const SgmWs L = sgm_ws(*p, batch);
    if (!workspace || workspace_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return SFF_ERR_WORKSPACE;
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    const int H = p->H, W = p->W, npx = H * W;
    uint8_t* gl = ws + L.grey;
    uint8_t* gr = gl + (size_t)batch * npx;
    uint32_t* cl = reinterpret_cast<uint32_t*>(ws + L.census);
    uint32_t* cr = reinterpret_cast<uint32_t*>(ws + L.census_r);
    uint8_t* L8 = ws + L.S;
    hipStream_t st = as_stream(stream);
    const dim3 pgrid((npx + 255) / 256, batch);
    hipLaunchKernelGGL(grey_kernel, pgrid, dim3(256), 0, st, left, gl, npx, p->C, pair_stride);
    hipLaunchKernelGGL(grey_kernel, pgrid, dim3(256), 0, st, right, gr, npx, p->C, pair_stride);
    hipLaunchKernelGGL(census_kernel, pgrid, dim3(256), 0, st, gl, cl, H, W, 0);
    hipLaunchKernelGGL(census_kernel, dim3((H * (W + kPad) + 255) / 256, batch), dim3(256), 0, st, gr, cr,
                       H, W, kPad);
    const int Dp = (D + 3) & ~3;
    PathArgs a{cl, cr, L8, H, W, D, Dp, P1, P2, batch};
    hipLaunchKernelGGL(sgm_path_kernel, dim3((H + W - 1 + 3) / 4, batch, 8), dim3(256), 0, st, a);
    hipLaunchKernelGGL(wta_kernel, dim3((npx + 4 * kWtaPix - 1) / (4 * kWtaPix), batch), dim3(256), 0, st,
                       reinterpret_cast<const uint32_t*>(L8), disp, npx, D, Dp / 4, batch);
    return launch_status();
}

extern "C" sff_status sff_disparity_fill(const sff_params* p, int32_t batch, const int16_t* hyp_fwd,
                                         const uint8_t* valid, const int16_t* disp, uint8_t* fill,
                                         void* stream) {
    if (!params_ok(p) || batch < 1 || batch > 32767 || !hyp_fwd || !valid || !disp || !fill ||
        (reinterpret_cast<uintptr_t>(hyp_fwd) & 7) != 0 || (reinterpret_cast<uintptr_t>(disp) & 1) != 0)
        return SFF_ERR_INVALID_ARG;
    hipLaunchKernelGGL(fill_kernel, dim3((p->H * p->W + 255) / 256, batch), dim3(256), 0,
                       as_stream(stream), hyp_fwd, valid, disp, fill, p->H, p->W, p->tau);
    return launch_status();
}
