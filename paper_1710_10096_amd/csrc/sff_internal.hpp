// Internal helpers of libsff (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "sff.h"

namespace sff {

constexpr int kMaxLevels = 5;  // pyramid factor n <= 16
constexpr int kMaxC = 4;

// Channels of a stored descriptor record (power of two >= C).
inline int rec_channels(int C) { return C == 3 ? 4 : C; }

struct LevelGeom {
    int n, Hk, Wk;
};

inline LevelGeom level_geom(const sff_params& p, int level) {
    LevelGeom g;
    g.n = 1 << level;
    g.Hk = (p.H + g.n - 1) / g.n;
    g.Wk = (p.W + g.n - 1) / g.n;
    return g;
}

// Host-side parameter validation shared by every entry point.
inline bool params_ok(const sff_params* p) {
    if (!p) return false;
    if (p->H < 1 || p->H > 16384 || p->W < 1 || p->W > 16384) return false;
    if (p->C < 1 || p->C > kMaxC) return false;
    if (p->levels < 1 || p->levels > kMaxLevels) return false;
    if (p->iters < 0 || p->iters > 64) return false;
    if (p->rs_samples < 0 || p->rs_samples > 16) return false;
    if (p->rs_r0 < 1 || p->rs_r0 > 4096) return false;
    if (p->fmax < 0 || p->fmax > 8192 || p->dmax < 0 || p->dmax > 8192) return false;
    if (p->tau < 0 || p->tau > 8192) return false;
    return true;
}

inline sff_status launch_status() {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFF_OK : SFF_ERR_HIP;
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------- device --
__device__ __forceinline__ int clampi(int a, int lo, int hi) { return min(max(a, lo), hi); }

// Blocks are dealt to the 8 XCDs round-robin (block id mod 8).  Renumber them
// so that each XCD receives one contiguous run of tiles (a bijection of
// [0, nb)); with tiles numbered column-major within a field that run is a
// vertical strip of the image, whose gather targets (shifted by locally
// coherent vectors) stay compact and in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
    const int xcd = bid & 7, k = bid >> 3;
    const int q = nb >> 3, rem = nb & 7;
    return xcd * q + min(xcd, rem) + k;
}

// Index of the calling wave (64 lanes) in its block, as a scalar: lets the
// compiler keep per-wave quantities and branches in scalar registers.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Philox4x32-10 (Salmon et al., SC'11): 10 rounds, multipliers 0xD2511F53 and
// 0xCD9E8D57, Weyl key increments 0x9E3779B9 and 0xBB67AE85.
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
        U4 o;
        o.x = hi1 ^ c.y ^ k0;
        o.y = lo1;
        o.z = hi0 ^ c.w ^ k1;
        o.w = lo0;
        c = o;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Uniform integer in [-r, r] from one 32-bit draw: floor(x (2r+1) / 2^32) - r.
__device__ __forceinline__ int uniform_offset(uint32_t x, int r) {
    return (int)(((uint64_t)x * (uint64_t)(2 * r + 1)) >> 32) - r;
}

}  // namespace sff
