// Internal helpers of libsff (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>

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

// Bin-sum planes of level k.  The 4x4 lowest-sequency block of a WHT patch is
// the 4-point Hadamard transform (both axes) of the patch's 4 x 4 grid of
// 2 x 2-bin sums, so the squared distance of two descriptors is exactly 16
// times that of their bin grids.  Bin (i, j) of the patch at (X, Y) sums the
// four pixels at X + n (2j - 3 + b), Y + n (2i - 3 + a), a, b in {0, 1}
// (replicated border); the bin at extended column ex = X + n (2j - 3) + 3n
// lives in phase plane ex mod 2n at index ex / 2n, so a patch is 4 x 4
// consecutive positions of one plane: columns X / 2n .. + 3 of plane X mod 2n,
// rows Y / 2n .. + 3 of plane Y mod 2n.  Plane (py, px) = py * 2n + px holds
// Hq x Wq entries; entry (r, q) holds the bins of plane rows r .. r + 3 at
// column q (each bin stored in four entries), so a patch is one contiguous run
// of 4 entries.  A bin is C uint16 channels, except for C = 3, where an
// entry's four bins of three 10-bit channels (a bin sums four bytes, at most
// 1020) are packed into 16 bytes (layout at BinRef<3>): 64-byte patches instead
// of 96, so a patch spans fewer cache lines and a gather moves two thirds of
// the bytes.  Patch = bin_pieces(C) pieces of 16 bytes.
struct BinGeom {
    int n, sh, P, Hq, Wq;  // n = 2^k, P = 2n = 1 << sh
};

inline BinGeom bin_geom(const sff_params& p, int level) {
    BinGeom g;
    g.n = 1 << level;
    g.sh = level + 1;
    g.P = 2 * g.n;
    g.Hq = (p.H - 1) / g.P + 1;
    g.Wq = (((p.W - 1) / g.P + 4) + 15) & ~15;
    return g;
}

// Bytes of one entry (4 plane rows of C channels), 16-byte pieces of a patch
// (4 entries), and bytes of one image's planes.
__host__ __device__ constexpr int bin_entry_bytes(int C) { return C == 3 ? 16 : 8 * C; }
__host__ __device__ constexpr int bin_pieces(int C) { return bin_entry_bytes(C) / 4; }
inline size_t bin_image_bytes(const sff_params& p, int level) {
    const BinGeom g = bin_geom(p, level);
    return (size_t)g.P * g.P * g.Hq * g.Wq * bin_entry_bytes(p.C);
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

// Each round's two 32 x 32 -> 64-bit products are formed as 64-bit multiplies
// (one v_mad_u64_u32 each instead of a low and a high multiply).
__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        U4 o;
        o.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        o.y = (uint32_t)p1;
        o.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        o.w = (uint32_t)p0;
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

// The library's helper stream of the current device (default priority, not
// blocking on the null stream, created on first use and kept until the
// process ends) with a fork and a join event, for a call that runs two
// independent launch sequences concurrently: helper_fork makes the helper
// wait for the work enqueued on st so far, helper_join makes st wait for the
// helper's.  Callers hold helper_lock() from the fork to the join (the events
// are shared); helper_for_current_device returns null on a runtime error.
struct HelperStream {
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
std::mutex& helper_lock();
HelperStream* helper_for_current_device();
bool helper_fork(HelperStream* h, hipStream_t st);
bool helper_join(HelperStream* h, hipStream_t st);

}  // namespace sff
