// Multi-scale propagation and random search at one level (SceneFlowFields,
// Section 3.1, "Multi-Scale Propagation"), with the eq. (1) matching cost.
//
// Schedule: per iteration a red half-step (pixels with (i + j) even) then a
// black one.  Pixels of one colour only read the other colour's vectors, so a
// half-step is a race-free Jacobi sweep and its result does not depend on the
// order in which threads run.  Each pixel: cheapest of [own, left, up, right,
// down] under strict improvement, then rs_samples random-search samples around
// that vector (Philox4x32-10), kept on strict improvement.
//
// The hand-off from the coarser level is fused into iteration 0: a pixel whose
// level-k vector has not been written yet reads its parent's vector from the
// coarse field and computes its cost at this level.
//
// Two kinds of feature maps feed the same kernel: descriptor records (one
// record of C x 16 int16 per pixel: the WHT descriptors, or any descriptors
// such as learned ones; sff_match_level), and the WHT descriptors' bin-sum
// planes (sff_match_level_bins).  The descriptor of a pixel is the 4x4
// lowest-sequency block of the WHT of its 8x8 patch, i.e. the 4-point Hadamard
// transform along both axes of the patch's 4 x 4 grid of 2 x 2-bin sums; that
// transform is orthogonal up to a factor of 4 per axis, so the squared
// distance of two descriptors is exactly 16 times the squared distance of
// their bin grids (all integers).  The bin grids of neighbouring pixels
// overlap, so one level's planes (BinGeom: 24 bytes per position at C = 3,
// each bin stored for four rows) are a fifth of the descriptor records' size
// and the gathers mostly hit the L2 instead of streaming records.
#include <cstdlib>
#include <cstring>

#include "sff_device.hpp"

namespace sff {
namespace {

struct MatchArgs {
    const uint8_t* maps;        // [batch][4] images of descriptor records or bin planes
    size_t img_bytes;           // bytes of one image's map
    const uint64_t* seeds;      // [batch]
    const int16_t* hyp_coarse;  // [ndir][batch][Hc][Wc][4] or null
    int16_t* hyp;               // [ndir][batch][Hk][Wk][4]
    uint32_t* cost;             // [ndir][batch][Hk][Wk]
    int H, W, n, level, Hk, Wk, Hc, Wc;
    int sh, Hq, Wq;             // bin planes (BinGeom)
    int rs_r0, rs_samples, fmax, dmax;
    int batch, dir0, ndir;
};

struct Hyp {
    int u, v, d0, d1;
};

__device__ __forceinline__ Hyp unpack(uint2 h) {
    Hyp r;
    r.u = (int)(int16_t)(h.x & 0xFFFFu);
    r.v = (int)(int16_t)(h.x >> 16);
    r.d0 = (int)(int16_t)(h.y & 0xFFFFu);
    r.d1 = (int)(int16_t)(h.y >> 16);
    return r;
}

__device__ __forceinline__ uint2 pack(const Hyp& h) {
    uint2 r;
    r.x = (uint32_t)(uint16_t)(int16_t)h.u | ((uint32_t)(uint16_t)(int16_t)h.v << 16);
    r.y = (uint32_t)(uint16_t)(int16_t)h.d0 | ((uint32_t)(uint16_t)(int16_t)h.d1 << 16);
    return r;
}

__device__ __forceinline__ bool same(const Hyp& a, const Hyp& b) {
    return a.u == b.u && a.v == b.v && a.d0 == b.d0 && a.d1 == b.d1;
}

// Wave-level ordering of LDS accesses made by different lanes of one wave.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Raw buffer descriptor of one image's map (wave-uniform base), with the
// image's size as its range: a load at an offset at or past `bytes` returns
// zeros without a memory access.  Offsets are 32-bit, so a map is smaller than
// 2 GiB.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t map_rsrc(const void* M, uint32_t bytes) {
    const uint64_t p = reinterpret_cast<uint64_t>(M);
    const uint64_t u = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)p) |
                       ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(p >> 32)) << 32);
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(u), (short)0,
                                             (int)__builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}

// Offset of no patch: past the range of every image (images are smaller).
constexpr int kNoTarget = 0x7FFFFFF0;

// Map of view v (0..3 in the canonical order) for direction s: the forward
// field has reference I_l^0 and targets I_l^1 (temporal), I_r^0 (stereo),
// I_r^1 (cross); the inverse field has reference I_r^1 and targets I_r^0,
// I_l^1, I_l^0.
struct Views {
    const uint8_t *R, *T, *S, *X;
    __device__ __forceinline__ Views(const MatchArgs& a, int b, int s) {
        const uint8_t* base = a.maps + (size_t)b * 4 * a.img_bytes;
        R = base + (size_t)(s > 0 ? 0 : 3) * a.img_bytes;
        T = base + (size_t)(s > 0 ? 1 : 2) * a.img_bytes;
        S = base + (size_t)(s > 0 ? 2 : 1) * a.img_bytes;
        X = base + (size_t)(s > 0 ? 3 : 0) * a.img_bytes;
    }
};

// s * v for a direction s = +1 or -1.
__device__ __forceinline__ int dirmul(int s, int v) { return s > 0 ? v : -v; }

// Descriptor gathers of one wave, done cooperatively.  Lane l of the wave owns
// one pixel (its reference descriptor and hypothesis); a descriptor is P = 2C
// pieces of 16 bytes.  Gathering one descriptor per owner takes P wave-wide
// loads; in load k lane l fetches piece w = f mod P of owner o = f / P, with
// f = 64 k + l, so the lanes of one load read consecutive pieces of a few
// records (each inside one cache line) instead of 64 unrelated lines.  Each
// lane keeps the reference pieces of its (o, w) slots in registers, forms the
// piece's partial squared distance, and the P partials of an owner are summed
// through the wave's LDS slice.  Gathers are buffer loads with 32-bit byte
// offsets from the map's base (one add per load instead of 64-bit address
// arithmetic), so a map must be smaller than 2 GiB.  Owners without a target
// (tp < 0) gather record 0 and have their sum zeroed once, after the
// reduction, instead of each piece being predicated.  A wave has O owners
// (64, or 32 to put twice as many waves on a level too small to fill the chip;
// lanes O..63 then only help gather), so a descriptor gather is K = O P / 64
// wave-wide loads.
template <int C, int O>
struct Coop {
    static_assert(O == 64 || O == 32, "owners per wave");
    static constexpr int P = 2 * C;
    static constexpr int K = O * P / 64;
    static constexpr int RS = 2 * kRecC<C>;  // record stride in 16-byte pieces
    uint4 refp[K];                          // reference piece of slot k
    uint32_t* part;                         // this wave's LDS slice [64 P]
    int lane;
    uint32_t bytes;                         // bytes of one map

    __device__ __forceinline__ static int owner(int k, int lane) { return (64 * k + lane) / P; }
    __device__ __forceinline__ static int piece(int k, int lane) { return (64 * k + lane) % P; }

    // Piece (k, lane) of the record at byte offset ob of the slot's owner.
    __device__ __forceinline__ uint4 gather(__amdgpu_buffer_rsrc_t rs, int ob, int k) const {
        const int off = __shfl(ob, owner(k, lane)) + piece(k, lane) * 16;
        return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
    }

    // Load the reference pieces; pix_of(o) is owner o's pixel in map R.
    template <class F>
    __device__ __forceinline__ void load_ref(const uint4* __restrict__ R, F pix_of) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            refp[k] = R[(size_t)pix_of(owner(k, lane)) * RS + piece(k, lane)];
    }

    // Squared distance between each owner's reference descriptor and the
    // descriptor of pixel tp in map M (0 for owners passing tp < 0).  Must be
    // called by all lanes of the wave.
    __device__ __forceinline__ uint32_t ssd(const uint4* M, int tp) {
        const __amdgpu_buffer_rsrc_t rs = map_rsrc(M, bytes);
        const int ob = max(tp, 0) * (RS * 16);
        uint4 v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = gather(rs, ob, k);
#pragma unroll
        for (int k = 0; k < K; ++k) part[64 * k + lane] = (uint32_t)piece_ssd(refp[k], v[k], 0);
        wave_sync();
        uint32_t c = 0;
        const int ol = lane & (O - 1);  // lanes past the owners read a valid slot
#pragma unroll
        for (int w = 0; w < P; ++w) c += part[ol * P + w];
        wave_sync();
        return tp >= 0 ? c : 0u;
    }

    // ssd for N targets per owner at once (all gathers in flight together);
    // needs a slice of N * 64 K words.
    template <int N>
    __device__ __forceinline__ void ssdN(const uint4* M, const int (&tp)[N], uint32_t (&c)[N]) {
        const __amdgpu_buffer_rsrc_t rs = map_rsrc(M, bytes);
        int ob[N];
#pragma unroll
        for (int m = 0; m < N; ++m) ob[m] = max(tp[m], 0) * (RS * 16);
        uint4 v[N][K];
#pragma unroll
        for (int m = 0; m < N; ++m)
#pragma unroll
            for (int k = 0; k < K; ++k) v[m][k] = gather(rs, ob[m], k);
#pragma unroll
        for (int m = 0; m < N; ++m)
#pragma unroll
            for (int k = 0; k < K; ++k) part[64 * (m * K + k) + lane] = (uint32_t)piece_ssd(refp[k], v[m][k], 0);
        wave_sync();
        const int ol = lane & (O - 1);
#pragma unroll
        for (int m = 0; m < N; ++m) {
            c[m] = 0;
#pragma unroll
            for (int w = 0; w < P; ++w) c[m] += part[64 * K * m + ol * P + w];
            c[m] = tp[m] >= 0 ? c[m] : 0u;
        }
        wave_sync();
    }
};

// eq. (1): temporal (x+u, y+v), stereo (x - s d0, y), cross (x+u - s d1, y+v),
// each target clamped to the image.  The three squared distances are
// non-negative, so once a partial sum reaches `bound` the candidate cannot be
// strictly cheaper than `bound`: the remaining gathers are skipped and a value
// >= bound is returned.  Below `bound` the exact cost is returned.  Lanes with
// want = false have no candidate; their result is meaningless.  The views are
// taken cross, temporal, stereo: the cross target moves with three of the four
// components (u, v, d1), the stereo one with d0 only, so this order rejects a
// poor candidate soonest (measured 1.8% faster at level 0 than temporal,
// stereo, cross).
//
// Two evaluators with the same results: LaneEval gathers each lane's records
// itself (fewest instructions and round trips; best when a launch has too few
// waves to fill the chip), CoopEval gathers cooperatively (fewest cache-line
// lookups; best when the chip is full).  CoopEval must be called by all lanes
// of the wave.
template <int C>
struct LaneEval {
    static constexpr int kOwners = 64;
    static constexpr int kLdsWords = 1;
    static constexpr int kPG = 1, kRG = 1;
    static constexpr bool kGroups = false;
    const uint4 *T, *S, *X, *R;
    int H, W, s;
    Desc<C> ref;

    __device__ __forceinline__ void setup(const MatchArgs& a, int b, int sd) {
        const Views v(a, b, sd);
        R = reinterpret_cast<const uint4*>(v.R);
        T = reinterpret_cast<const uint4*>(v.T);
        S = reinterpret_cast<const uint4*>(v.S);
        X = reinterpret_cast<const uint4*>(v.X);
        H = a.H;
        W = a.W;
        s = sd;
    }

    template <class F>
    __device__ __forceinline__ void init(int x, int y, int, uint32_t*, F) {
        ref = load_desc<C>(reinterpret_cast<const int16_t*>(R), (size_t)y * W + x);
    }

    __device__ __forceinline__ uint32_t map_ssd(const uint4* M, int pix) const {
        return desc_ssd<C>(ref, load_desc<C>(reinterpret_cast<const int16_t*>(M), (size_t)pix));
    }

    __device__ __forceinline__ uint32_t cost_below(bool want, int x, int y, const Hyp& h,
                                                   uint32_t bound) {
        if (!want) return 0xFFFFFFFFu;
        const int ty = clampi(y + h.v, 0, H - 1);
        uint32_t c = map_ssd(X, ty * W + clampi(x + h.u - dirmul(s, h.d1), 0, W - 1));
        if (c >= bound) return c;
        c += map_ssd(T, ty * W + clampi(x + h.u, 0, W - 1));
        if (c >= bound) return c;
        return c + map_ssd(S, y * W + clampi(x - dirmul(s, h.d0), 0, W - 1));
    }

    template <int N>
    __device__ __forceinline__ void cost_belowN(const bool (&)[N], const Hyp (&)[N], int, int,
                                                uint32_t, uint32_t (&)[N]) {}
};

// PG neighbour candidates and RG random-search samples are scored together
// (their gathers in flight at once); the LDS slice holds the partials of the
// larger group.
template <int C, int PG, int RG, int O = 64>
struct CoopEval {
    static constexpr int kOwners = O;
    static constexpr int kPG = PG, kRG = RG;
    static constexpr int kGroup = PG > RG ? PG : RG;
    static constexpr int kLdsWords = kGroup * 64 * Coop<C, O>::K;
    static constexpr bool kGroups = true;
    const uint4 *T, *S, *X, *R;
    int H, W, s;
    Coop<C, O> cp;

    __device__ __forceinline__ void setup(const MatchArgs& a, int b, int sd) {
        const Views v(a, b, sd);
        R = reinterpret_cast<const uint4*>(v.R);
        T = reinterpret_cast<const uint4*>(v.T);
        S = reinterpret_cast<const uint4*>(v.S);
        X = reinterpret_cast<const uint4*>(v.X);
        H = a.H;
        W = a.W;
        s = sd;
        cp.bytes = (uint32_t)a.img_bytes;
    }

    template <class F>
    __device__ __forceinline__ void init(int, int, int lane, uint32_t* part, F pix_of) {
        cp.lane = lane;
        cp.part = part;
        cp.load_ref(R, pix_of);
    }

    __device__ __forceinline__ uint32_t cost_below(bool want, int x, int y, const Hyp& h,
                                                   uint32_t bound) {
        const int ty = clampi(y + h.v, 0, H - 1);
        const int txX = clampi(x + h.u - dirmul(s, h.d1), 0, W - 1);
        uint32_t c = cp.ssd(X, want ? ty * W + txX : -1);
        bool alive = want && c < bound;
        if (__any(alive)) {
            const int txT = clampi(x + h.u, 0, W - 1);
            c += cp.ssd(T, alive ? ty * W + txT : -1);
            alive = alive && c < bound;
            if (__any(alive)) {
                const int txS = clampi(x - dirmul(s, h.d0), 0, W - 1);
                c += cp.ssd(S, alive ? y * W + txS : -1);
            }
        }
        return c;
    }

    // cost_below for N candidates of each lane, their gathers issued together
    // view by view; same results as N calls with the same bound.
    template <int N>
    __device__ __forceinline__ void cost_belowN(const bool (&w)[N], const Hyp (&h)[N], int x, int y,
                                                uint32_t bound, uint32_t (&c)[N]) {
        static_assert(N <= kGroup, "LDS slice sized for kGroup candidates");
        int ty[N], tp[N];
        bool al[N];
        bool any = false;
#pragma unroll
        for (int m = 0; m < N; ++m) {
            ty[m] = clampi(y + h[m].v, 0, H - 1);
            tp[m] = w[m] ? ty[m] * W + clampi(x + h[m].u - dirmul(s, h[m].d1), 0, W - 1) : -1;
        }
        cp.template ssdN<N>(X, tp, c);
#pragma unroll
        for (int m = 0; m < N; ++m) {
            al[m] = w[m] && c[m] < bound;
            any = any || al[m];
            tp[m] = al[m] ? ty[m] * W + clampi(x + h[m].u, 0, W - 1) : -1;
        }
        if (!__any(any)) return;
        uint32_t d[N];
        cp.template ssdN<N>(T, tp, d);
        any = false;
#pragma unroll
        for (int m = 0; m < N; ++m) {
            c[m] += d[m];
            al[m] = al[m] && c[m] < bound;
            any = any || al[m];
            tp[m] = al[m] ? y * W + clampi(x - dirmul(s, h[m].d0), 0, W - 1) : -1;
        }
        if (!__any(any)) return;
        cp.template ssdN<N>(S, tp, d);
#pragma unroll
        for (int m = 0; m < N; ++m) c[m] += d[m];
    }
};

// Bin-plane evaluators: eq. (1) as 16 x the bin-grid squared distance of the
// reference patch and the three target patches, with the same early-out and
// view order as the descriptor evaluators.  A patch is P = bin_pieces(C)
// pieces of 16 bytes, contiguous (4 entries of 4 plane rows; 4 pieces of
// packed bins for C = 3).
//
// BinLane: each lane gathers its own patches (fewest instructions and the
// shortest chain of round trips; for launches too small to fill the chip).
// BinCoop: the patches of a wave's owners are gathered cooperatively, as in
// Coop, so one wave-wide load reads the whole patches of a few owners instead
// of one piece each of 64 unrelated patches: the texture path handles about
// one 64-byte sector per clock per CU, and with the planes resident in the L2
// that, not the L2, bounds a full chip.  Owners without a target get an offset
// past the map's range (the load returns zeros without a memory access).
template <int C>
struct BinLane {
    static constexpr int P = bin_pieces(C);
    static constexpr int kOwners = 64;
    static constexpr int kLdsWords = 1;
    static constexpr int kPG = 1, kRG = 1;
    static constexpr bool kGroups = false;
    __amdgpu_buffer_rsrc_t rR, rT, rS, rX;
    BinAddr<C> addr;
    int H, W, s;
    BinRef<C> ref[P];

    __device__ __forceinline__ void setup(const MatchArgs& a, int b, int sd) {
        const Views v(a, b, sd);
        const uint32_t bytes = (uint32_t)a.img_bytes;
        rR = map_rsrc(v.R, bytes);
        rT = map_rsrc(v.T, bytes);
        rS = map_rsrc(v.S, bytes);
        rX = map_rsrc(v.X, bytes);
        H = a.H;
        W = a.W;
        s = sd;
        addr.sh = a.sh;
        addr.Hq = a.Hq;
        addr.RS = a.Wq * bin_entry_bytes(C);
    }

    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, int off, uint4* v) const {
#pragma unroll
        for (int k = 0; k < P; ++k)
            v[k] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16 * k, 0, 0));
    }

    template <class F>
    __device__ __forceinline__ void init(int x, int y, int, uint32_t*, F) {
        uint4 v[P];
        load(rR, addr(x, y), v);
#pragma unroll
        for (int k = 0; k < P; ++k) ref[k] = bin_ref<C>(v[k]);
    }

    __device__ __forceinline__ uint32_t view_cost(__amdgpu_buffer_rsrc_t rs, int X, int Y) const {
        uint4 v[P];
        load(rs, addr(X, Y), v);
        int acc = 0;
#pragma unroll
        for (int k = 0; k < P; ++k) acc = bin_piece_ssd<C>(ref[k], v[k], acc);
        return 16u * (uint32_t)acc;
    }

    __device__ __forceinline__ uint32_t cost_below(bool want, int x, int y, const Hyp& h,
                                                   uint32_t bound) {
        if (!want) return 0xFFFFFFFFu;
        const int ty = clampi(y + h.v, 0, H - 1);
        uint32_t c = view_cost(rX, clampi(x + h.u - dirmul(s, h.d1), 0, W - 1), ty);
        if (c >= bound) return c;
        c += view_cost(rT, clampi(x + h.u, 0, W - 1), ty);
        if (c >= bound) return c;
        return c + view_cost(rS, clampi(x - dirmul(s, h.d0), 0, W - 1), y);
    }

    template <int N>
    __device__ __forceinline__ void cost_belowN(const bool (&)[N], const Hyp (&)[N], int, int,
                                                uint32_t, uint32_t (&)[N]) {}
};

template <int C, int PG, int RG, int O = 64, bool XTS = false>
struct BinCoop {
    static_assert(O == 64 || O == 32 || O == 16, "owners per wave");
    static_assert(O * bin_pieces(C) % 64 == 0, "whole loads per gather");
    static constexpr int P = bin_pieces(C);
    static constexpr int K = O * P / 64;  // wave-wide loads per patch gather
    static constexpr int kOwners = O;
    static constexpr int kPG = PG, kRG = RG;
    static constexpr int kGroup = PG > RG ? PG : RG;
    static constexpr int kLdsWords = kGroup * 64 * K;
    static constexpr bool kGroups = true;
    __amdgpu_buffer_rsrc_t rR, rT, rS, rX;
    BinAddr<C> addr;
    int H, W, s;
    BinRef<C> refp[K];  // reference piece of slot k
    uint32_t* part;  // this wave's LDS slice
    int lane;

    __device__ __forceinline__ void setup(const MatchArgs& a, int b, int sd) {
        const Views v(a, b, sd);
        const uint32_t bytes = (uint32_t)a.img_bytes;
        rR = map_rsrc(v.R, bytes);
        rT = map_rsrc(v.T, bytes);
        rS = map_rsrc(v.S, bytes);
        rX = map_rsrc(v.X, bytes);
        H = a.H;
        W = a.W;
        s = sd;
        addr.sh = a.sh;
        addr.Hq = a.Hq;
        addr.RS = a.Wq * bin_entry_bytes(C);
    }

    __device__ __forceinline__ static int owner(int k, int l) { return (64 * k + l) / P; }
    __device__ __forceinline__ static int piece(int k, int l) { return (64 * k + l) % P; }

    // Offset of slot (k, lane): piece of its owner's patch at ob; an owner
    // without a target has ob = kNoTarget, and its slots, kNoTarget plus at
    // most 16 (P - 1) as unsigned 32-bit offsets, lie past every map's range
    // (maps are at most kNoTarget bytes), so their loads return zeros.
    __device__ __forceinline__ int slot_off(int ob, int k) const {
        return (int)((uint32_t)__shfl(ob, owner(k, lane)) + (uint32_t)(piece(k, lane) * 16));
    }

    template <class F>
    __device__ __forceinline__ void init(int x, int y, int l, uint32_t* lds, F) {
        lane = l;
        part = lds;
        const int ob = addr(x, y);
#pragma unroll
        for (int k = 0; k < K; ++k)
            refp[k] = bin_ref<C>(
                __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rR, slot_off(ob, k), 0, 0)));
    }

    // Squared distances (x 16) of N patches per owner, all gathers in flight
    // together; ob[m] = kNoTarget marks no target (result 0).  Must be called by all
    // lanes of the wave.
    // Patch m is read through rs_of(m) (views may differ between patches).
    template <int N, class RS>
    __device__ __forceinline__ void ssdN(RS rs_of, const int (&ob)[N], uint32_t (&c)[N]) {
        uint4 v[N][K];
        int so[N][K];
#pragma unroll
        for (int m = 0; m < N; ++m)
#pragma unroll
            for (int k = 0; k < K; ++k) so[m][k] = slot_off(ob[m], k);
#pragma unroll
        for (int m = 0; m < N; ++m)
#pragma unroll
            for (int k = 0; k < K; ++k)
                v[m][k] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs_of(m), so[m][k], 0, 0));
#pragma unroll
        for (int m = 0; m < N; ++m)
#pragma unroll
            for (int k = 0; k < K; ++k)
                part[64 * (m * K + k) + lane] = (uint32_t)bin_piece_ssd<C>(refp[k], v[m][k], 0);
        wave_sync();
        const int ol = lane & (O - 1);  // lanes past the owners read a valid slot
#pragma unroll
        for (int m = 0; m < N; ++m) {
            uint32_t t = 0;
#pragma unroll
            for (int w = 0; w < P; ++w) t += part[64 * K * m + ol * P + w];
            c[m] = ob[m] != kNoTarget ? 16u * t : 0u;
        }
        wave_sync();
    }

    // The cross, temporal and stereo distances (x 16) summed, of N candidates
    // per owner: the 3 N patches of ob (cross ones first, then temporal, then
    // stereo; a candidate without a target has kNoTarget in all three, result
    // 0) gathered together, and a slot's three pieces summed before the
    // partials go through LDS.  Must be called by all lanes of the wave.
    template <int N>
    __device__ __forceinline__ void ssd_views(const int (&ob)[3 * N], uint32_t (&c)[3 * N]) {
        uint4 v[3 * N][K];
        int so[3 * N][K];
#pragma unroll
        for (int m = 0; m < 3 * N; ++m)
#pragma unroll
            for (int k = 0; k < K; ++k) so[m][k] = slot_off(ob[m], k);
#pragma unroll
        for (int m = 0; m < 3 * N; ++m) {
            const __amdgpu_buffer_rsrc_t rs = m < N ? rX : m < 2 * N ? rT : rS;
#pragma unroll
            for (int k = 0; k < K; ++k)
                v[m][k] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, so[m][k], 0, 0));
        }
#pragma unroll
        for (int m = 0; m < N; ++m)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                int acc = bin_piece_ssd<C>(refp[k], v[m][k], 0);
                acc = bin_piece_ssd<C>(refp[k], v[N + m][k], acc);
                part[64 * (m * K + k) + lane] = (uint32_t)bin_piece_ssd<C>(refp[k], v[2 * N + m][k], acc);
            }
        wave_sync();
        const int ol = lane & (O - 1);  // lanes past the owners read a valid slot
#pragma unroll
        for (int m = 0; m < N; ++m) {
            uint32_t t = 0;
#pragma unroll
            for (int w = 0; w < P; ++w) t += part[64 * K * m + ol * P + w];
            c[m] = ob[m] != kNoTarget ? 16u * t : 0u;
        }
        wave_sync();
    }

    __device__ __forceinline__ uint32_t cost_below(bool want, int x, int y, const Hyp& h,
                                                   uint32_t bound) {
        bool w[1] = {want};
        Hyp hh[1] = {h};
        uint32_t c[1];
        cost_belowN<1>(w, hh, x, y, bound, c);
        return c[0];
    }

    // cost_below for N candidates of each lane, their gathers issued together
    // view by view with the early-out between views, or (XTS) all three views
    // in one round; same results as N calls with the same bound: a candidate
    // stopped at a view has a partial cost at or above the bound, one that
    // passes (or is scored in full) its exact cost.
    template <int N>
    __device__ __forceinline__ void cost_belowN(const bool (&w)[N], const Hyp (&h)[N], int x, int y,
                                                uint32_t bound, uint32_t (&c)[N]) {
        int ty[N], ob[N];
        bool al[N];
        bool any = false;
#pragma unroll
        for (int m = 0; m < N; ++m) {
            ty[m] = clampi(y + h[m].v, 0, H - 1);
            ob[m] = w[m] ? addr(clampi(x + h[m].u - dirmul(s, h[m].d1), 0, W - 1), ty[m]) : kNoTarget;
        }
        if constexpr (XTS) {
            int o3[3 * N];
            uint32_t c3[3 * N];
#pragma unroll
            for (int m = 0; m < N; ++m) {
                o3[m] = ob[m];
                o3[N + m] = w[m] ? addr(clampi(x + h[m].u, 0, W - 1), ty[m]) : kNoTarget;
                o3[2 * N + m] = w[m] ? addr(clampi(x - dirmul(s, h[m].d0), 0, W - 1), y) : kNoTarget;
            }
            ssd_views<N>(o3, c3);
#pragma unroll
            for (int m = 0; m < N; ++m) c[m] = c3[m];
            return;
        }
        ssdN<N>([&](int) { return rX; }, ob, c);
#pragma unroll
        for (int m = 0; m < N; ++m) {
            al[m] = w[m] && c[m] < bound;
            any = any || al[m];
            ob[m] = al[m] ? addr(clampi(x + h[m].u, 0, W - 1), ty[m]) : kNoTarget;
        }
        if (!__any(any)) return;
        uint32_t d[N];
        ssdN<N>([&](int) { return rT; }, ob, d);
        any = false;
#pragma unroll
        for (int m = 0; m < N; ++m) {
            c[m] += d[m];
            al[m] = al[m] && c[m] < bound;
            any = any || al[m];
            ob[m] = al[m] ? addr(clampi(x - dirmul(s, h[m].d0), 0, W - 1), y) : kNoTarget;
        }
        if (!__any(any)) return;
        ssdN<N>([&](int) { return rS; }, ob, d);
#pragma unroll
        for (int m = 0; m < N; ++m) c[m] += d[m];
    }
};

// mode: 0 = regular half-step; 1 = iteration-0 red half after a hand-off (own
// and neighbours from the coarse field); 2 = iteration-0 black half after a
// hand-off (own from the coarse field, neighbours already at this level);
// 3 = hand-off only (no propagation or search), used when iters == 0.
//
// Block = one wave: E::kOwners (64, or 32 for the smallest launches) pixels of
// the half-step's colour in one grid row (all pixels for mode 3).  Lanes past
// the row's end or past the owners stay in the wave (for the cooperative
// gathers) without a pixel of their own.  One-wave blocks let a
// finished wave's slot be refilled at once; the early-out makes wave times
// uneven (level 0 of the KITTI-size pair: 1.459 vs 1.482 ms per step with
// four-row blocks, level 2: 0.262 vs 0.286 ms).
template <int C, class E>
__global__ void __launch_bounds__(64) half_step_kernel(MatchArgs a, int it, int colour, int mode,
                                                       int tiles_x, int tiles_y) {
    __shared__ uint32_t part_lds[E::kLdsWords];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int per_field = tiles_x * tiles_y;
    const int z = tile / per_field;
    const int tr = tile - z * per_field;
    const int tx = tr / tiles_y, ty = tr - tx * tiles_y;
    const int lane = threadIdx.x;
    const int i = ty;
    const int par = mode == 3 ? 0 : ((i + colour) & 1);
    const int step = mode == 3 ? 1 : 2;
    constexpr int O = E::kOwners;
    const int j = step * (tx * O + lane) + par;
    const bool act = lane < O && j < a.Wk;
    const int di = z / a.batch, b = z - di * a.batch;
    const int s = (a.ndir == 2) ? (di == 0 ? 1 : -1) : a.dir0;
    E V;
    V.setup(a, b, s);
    const int n = a.n;
    const int x = n * min(j, a.Wk - 1), y = n * i;
    {
        const int j0 = step * tx * O + par, W = a.W, Wk1 = a.Wk - 1;
        V.init(x, y, lane, part_lds, [=](int o) { return y * W + n * min(j0 + step * o, Wk1); });
    }

    const size_t field_off = (size_t)z * a.Hk * a.Wk;
    const uint2* field = reinterpret_cast<const uint2*>(a.hyp) + field_off;
    const uint2* coarse = mode == 0 ? nullptr
                                    : reinterpret_cast<const uint2*>(a.hyp_coarse) +
                                          (size_t)z * a.Hc * a.Wc;
    const int jj = min(j, a.Wk - 1);
    const size_t o = (size_t)i * a.Wk + jj;

    Hyp best;
    uint32_t bestc;
    if (mode == 0) {
        best = unpack(field[o]);
        bestc = a.cost[field_off + o];
    } else {
        best = unpack(coarse[(size_t)(i >> 1) * a.Wc + (jj >> 1)]);
        bestc = V.cost_below(act, x, y, best, 0xFFFFFFFFu);
    }
    if (mode != 3) {
        // propagation: left, up, right, down.  A vector equal to one already
        // scored has the same cost and cannot be a strict improvement.
        const int ni[4] = {i, i - 1, i, i + 1};
        const int nj[4] = {jj - 1, jj, jj + 1, jj};
        uint2 nh[4];
        bool in[4];
        const uint2 own = pack(best);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            in[q] = act && ni[q] >= 0 && ni[q] < a.Hk && nj[q] >= 0 && nj[q] < a.Wk;
            nh[q] = own;
            if (in[q])
                nh[q] = mode == 1 ? coarse[(size_t)(ni[q] >> 1) * a.Wc + (nj[q] >> 1)]
                                  : field[(size_t)ni[q] * a.Wk + nj[q]];
        }
        bool want[4];
        Hyp hq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            bool dup = nh[q].x == own.x && nh[q].y == own.y;
#pragma unroll
            for (int p = 0; p < q; ++p) dup = dup || (in[p] && nh[q].x == nh[p].x && nh[q].y == nh[p].y);
            want[q] = in[q] && !dup;
            hq[q] = unpack(nh[q]);
        }
        // Candidates are accepted one after the other in their order.  The
        // cooperative evaluator scores a group at a time against the bound
        // from before the group: a later candidate rejected against that bound
        // is at least as costly as the updated best, and one scored below it
        // has its exact cost, so the results are those of one at a time, and
        // the group's gathers are in flight together instead of in sequence.
        auto take = [&](bool w, const Hyp& h, uint32_t c) {
            if (w && c < bestc) {
                bestc = c;
                best = h;
            }
        };
        constexpr int kPropGroup = E::kPG;
        if constexpr (E::kGroups) {
#pragma unroll
            for (int q0 = 0; q0 < 4; q0 += kPropGroup) {
                bool wg[kPropGroup];
                Hyp hg[kPropGroup];
                bool any = false;
#pragma unroll
                for (int m = 0; m < kPropGroup; ++m) {
                    wg[m] = want[q0 + m];
                    hg[m] = hq[q0 + m];
                    any = any || wg[m];
                }
                if (!__any(any)) continue;
                uint32_t c[kPropGroup];
                V.template cost_belowN<kPropGroup>(wg, hg, x, y, bestc, c);
#pragma unroll
                for (int m = 0; m < kPropGroup; ++m) take(wg[m], hg[m], c[m]);
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (!__any(want[q])) continue;
                take(want[q], hq[q], V.cost_below(want[q], x, y, hq[q], bestc));
            }
        }
        // random search around the propagated vector
        const Hyp centre = best;
        const uint64_t seed = a.seeds[b];
        const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
        auto draw = [&](int t, int col) {  // the Philox draws of sample t at grid column col
            U4 ctr;
            ctr.x = (uint32_t)(i * a.Wk + col);
            ctr.y = (uint32_t)it;
            ctr.z = ((uint32_t)a.level << 16) | ((uint32_t)t << 8) | (s < 0 ? 1u : 0u);
            ctr.w = 0u;
            return philox4x32_10(ctr, k0, k1);
        };
        auto offset = [&](int t, const U4& rnd) {
            const int r = max(1, a.rs_r0 >> t) * n;
            Hyp c;
            c.u = clampi(centre.u + uniform_offset(rnd.x, r), -a.fmax, a.fmax);
            c.v = clampi(centre.v + uniform_offset(rnd.y, r), -a.fmax, a.fmax);
            c.d0 = clampi(centre.d0 + uniform_offset(rnd.z, r), 0, a.dmax);
            c.d1 = clampi(centre.d1 + uniform_offset(rnd.w, r), 0, a.dmax);
            return c;
        };
        auto sample = [&](int t) { return offset(t, draw(t, jj)); };
        constexpr int kRS = E::kRG;
        for (int t = 0; t < a.rs_samples; t += kRS) {
            if (kRS > 1 && t + kRS <= a.rs_samples) {
                Hyp cg[kRS];
                bool wg[kRS];
                bool any = false;
                if constexpr (O < 64) {
                    // the lanes past the owners draw too: lane group g = lane / O
                    // draws sample t + LG p + g of owner lane mod O in pass p, and
                    // each owner collects its draws by shuffles (the same numbers,
                    // fewer Philox evaluations per lane)
                    constexpr int LG = 64 / O, NP = (kRS + LG - 1) / LG;
                    const int og = lane % O, grp = lane / O;
                    const int col = min(step * (tx * O + og) + par, a.Wk - 1);
                    U4 rr[NP];
#pragma unroll
                    for (int p = 0; p < NP; ++p) rr[p] = draw(t + LG * p + grp, col);
#pragma unroll
                    for (int m = 0; m < kRS; ++m) {
                        const int src = (m % LG) * O + og;
                        U4 d;
                        d.x = (uint32_t)__shfl((int)rr[m / LG].x, src);
                        d.y = (uint32_t)__shfl((int)rr[m / LG].y, src);
                        d.z = (uint32_t)__shfl((int)rr[m / LG].z, src);
                        d.w = (uint32_t)__shfl((int)rr[m / LG].w, src);
                        cg[m] = offset(t + m, d);
                    }
                } else {
#pragma unroll
                    for (int m = 0; m < kRS; ++m) cg[m] = sample(t + m);
                }
#pragma unroll
                for (int m = 0; m < kRS; ++m) {
                    wg[m] = act && !same(cg[m], centre);
                    any = any || wg[m];
                }
                if (!__any(any)) continue;
                uint32_t cc[kRS];
                if constexpr (E::kGroups) V.template cost_belowN<kRS>(wg, cg, x, y, bestc, cc);
#pragma unroll
                for (int m = 0; m < kRS; ++m) take(wg[m], cg[m], cc[m]);
            } else {
                for (int u = t; u < min(t + kRS, a.rs_samples); ++u) {
                    const Hyp c0 = sample(u);
                    const bool w0 = act && !same(c0, centre);
                    if (!__any(w0)) continue;
                    take(w0, c0, V.cost_below(w0, x, y, c0, bestc));
                }
            }
        }
    }
    if (act) {
        reinterpret_cast<uint2*>(a.hyp)[field_off + o] = pack(best);
        a.cost[field_off + o] = bestc;
    }
}

// Below this many pixel updates per launch (about a third of a wave per SIMD)
// each wave's chain of dependent gathers sets the time and the per-lane
// evaluator has the shorter chain.  Above it the cooperative one wins even
// with the chip far from full: level 2 of the KITTI-size pair (29,328 updates)
// takes 0.232 ms per step with it and 0.261 ms per lane.
constexpr long kCoopMinUpdates = 20000;

template <int C, class E>
sff_status launch_level(const MatchArgs& a, int iters, hipStream_t st) {
    const int nz = a.ndir * a.batch;
    const int tiles_y = a.Hk;
    const dim3 block(64);
    if (a.hyp_coarse && iters == 0) {
        const int tiles_x = (a.Wk + E::kOwners - 1) / E::kOwners;
        hipLaunchKernelGGL((half_step_kernel<C, E>), dim3(tiles_x * tiles_y * nz), block, 0, st, a,
                           0, 0, 3, tiles_x, tiles_y);
        return launch_status();
    }
    const int tiles_x = ((a.Wk + 1) / 2 + E::kOwners - 1) / E::kOwners;
    for (int it = 0; it < iters; ++it)
        for (int colour = 0; colour < 2; ++colour) {
            int mode = 0;
            if (a.hyp_coarse && it == 0) mode = colour == 0 ? 1 : 2;
            hipLaunchKernelGGL((half_step_kernel<C, E>), dim3(tiles_x * tiles_y * nz), block, 0, st,
                               a, it, colour, mode, tiles_x, tiles_y);
        }
    return launch_status();
}

// From this many pixel updates per launch the wider groups (4 neighbours,
// 3 samples) pay off; below it their registers cost more occupancy than the
// extra gathers in flight gain (measured at level 0 and 1 of the KITTI-size
// pair: 4/3 takes 1.48 vs 1.53 ms at level 0 and 0.49 vs 0.48 ms at level 1
// against 2/3; one candidate at a time 1.71 and 0.47 ms).
constexpr long kWideMinUpdates = 262144;

// Below this many pixel updates per launch a cooperative wave has 32 owners:
// twice the waves, half the gather registers (level 2 of the KITTI-size pair,
// 29,328 updates, 564 waves with 64 owners: 0.203 vs 0.236 ms per step;
// level 1, 116,936 updates: 0.471 vs 0.469 ms; level 0: 1.470 vs 1.442 ms).
constexpr long kHalfOwnersMaxUpdates = 50000;

// Largest descriptor map (bytes) the cooperative evaluators address.
constexpr size_t kMaxCoopMapBytes = 0x7FFFFFFF;

// SFF_MATCH_EVAL = "lane", "coop" (group sizes and owners by size),
// "coop-narrow", "coop-wide" (64 owners) or "coop-narrow-32", "coop-wide-32"
// (32 owners) forces an evaluator (all give identical results; the switch
// exists to test and time each one); anything else: auto.
template <int C>
sff_status run_level(const MatchArgs& a, int iters, hipStream_t st) {
    const long updates = (long)a.ndir * a.batch * a.Hk * ((a.Wk + 1) / 2);
    bool coop = updates >= kCoopMinUpdates, wide = updates >= kWideMinUpdates;
    bool half = updates < kHalfOwnersMaxUpdates;
    if (const char* e = std::getenv("SFF_MATCH_EVAL")) {
        if (std::strcmp(e, "lane") == 0) coop = false;
        if (std::strcmp(e, "coop") == 0) coop = true;
        if (std::strcmp(e, "coop-narrow") == 0) coop = true, wide = false, half = false;
        if (std::strcmp(e, "coop-wide") == 0) coop = true, wide = true, half = false;
        if (std::strcmp(e, "coop-narrow-32") == 0) coop = true, wide = false, half = true;
        if (std::strcmp(e, "coop-wide-32") == 0) coop = true, wide = true, half = true;
    }
    // The cooperative gathers address a map with 32-bit offsets.
    if (a.img_bytes > kMaxCoopMapBytes) coop = false;
    if (!coop) return launch_level<C, LaneEval<C>>(a, iters, st);
    if (half) {
        if (wide) return launch_level<C, CoopEval<C, 4, 3, 32>>(a, iters, st);
        return launch_level<C, CoopEval<C, 2, 3, 32>>(a, iters, st);
    }
    if (wide) return launch_level<C, CoopEval<C, 4, 3>>(a, iters, st);
    return launch_level<C, CoopEval<C, 2, 3>>(a, iters, st);
}

// From this many updates per half-step the bin matcher scores one candidate
// at a time with all three views per round (below: 4 neighbours and 3
// samples per group, 32 owners, view by view).
constexpr long kBinXtsMinUpdates = 262144;

// Bin-plane evaluators by launch size (updates per half-step), measured on the
// KITTI-size pair (C = 3, packed bins, fields on two streams from 100,000
// updates) with every shape giving identical fields; ms per level:
//  - level 2 (29,328 updates, under one wave per SIMD): all 4 neighbours and
//    all 6 samples in one group each, every view in one round, 16 owners per
//    wave: 0.16 (32 owners with the view-by-view early-out: 0.18; groups of
//    2 and 3 with 64 owners: 0.24) -- a lone wave's chain of dependent round
//    trips is what these launches wait on, so the fewest rounds and the most
//    waves win;
//  - level 1 (116,936 updates): groups of 4 neighbours and 3 samples, view by
//    view, 32 owners: 0.29 (one candidate with three views a round, 64
//    owners: 0.31);
//  - level 0 (465,750 updates): one candidate at a time with its three views
//    in one round, 64 owners: 0.73 (groups of 2 and 3 with the early-out:
//    0.73; 32 owners: 0.88-0.97).  This level is bound by the vector ALU
//    (unpacking and squared distances of the gathered pieces), and the
//    early-out rejects only ~15 % of candidates at the cross view, so a round
//    per view saves little.
// Other tile orders were slower (row-major 1.10 ms at level 0, no XCD
// grouping 1.37 ms, with unpacked patches).  Below 20,000 updates each lane
// gathers its own patches.  SFF_MATCH_EVAL = "lane", "coop" (2/3, 64 owners,
// early-out), "coop-32", "coop-43-32", "coop-46-32" (32 owners, early-out),
// "coop-xts" (1/1, 64 owners, three views a round) or "coop-46-16-xts" forces
// one (all give identical results; 16-owner shapes need 4 pieces a patch,
// C >= 2, and fall back to "coop-46-32" otherwise); anything else: auto.
template <int C>
sff_status launch_bin_pick(int pick, const MatchArgs& a, int iters, hipStream_t st) {
    switch (pick) {
        case 0: return launch_level<C, BinLane<C>>(a, iters, st);
        case 1: return launch_level<C, BinCoop<C, 2, 3>>(a, iters, st);
        case 2: return launch_level<C, BinCoop<C, 2, 3, 32>>(a, iters, st);
        case 3: return launch_level<C, BinCoop<C, 4, 3, 32>>(a, iters, st);
        case 5: return launch_level<C, BinCoop<C, 1, 1, 64, true>>(a, iters, st);
        case 6:
            if constexpr (16 * bin_pieces(C) % 64 == 0) return launch_level<C, BinCoop<C, 4, 6, 16, true>>(a, iters, st);
            break;
        default: break;
    }
    return launch_level<C, BinCoop<C, 4, 6, 32>>(a, iters, st);
}

// The forward and inverse fields of a level are independent (each reads only
// its own field and the read-only planes), so for large launches they run as
// two launch sequences on two streams: the caller's and a helper stream of
// the library, joined to the caller's by events before and after.  A launch
// that drains (its last waves finishing while most compute units idle) then
// overlaps the other field's launch instead of the next half-step waiting for
// it: level 0 of the KITTI-size pair 0.96 -> 0.82 ms, level 1 0.345 -> 0.334
// (measured with 18-operation unpacking); below ~100,000 updates (level 2:
// 0.167 vs 0.176 ms) one launch per half-step for both fields is faster.
// Identical fields either way.
constexpr long kSplitMinUpdates = 100000;

// SFF_MATCH_SPLIT = "0" or "1" forces one launch sequence for both fields or
// the two-stream split (identical results; the switch exists to test and time
// both); anything else: by launch size.
template <int C>
sff_status run_bin_level(const MatchArgs& a, int iters, hipStream_t st) {
    const long updates = (long)a.ndir * a.batch * a.Hk * ((a.Wk + 1) / 2);
    int pick = updates < kCoopMinUpdates         ? 0
               : updates < kHalfOwnersMaxUpdates ? 6
               : updates < kBinXtsMinUpdates     ? 3
                                                 : 5;
    bool split = a.ndir == 2 && updates >= kSplitMinUpdates;
    if (const char* e = std::getenv("SFF_MATCH_EVAL")) {
        if (std::strcmp(e, "lane") == 0) pick = 0;
        if (std::strcmp(e, "coop") == 0) pick = 1;
        if (std::strcmp(e, "coop-32") == 0) pick = 2;
        if (std::strcmp(e, "coop-43-32") == 0) pick = 3;
        if (std::strcmp(e, "coop-46-32") == 0) pick = 4;
        if (std::strcmp(e, "coop-xts") == 0) pick = 5;
        if (std::strcmp(e, "coop-46-16-xts") == 0) pick = 6;
    }
    if (const char* e = std::getenv("SFF_MATCH_SPLIT")) {
        if (std::strcmp(e, "0") == 0) split = false;
        if (std::strcmp(e, "1") == 0) split = a.ndir == 2;
    }
    if (!split) return launch_bin_pick<C>(pick, a, iters, st);
    // field 0 (forward) on the caller's stream, field 1 (inverse) on the helper
    MatchArgs f0 = a, f1 = a;
    f0.ndir = f1.ndir = 1;
    f0.dir0 = 1;
    f1.dir0 = -1;
    const size_t fine = (size_t)a.batch * a.Hk * a.Wk, coarse = (size_t)a.batch * a.Hc * a.Wc;
    f1.hyp = a.hyp + 4 * fine;
    f1.cost = a.cost + fine;
    if (a.hyp_coarse) f1.hyp_coarse = a.hyp_coarse + 4 * coarse;
    std::lock_guard<std::mutex> lock(helper_lock());
    HelperStream* hs = helper_for_current_device();
    if (!hs) return launch_bin_pick<C>(pick, a, iters, st);
    if (!helper_fork(hs, st)) return SFF_ERR_HIP;
    const sff_status r0 = launch_bin_pick<C>(pick, f0, iters, st);
    const sff_status r1 = launch_bin_pick<C>(pick, f1, iters, hs->stream);
    // join even after a launch error, so the caller's stream never runs ahead
    if (!helper_join(hs, st)) return SFF_ERR_HIP;
    return r0 != SFF_OK ? r0 : r1;
}

}  // namespace
}  // namespace sff

using namespace sff;

extern "C" sff_status sff_match_level(const sff_params* p, int32_t batch, int32_t dir,
                                      int32_t level, const int16_t* desc, const uint64_t* seeds,
                                      const int16_t* hyp_coarse, int16_t* hyp, uint32_t* cost,
                                      void* stream) {
    if (!params_ok(p) || batch < 1 || batch > 32767 || (dir != 1 && dir != -1 && dir != 0) ||
        level < 0 || level >= p->levels || !desc || !seeds || !hyp || !cost)
        return SFF_ERR_INVALID_ARG;
    if (hyp_coarse && level >= p->levels - 1) return SFF_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(desc) & 15) != 0 || (reinterpret_cast<uintptr_t>(hyp) & 7) != 0 ||
        (reinterpret_cast<uintptr_t>(cost) & 3) != 0 ||
        (reinterpret_cast<uintptr_t>(hyp_coarse) & 7) != 0)
        return SFF_ERR_INVALID_ARG;
    const LevelGeom g = level_geom(*p, level);
    const int ndir = dir == 0 ? 2 : 1;
    const size_t fine_bytes = (size_t)ndir * batch * g.Hk * g.Wk * 8;
    if (hyp_coarse) {
        const LevelGeom gc = level_geom(*p, level + 1);
        const size_t coarse_bytes = (size_t)ndir * batch * gc.Hk * gc.Wk * 8;
        const uintptr_t f0 = reinterpret_cast<uintptr_t>(hyp), f1 = f0 + fine_bytes;
        const uintptr_t c0 = reinterpret_cast<uintptr_t>(hyp_coarse), c1 = c0 + coarse_bytes;
        if (f0 < c1 && c0 < f1) return SFF_ERR_INVALID_ARG;
    }
    MatchArgs a;
    a.maps = reinterpret_cast<const uint8_t*>(desc);
    a.img_bytes = (size_t)p->H * p->W * rec_channels(p->C) * 32;
    a.sh = a.Hq = a.Wq = 0;
    a.seeds = seeds;
    a.hyp_coarse = hyp_coarse;
    a.hyp = hyp;
    a.cost = cost;
    a.H = p->H;
    a.W = p->W;
    a.n = g.n;
    a.level = level;
    a.Hk = g.Hk;
    a.Wk = g.Wk;
    if (hyp_coarse) {
        const LevelGeom gc = level_geom(*p, level + 1);
        a.Hc = gc.Hk;
        a.Wc = gc.Wk;
    } else {
        a.Hc = a.Wc = 0;
    }
    a.rs_r0 = p->rs_r0;
    a.rs_samples = p->rs_samples;
    a.fmax = p->fmax;
    a.dmax = p->dmax;
    a.batch = batch;
    a.ndir = ndir;
    a.dir0 = dir == 0 ? 1 : dir;
    hipStream_t st = as_stream(stream);
    switch (p->C) {
        case 1: return run_level<1>(a, p->iters, st);
        case 2: return run_level<2>(a, p->iters, st);
        case 3: return run_level<3>(a, p->iters, st);
        default: return run_level<4>(a, p->iters, st);
    }
}

extern "C" sff_status sff_match_level_bins(const sff_params* p, int32_t batch, int32_t dir,
                                           int32_t level, const uint16_t* bins, const uint64_t* seeds,
                                           const int16_t* hyp_coarse, int16_t* hyp, uint32_t* cost,
                                           void* stream) {
    if (!params_ok(p) || batch < 1 || batch > 32767 || (dir != 1 && dir != -1 && dir != 0) ||
        level < 0 || level >= p->levels || !bins || !seeds || !hyp || !cost)
        return SFF_ERR_INVALID_ARG;
    if (hyp_coarse && level >= p->levels - 1) return SFF_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(bins) & 15) != 0 || (reinterpret_cast<uintptr_t>(hyp) & 7) != 0 ||
        (reinterpret_cast<uintptr_t>(cost) & 3) != 0 ||
        (reinterpret_cast<uintptr_t>(hyp_coarse) & 7) != 0)
        return SFF_ERR_INVALID_ARG;
    const size_t img_bytes = bin_image_bytes(*p, level);
    if (img_bytes > (size_t)kNoTarget) return SFF_ERR_UNSUPPORTED;  // 32-bit gather offsets
    const LevelGeom g = level_geom(*p, level);
    const BinGeom bg = bin_geom(*p, level);
    const int ndir = dir == 0 ? 2 : 1;
    const size_t fine_bytes = (size_t)ndir * batch * g.Hk * g.Wk * 8;
    MatchArgs a;
    if (hyp_coarse) {
        const LevelGeom gc = level_geom(*p, level + 1);
        const size_t coarse_bytes = (size_t)ndir * batch * gc.Hk * gc.Wk * 8;
        const uintptr_t f0 = reinterpret_cast<uintptr_t>(hyp), f1 = f0 + fine_bytes;
        const uintptr_t c0 = reinterpret_cast<uintptr_t>(hyp_coarse), c1 = c0 + coarse_bytes;
        if (f0 < c1 && c0 < f1) return SFF_ERR_INVALID_ARG;
        a.Hc = gc.Hk;
        a.Wc = gc.Wk;
    } else {
        a.Hc = a.Wc = 0;
    }
    a.maps = reinterpret_cast<const uint8_t*>(bins);
    a.img_bytes = img_bytes;
    a.seeds = seeds;
    a.hyp_coarse = hyp_coarse;
    a.hyp = hyp;
    a.cost = cost;
    a.H = p->H;
    a.W = p->W;
    a.n = g.n;
    a.level = level;
    a.Hk = g.Hk;
    a.Wk = g.Wk;
    a.sh = bg.sh;
    a.Hq = bg.Hq;
    a.Wq = bg.Wq;
    a.rs_r0 = p->rs_r0;
    a.rs_samples = p->rs_samples;
    a.fmax = p->fmax;
    a.dmax = p->dmax;
    a.batch = batch;
    a.ndir = ndir;
    a.dir0 = dir == 0 ? 1 : dir;
    hipStream_t st = as_stream(stream);
    switch (p->C) {
        case 1: return run_bin_level<1>(a, p->iters, st);
        case 2: return run_bin_level<2>(a, p->iters, st);
        case 3: return run_bin_level<3>(a, p->iters, st);
        default: return run_bin_level<4>(a, p->iters, st);
    }
}
