// Device-side descriptor helpers of libsff: loading C x 16 int16 WHT
// coefficients and their exact squared distance with packed 16-bit subtracts
// and 2-way int16 dot products (v_pk_sub_i16, v_dot2c_i32_i16).
#pragma once

#include "sff_internal.hpp"

namespace sff {

typedef short short2v __attribute__((ext_vector_type(2)));

// Descriptor records are padded to a power-of-two channel count (1, 2, 4, 4
// for C = 1..4), so a record is 32, 64 or 128 bytes and, in a map aligned to
// 128 bytes, never straddles a cache line.  The padding is never read.
template <int C>
constexpr int kRecC = C == 3 ? 4 : C;

// C channels x 16 coefficients = 8 C packed int16 pairs.
template <int C>
struct Desc {
    uint32_t w[8 * C];
};

template <int C>
__device__ __forceinline__ Desc<C> load_desc(const int16_t* __restrict__ map, size_t pix) {
    const uint4* p = reinterpret_cast<const uint4*>(map + pix * (size_t)(16 * kRecC<C>));
    Desc<C> d;
#pragma unroll
    for (int k = 0; k < 2 * C; ++k) {
        const uint4 v = p[k];
        d.w[4 * k + 0] = v.x;
        d.w[4 * k + 1] = v.y;
        d.w[4 * k + 2] = v.z;
        d.w[4 * k + 3] = v.w;
    }
    return d;
}

// Squared distance of one 16-byte piece (8 coefficients) of two descriptors.
__device__ __forceinline__ int piece_ssd(uint4 a, uint4 b, int acc) {
    const uint32_t aw[4] = {a.x, a.y, a.z, a.w}, bw[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const short2v d = __builtin_bit_cast(short2v, aw[k]) - __builtin_bit_cast(short2v, bw[k]);
        acc = __builtin_amdgcn_sdot2(d, d, acc, false);
    }
    return acc;
}

// Squared distance of two descriptors.  Coefficients lie in [-16320, 16320],
// so each difference fits int16; by Parseval one channel contributes at most
// 64 * 64 * 255^2 < 2^28, four channels stay below 2^31.
template <int C>
__device__ __forceinline__ uint32_t desc_ssd(const Desc<C>& a, const Desc<C>& b) {
    int acc = 0;
#pragma unroll
    for (int k = 0; k < 8 * C; ++k) {
        const short2v d = __builtin_bit_cast(short2v, a.w[k]) - __builtin_bit_cast(short2v, b.w[k]);
        acc = __builtin_amdgcn_sdot2(d, d, acc, false);
    }
    return (uint32_t)acc;
}

// a * b + c on the 24-bit multiplier (full rate; the operands are below 2^24).
// Written out because the compiler otherwise forms a quarter-rate 64-bit
// multiply-add for it.
__device__ __forceinline__ uint32_t mad24(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t d;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// Byte offset of the patch of target (X, Y) (inside the image) in an image's
// bin planes.  An image is below 2^31 bytes and a plane row at least 128, so
// plane * Hq + row < 2^24, and so is the row stride Wq * entry bytes.
template <int C>
struct BinAddr {
    int sh, Hq, RS;  // RS = Wq * entry bytes
    __device__ __forceinline__ int operator()(int X, int Y) const {
        const uint32_t m = (1u << sh) - 1u, x = (uint32_t)X, y = (uint32_t)Y;
        const uint32_t plane = ((y & m) << sh) + (x & m);
        const uint32_t row = mad24(plane, (uint32_t)Hq, y >> sh);
        return (int)mad24(row, (uint32_t)RS, __umul24(x >> sh, (uint32_t)bin_entry_bytes(C)));
    }
};

// A 16-byte piece of a bin patch in the form its squared distances are taken
// from: as stored (8 uint16 bins) for C != 3; for C = 3 (one entry: four bins
// m = 0..3 of three 10-bit channels, packed as the bin planes store it)
// unpacked to six uint16 pairs.  The packing puts channel 0 of bins (0, 1) and
// (2, 3) and channel 1 of bins (0, 1) and (2, 3) in the low 10 bits of the two
// halves of words 0..3, and splits channel 2 of bins (0, 1) over the spare
// bits 10..15 of both halves of word 0 (low 6 bits) and word 1 (high 4), of
// bins (2, 3) over words 2 and 3; so each pair costs one mask, or two shifts
// and two masks for the channel-2 pairs.
template <int C>
struct BinRef {
    uint32_t w[4];
};
template <>
struct BinRef<3> {
    uint32_t w[6];
};

template <int C>
__device__ __forceinline__ BinRef<C> bin_ref(uint4 v) {
    BinRef<C> r;
    const uint32_t t[4] = {v.x, v.y, v.z, v.w};
    if constexpr (C == 3) {
#pragma unroll
        for (int m = 0; m < 4; ++m) r.w[m] = t[m] & 0x03FF03FFu;
        r.w[4] = ((t[0] >> 10) & 0x003F003Fu) | ((t[1] >> 4) & 0x03C003C0u);
        r.w[5] = ((t[2] >> 10) & 0x003F003Fu) | ((t[3] >> 4) & 0x03C003C0u);
    } else {
#pragma unroll
        for (int m = 0; m < 4; ++m) r.w[m] = t[m];
    }
    return r;
}

// acc + squared distance of two pieces (bins are at most 1020, so every
// difference fits int16).
template <int C>
__device__ __forceinline__ int bin_piece_ssd(const BinRef<C>& a, uint4 b, int acc) {
    const BinRef<C> u = bin_ref<C>(b);
    constexpr int NW = C == 3 ? 6 : 4;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const short2v d = __builtin_bit_cast(short2v, a.w[k]) - __builtin_bit_cast(short2v, u.w[k]);
        acc = __builtin_amdgcn_sdot2(d, d, acc, false);
    }
    return acc;
}

}  // namespace sff
