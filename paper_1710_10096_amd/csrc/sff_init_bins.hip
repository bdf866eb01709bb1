// Initialisation at the coarsest level (SceneFlowFields, Section 3.1,
// "Initialization") on the WHT bin-sum planes: exact nearest neighbours of
// each reference grid pixel's WHT descriptor among grid pixels of the temporal
// partner (box |u|,|v| <= fmax), the stereo partner (same row, 0 <= d0 <=
// dmax) and the cross partner (row y + v*, 0 <= d1 <= dmax), ties to the
// smallest target index; the combination's eq. (1) cost is stored with it.
// Same results as sff_init_nn on the level's descriptors.
//
// A descriptor's squared distance is 16 times that of its 4 x 4 grid of 2 x 2
// bin sums (16 C values, each 0..1020), so distances and their argmins are
// taken on the bin grids.  The temporal search is a dense contraction:
// |a - b|^2 = |a'|^2 + |b'|^2 - 2 a'.b' with the centred grids a' = a - 510,
// b' = b - 510 (|a'_k|, |b'_k| <= 510).  Candidates b' and queries -2 a' are
// exact in fp16, every partial sum of -2 a'.b' over at most 64 values is an
// even integer of magnitude below 2^25 and so exact in fp32: the fp16 MFMAs
// (16x16x32 with K = 16 C, zero-padded to a multiple of 32; 16x16x16 for
// C = 1) give -2 a'.b' exactly, and the argmin key |b'|^2 - 2 a'.b' =
// |a - b|^2 - |a'|^2 is one conversion and one add per candidate.
#include <climits>
#include <type_traits>

#include "sff_device.hpp"

namespace sff {
namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kQRows = 8;    // query rows per block (one 16-query MFMA tile each)
constexpr int kParts = 256 / (16 * kQRows);  // threads per query in the epipolar searches
constexpr int kWaves = 4;    // waves per block, splitting the candidate rows
constexpr int kCentre = 510;  // bins lie in 0..1020

// K = 16 C values per grid, taken as N32 chunks of 32 (16x16x32 MFMA) or, for
// C = 1, one chunk of 16 (16x16x16 MFMA); C = 3 is padded with zeros to 64.
// Only MFMAs of one shape are chained through an accumulator: a 16x16x32
// followed by a 16x16x16 reading its result (K = 48 exactly) gave wrong sums
// here when the two were issued back to back.
template <int C>
struct KSplit {
    static constexpr int K = 16 * C;
    static constexpr int N32 = C == 1 ? 0 : (K + 31) / 32, N16 = C == 1 ? 1 : 0;
    static constexpr int KP = 32 * N32 + 16 * N16;  // padded length
};

struct BinInitArgs {
    const uint8_t* bins;  // [batch][4] images of bin planes
    size_t img_bytes;
    int16_t* hyp;    // [ndir][batch][Hk][Wk][4]
    uint32_t* cost;  // [ndir][batch][Hk][Wk]
    int H, W, n, Hk, Wk, fm, dm;
    int sh, Hq, Wq;  // bin planes (BinGeom)
    int batch, dir0, ndir;
};

// Operand planes of the coarsest grid of all four views, z = pair * 4 + view,
// p = i * Wk + j, Nk = Hk * Wk:
//   c32[c][z][p][32], c16[z][p][16]: candidates b' (fp16), chunk c of K;
//   q32, q16: queries -2 a' (fp16), same layout;
//   sq[z][p] = |b'|^2; sqx[z][i][wx] the same norms as fp32 (exact) with column j at
//   offx + j and the edge values repeated over 16+ columns on either side, so
//   the 4 candidates of a lane are one aligned 16-byte load (offx = 16 +
//   (F mod 4) makes offx + c0 + 4g a multiple of 4 for every tile start
//   c0 = j0 - F + 16 t, j0 a multiple of 16).
struct OpPlanes {
    _Float16 *c32, *c16, *q32, *q16;
    uint32_t* sq;
    float* sqx;
    size_t nzk;  // nz * Nk
    int wx, offx;
};

__host__ __device__ inline int sqx_offset(int F) { return 16 + (F & 3); }
__host__ __device__ inline int sqx_width(int F, int Wk) { return (sqx_offset(F) + Wk + 16 + 3) & ~3; }

__device__ __forceinline__ __amdgpu_buffer_rsrc_t image_rsrc(const uint8_t* M, uint32_t bytes) {
    const uint64_t p = reinterpret_cast<uint64_t>(M);
    const uint64_t u = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)p) |
                       ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(p >> 32)) << 32);
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(u), (short)0,
                                             (int)__builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}

// The 16-byte pieces of the bin grid of (X, Y) as stored.
template <int C>
__device__ __forceinline__ void load_grid(__amdgpu_buffer_rsrc_t rs, int off, uint4 (&v)[bin_pieces(C)]) {
#pragma unroll
    for (int k = 0; k < bin_pieces(C); ++k)
        v[k] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16 * k, 0, 0));
}

template <int C>
__device__ __forceinline__ uint32_t grid_ssd(const uint4 (&a)[bin_pieces(C)], const uint4 (&b)[bin_pieces(C)]) {
    int acc = 0;
#pragma unroll
    for (int k = 0; k < bin_pieces(C); ++k) acc = bin_piece_ssd<C>(bin_ref<C>(a[k]), b[k], acc);
    return (uint32_t)acc;
}

// Bin value k of a grid as stored at g: uint16 k (entry k / 4C, plane row
// (k / C) mod 4, channel k mod C), or for C = 3 half k mod 2 of pair (k mod
// 12) / 2 of entry k / 12 as the matcher unpacks it; the operand planes take
// the values in this order (the same for queries and candidates).
template <int C>
__device__ __forceinline__ int grid_value(const uint8_t* g, int k) {
    if constexpr (C == 3) {
        const uint4 v = reinterpret_cast<const uint4*>(g)[k / 12];
        const BinRef<3> u = bin_ref<3>(v);
        return (int)((u.w[(k % 12) >> 1] >> (16 * (k & 1))) & 0xFFFFu);
    } else {
        return (int)reinterpret_cast<const uint16_t*>(g)[k];
    }
}

// One thread per (z, grid pixel): its bin grid into the operand planes.
template <int C>
__global__ void __launch_bounds__(256) op_planes_kernel(BinInitArgs a, OpPlanes P, int nz) {
    using KS = KSplit<C>;
    const int p = blockIdx.x * 256 + threadIdx.x;
    const int z = blockIdx.y;
    if (p >= a.Hk * a.Wk || z >= nz) return;
    const int i = p / a.Wk, j = p - i * a.Wk;
    BinAddr<C> addr;
    addr.sh = a.sh;
    addr.Hq = a.Hq;
    addr.RS = a.Wq * bin_entry_bytes(C);
    const uint8_t* g = a.bins + (size_t)z * a.img_bytes + addr(a.n * j, a.n * i);
    _Float16 b[KS::KP], q[KS::KP];
    uint32_t sq = 0;
#pragma unroll
    for (int k = 0; k < KS::KP; ++k) {
        const int v = k < KS::K ? grid_value<C>(g, k) - kCentre : 0;  // padding adds nothing
        sq += (uint32_t)(v * v);
        b[k] = (_Float16)v;
        q[k] = (_Float16)(-2 * v);
    }
    const size_t o = (size_t)z * a.Hk * a.Wk + p;
#pragma unroll
    for (int c = 0; c < KS::N32; ++c) {
        h8* cb = reinterpret_cast<h8*>(P.c32 + ((size_t)c * P.nzk + o) * 32);
        h8* cq = reinterpret_cast<h8*>(P.q32 + ((size_t)c * P.nzk + o) * 32);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            h8 vb, vq;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                vb[e] = b[32 * c + 8 * u + e];
                vq[e] = q[32 * c + 8 * u + e];
            }
            cb[u] = vb;
            cq[u] = vq;
        }
    }
    if constexpr (KS::N16 > 0) {
        h4* cb = reinterpret_cast<h4*>(P.c16 + o * 16);
        h4* cq = reinterpret_cast<h4*>(P.q16 + o * 16);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            h4 vb, vq;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                vb[e] = b[32 * KS::N32 + 4 * u + e];
                vq[e] = q[32 * KS::N32 + 4 * u + e];
            }
            cb[u] = vb;
            cq[u] = vq;
        }
    }
    P.sq[o] = sq;
    float* row = P.sqx + ((size_t)z * a.Hk + i) * P.wx;
    const float sqf = (float)sq;  // exact: below 2^24
    row[P.offx + j] = sqf;
    if (j == 0)
        for (int x = 0; x < P.offx; ++x) row[x] = sqf;
    if (j == a.Wk - 1)
        for (int x = P.offx + a.Wk; x < P.wx; ++x) row[x] = sqf;
}

// One block: kQRows rows x 16 consecutive columns of reference grid pixels of
// one field.  Wave w scans the candidate rows r = rlo + w (mod kWaves) of the
// union of the queries' boxes, 16 candidates per MFMA tile.
//
// MFMA operands: A (16 x K) holds candidates, lane l giving candidate l % 16;
// B (K x 16) holds queries, lane l giving query l % 16; both with the same K
// chunk for lane group l / 16 (8 values of a 32-chunk, 4 of a 16-chunk), so
// each product sums over all K values.  Lane l receives D[4 (l / 16) + e]
// [l % 16], e = 0..3: candidates 4 g + e of the tile against its own query.
//
// K > 1 (initialisation with K temporal leaves): each lane keeps its K best
// (key, target index) per query, sorted (a candidate enters after kept ones of
// equal key, which have smaller indices); the lists are merged per query in
// LDS, each leaf gets its own cross-row search, and the combination with the
// smallest T + S + X distance wins (the earlier leaf on ties).
template <int C, int K>
__global__ void __launch_bounds__(256) init_bins_kernel(BinInitArgs a, OpPlanes P) {
    using KS = KSplit<C>;
    __shared__ unsigned long long red[kWaves * 4][kQRows][16][K];
    __shared__ int res_u[kQRows][16][K], res_v[kQRows][16][K];
    __shared__ uint32_t res_t[kQRows][16][K];
    __shared__ int res_n[kQRows][16];
    __shared__ unsigned long long red2[kParts][kQRows][16];
    __shared__ unsigned long long redx[K][kParts][kQRows][16];
    const int lane = threadIdx.x & 63, w = wave_id();
    const int nq = lane & 15, g = lane >> 4;
    const int j0 = blockIdx.x * 16, i0 = blockIdx.y * kQRows;
    const int z = blockIdx.z;  // dir_index * batch + b
    const int di = z / a.batch, b = z - di * a.batch;
    const int s = (a.ndir == 2) ? (di == 0 ? 1 : -1) : a.dir0;
    const int Hk = a.Hk, Wk = a.Wk, n = a.n;
    const int F = a.fm / n;
    const int vR = s > 0 ? 0 : 3, vT = s > 0 ? 1 : 2, vS = s > 0 ? 2 : 1, vX = s > 0 ? 3 : 0;
    const size_t Nk = (size_t)Hk * Wk;
    const size_t zR = ((size_t)b * 4 + vR) * Nk, zT = ((size_t)b * 4 + vT) * Nk;
    const size_t zTx = ((size_t)b * 4 + vT) * Hk;  // row index base in sqx

    const uint8_t* base = a.bins + (size_t)b * 4 * a.img_bytes;
    const uint32_t ib = (uint32_t)a.img_bytes;
    BinAddr<C> addr;
    addr.sh = a.sh;
    addr.Hq = a.Hq;
    addr.RS = a.Wq * bin_entry_bytes(C);

    // queries (B operands), one 16-column tile per query row
    h8 q32[kQRows][KS::N32 > 0 ? KS::N32 : 1];
    h4 q16[kQRows];
    int best[kQRows], btile[kQRows];   // K = 1: minimum key and its first tile
    int tk[kQRows][K], ti[kQRows][K];  // K > 1: sorted keys and target indices
    const int jq = min(j0 + nq, Wk - 1);
#pragma unroll
    for (int t = 0; t < kQRows; ++t) {
        const size_t o = zR + (size_t)min(i0 + t, Hk - 1) * Wk + jq;
#pragma unroll
        for (int c = 0; c < KS::N32; ++c)
            q32[t][c] = *reinterpret_cast<const h8*>(P.q32 + ((size_t)c * P.nzk + o) * 32 + 8 * g);
        if constexpr (KS::N16 > 0) q16[t] = *reinterpret_cast<const h4*>(P.q16 + o * 16 + 4 * g);
    }
    // Scan: per query only the minimum key over this lane's candidates and the
    // first tile (in increasing target index) that reaches it are kept; the
    // target inside that tile is recovered afterwards.
    const int rlo = max(0, i0 - F), rhi = min(Hk - 1, i0 + kQRows - 1 + F);
    const int nct = (16 + 2 * F + 15) / 16;
    const int ct_lo = max(0, (F - j0) >> 4);                 // first c0 + 15 >= 0
    const int ct_hi = min(nct - 1, (Wk - 1 - j0 + F) >> 4);  // last c0 < Wk
    const int ntl = ct_hi - ct_lo + 1;
    const int nrw = rlo + w <= rhi ? (rhi - rlo - w) / kWaves + 1 : 0;
    const int total = ntl > 0 ? nrw * ntl : 0;

    struct Tile {
        h8 a32[KS::N32 > 0 ? KS::N32 : 1];
        h4 a16;
        float bsq[4];  // |b'|^2, exact in fp32 (below 2^24)
    };
    // Loads of tile (r, ct); the scan issues those of the next tile before it
    // scores the current one.
    auto load_tile = [&](int r, int ct) {
        Tile T;
        const size_t rowT = zT + (size_t)r * Wk;
        const int c0 = j0 - F + 16 * ct;
        const size_t oa = rowT + clampi(c0 + nq, 0, Wk - 1);
#pragma unroll
        for (int c = 0; c < KS::N32; ++c)
            T.a32[c] = *reinterpret_cast<const h8*>(P.c32 + ((size_t)c * P.nzk + oa) * 32 + 8 * g);
        if constexpr (KS::N16 > 0) T.a16 = *reinterpret_cast<const h4*>(P.c16 + oa * 16 + 4 * g);
        const float4 q = *reinterpret_cast<const float4*>(P.sqx + (zTx + (size_t)r) * P.wx + P.offx + c0 + 4 * g);
        T.bsq[0] = q.x;
        T.bsq[1] = q.y;
        T.bsq[2] = q.z;
        T.bsq[3] = q.w;
        return T;
    };
    // The scan, with keys as fp32 (the fast form) or as int32 (exact for any
    // key).  An fp32 key is the correctly rounded sum of two exact terms, so
    // it is exact whenever the key is below 2^24 in magnitude, and a key at or
    // above 2^24 rounds to a value at or above 2^24: the kept minimum (or the
    // K kept keys) and their order are exact unless one of them is at or above
    // 2^24, and then the block scans again with int32 keys.
    auto run_scan = [&](auto key_tag, auto& S) {
        using KT = decltype(key_tag);
        constexpr bool kFloat = std::is_same<KT, float>::value;
        const KT kNone = kFloat ? (KT)__builtin_huge_valf() : (KT)INT_MAX;
#pragma unroll
        for (int t = 0; t < kQRows; ++t) {
            S.best[t] = kNone;
            S.btile[t] = 0;
#pragma unroll
            for (int l = 0; l < K; ++l) {
                S.tk[t][l] = kNone;
                S.ti[t][l] = 0;
            }
        }
        Tile ta{}, tb{};
        int r = rlo + w, ct = ct_lo;
        if (total > 0) ta = load_tile(r, ct);
        auto scan_one = [&](const Tile& cur, Tile& nxt, int q) {
            int rn = r, ctn = ct + 1;
            if (ctn > ct_hi) {
                ctn = ct_lo;
                rn += kWaves;
            }
            if (q + 1 < total) nxt = load_tile(rn, ctn);
            const int c0 = j0 - F + 16 * ct;
            const int tile_id = (r << 16) | ct;
            // every query row of the block has row r inside its box (wave-uniform)
            const bool all_rows = i0 + kQRows - 1 < Hk && r >= i0 + kQRows - 1 - F && r <= i0 + F;
            // Keys of one tile for every query row.  Candidates outside the image
            // or this lane's query box get INT_MAX (above any true key); interior
            // tiles (every candidate inside every query's box) and rows inside
            // every query row's box skip those tests.  Both conditions are
            // wave-uniform.
            auto score = [&](auto interior, auto rows_in) {
                constexpr bool kInterior = decltype(interior)::value;
                constexpr bool kRowsIn = decltype(rows_in)::value;
                bool ok[4] = {true, true, true, true};
                // fp32 keys: a candidate outside the box or the image gets an
                // infinite norm once per tile, so its keys come out infinite
                // (the kNone of this form) in every row without a select each
                float bq[4] = {cur.bsq[0], cur.bsq[1], cur.bsq[2], cur.bsq[3]};
                if constexpr (!kInterior) {
    #pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int jc = c0 + 4 * g + e;
                        ok[e] = (unsigned)(jc - jq + F) <= (unsigned)(2 * F) && (unsigned)jc < (unsigned)Wk;
                        if constexpr (kFloat) bq[e] = ok[e] ? bq[e] : __builtin_huge_valf();
                    }
                }
    #pragma unroll
                for (int t = 0; t < kQRows; ++t) {
                    if constexpr (!kRowsIn) {
                        const int iq = i0 + t;
                        if (iq >= Hk || r < iq - F || r > iq + F) continue;
                    }
                    f4 acc = {0.f, 0.f, 0.f, 0.f};
    #pragma unroll
                    for (int c = 0; c < KS::N32; ++c)
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(cur.a32[c], q32[t][c], acc, 0, 0, 0);
                    if constexpr (KS::N16 > 0)
                        acc = __builtin_amdgcn_mfma_f32_16x16x16f16(cur.a16, q16[t], acc, 0, 0, 0);
                    KT k[4];
    #pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        // |b'|^2 + (-2 a'.b'), the product exact in fp32
                        if constexpr (kFloat) {
                            k[e] = bq[e] + acc[e];
                        } else {
                            k[e] = (int)cur.bsq[e] + (int)acc[e];
                            if constexpr (!kInterior) k[e] = ok[e] ? k[e] : kNone;
                        }
                    }
                    if constexpr (K == 1) {
                        // the running minimum folded in (two 3-input minima), the
                        // tile recorded when it strictly decreases
                        const KT nb = min(min(S.best[t], k[0]), min(min(k[1], k[2]), k[3]));
                        S.btile[t] = nb < S.best[t] ? tile_id : S.btile[t];
                        S.best[t] = nb;
                    } else {
    #pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            if (!__any(k[e] < S.tk[t][K - 1])) continue;  // wave-uniform
                            KT nk = k[e];
                            int ni = r * Wk + c0 + 4 * g + e;
    #pragma unroll
                            for (int l = 0; l < K; ++l) {
                                const bool lt = nk < S.tk[t][l];
                                const KT ok_ = S.tk[t][l];
                                const int oi = S.ti[t][l];
                                S.tk[t][l] = lt ? nk : ok_;
                                S.ti[t][l] = lt ? ni : oi;
                                nk = lt ? ok_ : nk;
                                ni = lt ? oi : ni;
                            }
                        }
                    }
                }
            };
            const bool interior = c0 >= 0 && c0 + 15 < Wk && c0 >= j0 + 15 - F && c0 + 15 <= j0 + F;
            if (interior) {
                if (all_rows)
                    score(std::true_type{}, std::true_type{});
                else
                    score(std::true_type{}, std::false_type{});
            } else {
                if (all_rows)
                    score(std::false_type{}, std::true_type{});
                else
                    score(std::false_type{}, std::false_type{});
            }
            r = rn;
            ct = ctn;
        };
        for (int q = 0; q < total; q += 2) {
            scan_one(ta, tb, q);
            if (q + 1 < total) scan_one(tb, ta, q + 1);
        }
    };
    struct StateF {
        float best[kQRows];
        int btile[kQRows];
        float tk[kQRows][K];
        int ti[kQRows][K];
    } SF;
    run_scan(0.f, SF);
    bool redo = false;
    const float kExact = 16777216.f;  // 2^24
#pragma unroll
    for (int t = 0; t < kQRows; ++t) {
        if constexpr (K == 1) redo = redo || (SF.best[t] >= kExact && SF.best[t] != __builtin_huge_valf());
#pragma unroll
        for (int l = 0; l < K; ++l)
            if constexpr (K > 1) redo = redo || (SF.tk[t][l] >= kExact && SF.tk[t][l] != __builtin_huge_valf());
    }
    if (__syncthreads_or(redo)) {
        struct StateI {
            int best[kQRows];
            int btile[kQRows];
            int tk[kQRows][K];
            int ti[kQRows][K];
        } SI;
        run_scan(0, SI);
#pragma unroll
        for (int t = 0; t < kQRows; ++t) {
            best[t] = SI.best[t];
            btile[t] = SI.btile[t];
#pragma unroll
            for (int l = 0; l < K; ++l) {
                tk[t][l] = SI.tk[t][l];
                ti[t][l] = SI.ti[t][l];
            }
        }
    } else {
#pragma unroll
        for (int t = 0; t < kQRows; ++t) {
            best[t] = SF.best[t] == __builtin_huge_valf() ? INT_MAX : (int)SF.best[t];
            btile[t] = SF.btile[t];
#pragma unroll
            for (int l = 0; l < K; ++l) {
                tk[t][l] = SF.tk[t][l] == __builtin_huge_valf() ? INT_MAX : (int)SF.tk[t][l];
                ti[t][l] = SF.ti[t][l];
            }
        }
    }
    // the smallest target index of the winning tile that reaches the minimum
    // (exact bin-grid squared distances, equal to the MFMA identity's)
    const __amdgpu_buffer_rsrc_t rR = image_rsrc(base + (size_t)vR * a.img_bytes, ib);
    const __amdgpu_buffer_rsrc_t rT = image_rsrc(base + (size_t)vT * a.img_bytes, ib);
    const __amdgpu_buffer_rsrc_t rS = image_rsrc(base + (size_t)vS * a.img_bytes, ib);
    const __amdgpu_buffer_rsrc_t rX = image_rsrc(base + (size_t)vX * a.img_bytes, ib);
#pragma unroll 1
    for (int t = 0; t < kQRows; ++t) {
        if constexpr (K > 1) {
            const uint32_t asq = P.sq[zR + (size_t)min(i0 + t, Hk - 1) * Wk + jq];
#pragma unroll
            for (int l = 0; l < K; ++l)
                red[w * 4 + g][t][nq][l] =
                    tk[t][l] == INT_MAX
                        ? ~0ull
                        : ((unsigned long long)((uint32_t)tk[t][l] + asq) << 32) | (uint32_t)ti[t][l];
            continue;
        }
        uint32_t bssd = 0xFFFFFFFFu, bidx = 0;
        if (best[t] != INT_MAX) {
            const int r = btile[t] >> 16, c0 = j0 - F + 16 * (btile[t] & 0xFFFF);
            uint4 qg[bin_pieces(C)];
            load_grid<C>(rR, addr(n * jq, n * min(i0 + t, Hk - 1)), qg);
            const uint32_t asq = P.sq[zR + (size_t)min(i0 + t, Hk - 1) * Wk + jq];
            bssd = (uint32_t)best[t] + asq;
            bool found = false;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int jc = c0 + 4 * g + e;
                const bool ok = (unsigned)(jc - jq + F) <= (unsigned)(2 * F) && (unsigned)jc < (unsigned)Wk;
                if (ok && !found) {
                    uint4 cg[bin_pieces(C)];
                    load_grid<C>(rT, addr(n * jc, n * r), cg);
                    if (grid_ssd<C>(qg, cg) == bssd) {
                        found = true;
                        bidx = (uint32_t)(r * Wk + jc);
                    }
                }
            }
        }
        red[w * 4 + g][t][nq][0] = ((unsigned long long)bssd << 32) | bidx;
    }
    __syncthreads();
    // combine the 16 partial lists (waves x lane groups) of each query: the K
    // smallest (ssd, index) keys, by K selection passes (indices are distinct)
    if (threadIdx.x < kQRows * 16) {
        const int t = threadIdx.x >> 4, q = threadIdx.x & 15;
        unsigned long long prev = 0;
        int nl = 0;
#pragma unroll 1
        for (int l = 0; l < K; ++l) {
            unsigned long long m = ~0ull;
            for (int k = 0; k < kWaves * 4; ++k)
#pragma unroll
                for (int e = 0; e < K; ++e) {
                    const unsigned long long v = red[k][t][q][e];
                    if ((l == 0 || v > prev) && v < m) m = v;
                }
            if (m == ~0ull) break;
            const uint32_t idx = (uint32_t)m;
            const int ri = (int)(idx / (uint32_t)Wk), rj = (int)(idx % (uint32_t)Wk);
            res_v[t][q][l] = n * (ri - (i0 + t));
            res_u[t][q][l] = n * (rj - min(j0 + q, Wk - 1));
            res_t[t][q][l] = (uint32_t)(m >> 32);
            prev = m;
            nl = l + 1;
        }
        res_n[t][q] = nl;
    }
    __syncthreads();

    // epipolar searches: kParts threads per query, candidates interleaved
    const int q = threadIdx.x & 15, t = (threadIdx.x >> 4) % kQRows, part = threadIdx.x / (16 * kQRows);
    const int iq = i0 + t, jqq = j0 + q;
    const bool live = iq < Hk && jqq < Wk;
    const int x = n * min(jqq, Wk - 1), y = n * min(iq, Hk - 1);
    uint4 qg[bin_pieces(C)];
    load_grid<C>(rR, addr(x, y), qg);
    const int W = a.W;
    // stereo partner on row y: target tx = x - s d0, increasing tx
    unsigned long long kS = ~0ull;
    if (live) {
        const int txlo = s > 0 ? x - min(a.dm, x) : x;
        const int txhi = s > 0 ? x : x + min(a.dm, ((W - 1 - x) / n) * n);
        for (int tx = txlo + n * part; tx <= txhi; tx += kParts * n) {
            uint4 cg[bin_pieces(C)];
            load_grid<C>(rS, addr(tx, y), cg);
            const unsigned long long k = ((unsigned long long)grid_ssd<C>(qg, cg) << 32) | (uint32_t)tx;
            kS = k < kS ? k : kS;
        }
    }
    red2[part][t][q] = kS;
    __syncthreads();
    unsigned long long mS = red2[0][t][q];
#pragma unroll
    for (int k = 1; k < kParts; ++k) mS = red2[k][t][q] < mS ? red2[k][t][q] : mS;
    __syncthreads();
    // cross partner of each temporal leaf on row y + v: target tx = x + u - s d1,
    // increasing tx
    const int nl = live ? res_n[t][q] : 0;
#pragma unroll 1
    for (int l = 0; l < K; ++l) {
        unsigned long long kX = ~0ull;
        if (l < nl) {
            const int xc = x + res_u[t][q][l], yc = y + res_v[t][q][l];
            const int txlo = s > 0 ? xc - min(a.dm, xc) : xc;
            const int txhi = s > 0 ? xc : xc + min(a.dm, ((W - 1 - xc) / n) * n);
            for (int tx = txlo + n * part; tx <= txhi; tx += kParts * n) {
                uint4 cg[bin_pieces(C)];
                load_grid<C>(rX, addr(tx, yc), cg);
                const unsigned long long k = ((unsigned long long)grid_ssd<C>(qg, cg) << 32) | (uint32_t)tx;
                kX = k < kX ? k : kX;
            }
        }
        redx[l][part][t][q] = kX;
    }
    __syncthreads();
    if (part != 0 || !live) return;
    // the cheapest combination (every target lies inside the image, so its
    // eq. (1) cost is 16 x the sum of the three bin-grid distances); the
    // earlier leaf on ties
    const uint32_t eS = (uint32_t)(mS >> 32);
    uint64_t bestJ = ~0ull;
    int bu = 0, bv = 0, bd1 = 0;
    for (int l = 0; l < nl; ++l) {
        unsigned long long mX = redx[l][0][t][q];
#pragma unroll
        for (int k = 1; k < kParts; ++k) mX = redx[l][k][t][q] < mX ? redx[l][k][t][q] : mX;
        const uint64_t joint = (uint64_t)res_t[t][q][l] + eS + (uint32_t)(mX >> 32);
        if (joint < bestJ) {
            bestJ = joint;
            bu = res_u[t][q][l];
            bv = res_v[t][q][l];
            bd1 = s * (x + bu - (int)(uint32_t)mX);
        }
    }
    const int bd0 = s * (x - (int)(uint32_t)mS);
    const size_t o = ((size_t)z * Hk + iq) * Wk + jqq;
    uint2 hv;
    hv.x = (uint32_t)(uint16_t)(int16_t)bu | ((uint32_t)(uint16_t)(int16_t)bv << 16);
    hv.y = (uint32_t)(uint16_t)(int16_t)bd0 | ((uint32_t)(uint16_t)(int16_t)bd1 << 16);
    reinterpret_cast<uint2*>(a.hyp)[o] = hv;
    a.cost[o] = 16u * (uint32_t)bestJ;
}

template <int C>
void launch_init_bins(int leaves, dim3 grid, hipStream_t st, const BinInitArgs& a, const OpPlanes& P) {
    switch (leaves) {
        case 1: hipLaunchKernelGGL((init_bins_kernel<C, 1>), grid, dim3(256), 0, st, a, P); break;
        case 2: hipLaunchKernelGGL((init_bins_kernel<C, 2>), grid, dim3(256), 0, st, a, P); break;
        default: hipLaunchKernelGGL((init_bins_kernel<C, 4>), grid, dim3(256), 0, st, a, P); break;
    }
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct OpWs {
    size_t c32, c16, q32, q16, sq, sqx, total;
    int wx, offx;
    size_t nzk;
};

OpWs op_ws(const sff_params& p, int batch) {
    const LevelGeom g = level_geom(p, p.levels - 1);
    const size_t nzk = (size_t)batch * 4 * g.Hk * g.Wk;
    const int n32 = p.C == 1 ? 0 : (16 * p.C + 31) / 32, n16 = p.C == 1 ? 1 : 0;
    OpWs L;
    L.nzk = nzk;
    L.c32 = 0;
    L.c16 = L.c32 + align256(nzk * 64 * n32);
    L.q32 = L.c16 + align256(nzk * 32 * n16);
    L.q16 = L.q32 + align256(nzk * 64 * n32);
    L.sq = L.q16 + align256(nzk * 32 * n16);
    L.sqx = L.sq + align256(nzk * sizeof(uint32_t));
    const int F = p.fmax / g.n;
    L.offx = sqx_offset(F);
    L.wx = sqx_width(F, g.Wk);
    L.total = L.sqx + align256((size_t)batch * 4 * g.Hk * L.wx * sizeof(uint32_t));
    return L;
}

}  // namespace
}  // namespace sff

using namespace sff;

extern "C" size_t sff_init_bins_workspace_bytes(const sff_params* p, int32_t batch) {
    if (!params_ok(p) || batch < 1 || batch > 32767) return 0;
    return op_ws(*p, batch).total;
}

extern "C" sff_status sff_init_nn_bins(const sff_params* p, int32_t batch, int32_t dir,
                                       int32_t leaves, const uint16_t* bins, int16_t* hyp,
                                       uint32_t* cost, void* workspace, size_t workspace_bytes,
                                       void* stream) {
    if (!params_ok(p) || batch < 1 || batch > 32767 || (dir != 1 && dir != -1 && dir != 0) ||
        !bins || !hyp || !cost || leaves < 1)
        return SFF_ERR_INVALID_ARG;
    if (leaves != 1 && leaves != 2 && leaves != 4) return SFF_ERR_UNSUPPORTED;
    if ((reinterpret_cast<uintptr_t>(bins) & 15) != 0 || (reinterpret_cast<uintptr_t>(hyp) & 7) != 0 ||
        (reinterpret_cast<uintptr_t>(cost) & 3) != 0)
        return SFF_ERR_INVALID_ARG;
    const int level = p->levels - 1;
    const size_t img_bytes = bin_image_bytes(*p, level);
    if (img_bytes > 0x7FFFFFF0u) return SFF_ERR_UNSUPPORTED;  // 32-bit gather offsets
    const OpWs L = op_ws(*p, batch);
    if (!workspace || workspace_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return SFF_ERR_WORKSPACE;
    const LevelGeom g = level_geom(*p, level);
    const BinGeom bg = bin_geom(*p, level);
    BinInitArgs a;
    a.bins = reinterpret_cast<const uint8_t*>(bins);
    a.img_bytes = img_bytes;
    a.hyp = hyp;
    a.cost = cost;
    a.H = p->H;
    a.W = p->W;
    a.n = g.n;
    a.Hk = g.Hk;
    a.Wk = g.Wk;
    a.fm = (p->fmax / g.n) * g.n;
    a.dm = (p->dmax / g.n) * g.n;
    a.sh = bg.sh;
    a.Hq = bg.Hq;
    a.Wq = bg.Wq;
    a.batch = batch;
    a.ndir = dir == 0 ? 2 : 1;
    a.dir0 = dir == 0 ? 1 : dir;
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    OpPlanes P;
    P.c32 = reinterpret_cast<_Float16*>(ws + L.c32);
    P.c16 = reinterpret_cast<_Float16*>(ws + L.c16);
    P.q32 = reinterpret_cast<_Float16*>(ws + L.q32);
    P.q16 = reinterpret_cast<_Float16*>(ws + L.q16);
    P.sq = reinterpret_cast<uint32_t*>(ws + L.sq);
    P.sqx = reinterpret_cast<float*>(ws + L.sqx);
    P.nzk = L.nzk;
    P.wx = L.wx;
    P.offx = L.offx;
    const int nz4 = 4 * batch;
    const dim3 sgrid((g.Hk * g.Wk + 255) / 256, nz4);
    const dim3 grid((g.Wk + 15) / 16, (g.Hk + kQRows - 1) / kQRows, a.ndir * batch);
    hipStream_t st = as_stream(stream);
    switch (p->C) {
        case 1:
            hipLaunchKernelGGL(op_planes_kernel<1>, sgrid, dim3(256), 0, st, a, P, nz4);
            launch_init_bins<1>(leaves, grid, st, a, P);
            break;
        case 2:
            hipLaunchKernelGGL(op_planes_kernel<2>, sgrid, dim3(256), 0, st, a, P, nz4);
            launch_init_bins<2>(leaves, grid, st, a, P);
            break;
        case 3:
            hipLaunchKernelGGL(op_planes_kernel<3>, sgrid, dim3(256), 0, st, a, P, nz4);
            launch_init_bins<3>(leaves, grid, st, a, P);
            break;
        default:
            hipLaunchKernelGGL(op_planes_kernel<4>, sgrid, dim3(256), 0, st, a, P, nz4);
            launch_init_bins<4>(leaves, grid, st, a, P);
            break;
    }
    return launch_status();
}
