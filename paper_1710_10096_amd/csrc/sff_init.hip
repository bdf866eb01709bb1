// Initialisation at the coarsest level (SceneFlowFields, Section 3.1,
// "Initialization"): exact nearest neighbours of each reference grid pixel's
// WHT descriptor among grid pixels of the temporal partner (box |u|,|v| <=
// fmax), the stereo partner (same row, 0 <= d0 <= dmax) and the cross partner
// (row y + v*, 0 <= d1 <= dmax), ties to the smallest target index; the
// combination's eq. (1) cost is stored with it.
//
// The temporal search is a dense contraction: for a query descriptor a and a
// candidate b, |a - b|^2 = |a|^2 + |b|^2 - 2 a.b.  It runs on int8 MFMA with
// every int16 coefficient split exactly into a = 256 a_h + a_l (a_l in
// [-128, 127], a_h in [-64, 64]):
//   a.b = 65536 (a_h.b_h) + 256 (a_h.b_l + a_l.b_h) + a_l.b_l,
// each partial an exact int32 MFMA accumulation.  The queries enter negated
// (the split of -a), so the MFMAs give the partials of -a.b, and the argmin
// key |b|^2 - 2 a.b = |a - b|^2 - |a|^2 is three shift-adds per candidate.
// A squared distance of one view is below 2^31 (at most 4 channels), so the
// key lies in (-2^31, 2^31) and its int32 value, computed modulo 2^32, is
// exact; |a|^2 is added back to the winner.
#include <climits>
#include <type_traits>

#include "sff_device.hpp"

namespace sff {
namespace {

struct InitArgs {
    const int16_t* desc;  // [batch][4][H][W][Cp][16], Cp = kRecC<C>
    int16_t* hyp;         // [ndir][batch][Hk][Wk][4]
    uint32_t* cost;       // [ndir][batch][Hk][Wk]
    int H, W, n, Hk, Wk, fm, dm;
    int batch, dir0, ndir;
};

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kQRows = 4;    // query rows per block (one 16-query MFMA tile each)
constexpr int kWaves = 4;    // waves per block, splitting the candidate rows
constexpr int kKBytes = 64;  // MFMA K: 16 C int8 values, zero padded (C <= 4)

// Split planes of the coarsest-level grid of all four views:
//   hi[z][p][64], lo[z][p][64] int8 (the split of desc), nhi, nlo (the split
//   of -desc) and sq[z][p] = |desc|^2, z = pair * 4 + view, p = i * Wk + j.
// sqx[z][i][wx] holds the same norms with column j at offx + j and the edge
// values repeated over 16+ columns on either side, so the 4 candidates of a
// lane (columns c0 + 4g .. c0 + 4g + 3, never beyond -15 .. Wk + 14) are one
// aligned 16-byte load: offx = 16 + (F mod 4) makes offx + c0 + 4g a multiple
// of 4 for every tile start c0 = j0 - F + 16 t (j0 a multiple of 16).
struct SplitPlanes {
    int8_t* hi;
    int8_t* lo;
    int8_t* nhi;
    int8_t* nlo;
    uint32_t* sq;
    uint32_t* sqx;
    int wx, offx;
};

__host__ __device__ inline int sqx_offset(int F) { return 16 + (F & 3); }
__host__ __device__ inline int sqx_width(int F, int Wk) { return (sqx_offset(F) + Wk + 16 + 3) & ~3; }

template <int C>
__global__ void __launch_bounds__(256) split_kernel(const int16_t* __restrict__ desc, SplitPlanes P,
                                                    int H, int W, int n, int Hk, int Wk, int nz) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    const int z = blockIdx.y;
    if (p >= Hk * Wk || z >= nz) return;
    const int i = p / Wk, j = p - i * Wk;
    const size_t mapsz = (size_t)H * W * 16 * kRecC<C>;
    const int16_t* d = desc + (size_t)z * mapsz + ((size_t)(n * i) * W + n * j) * 16 * kRecC<C>;
    uint32_t hw[2][kKBytes / 4], lw[2][kKBytes / 4];
    uint32_t sq = 0;
#pragma unroll
    for (int w = 0; w < kKBytes / 4; ++w) {
        hw[0][w] = lw[0][w] = hw[1][w] = lw[1][w] = 0;
    }
#pragma unroll
    for (int k = 0; k < 16 * C; ++k) {
        const int a = d[k];
        sq += (uint32_t)(a * a);
#pragma unroll
        for (int neg = 0; neg < 2; ++neg) {
            const int v = neg ? -a : a;
            const int lo = ((v + 128) & 255) - 128;
            const int hi = (v - lo) >> 8;
            hw[neg][k >> 2] |= (uint32_t)(uint8_t)(int8_t)hi << (8 * (k & 3));
            lw[neg][k >> 2] |= (uint32_t)(uint8_t)(int8_t)lo << (8 * (k & 3));
        }
    }
    const size_t o = (size_t)z * Hk * Wk + p;
    int8_t* const dst[4] = {P.hi, P.lo, P.nhi, P.nlo};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const uint32_t* src = (m & 1) ? lw[m >> 1] : hw[m >> 1];
        uint4* out = reinterpret_cast<uint4*>(dst[m] + o * kKBytes);
#pragma unroll
        for (int q = 0; q < kKBytes / 16; ++q)
            out[q] = make_uint4(src[4 * q], src[4 * q + 1], src[4 * q + 2], src[4 * q + 3]);
    }
    P.sq[o] = sq;
    uint32_t* row = P.sqx + ((size_t)z * Hk + i) * P.wx;
    row[P.offx + j] = sq;
    if (j == 0)
        for (int x = 0; x < P.offx; ++x) row[x] = sq;
    if (j == Wk - 1)
        for (int x = P.offx + Wk; x < P.wx; ++x) row[x] = sq;
}

__device__ __forceinline__ v4i load16(const int8_t* p) {
    return __builtin_bit_cast(v4i, *reinterpret_cast<const uint4*>(p));
}

// One block: kQRows rows x 16 consecutive columns of reference grid pixels of
// one field.  Wave w scans the candidate rows r = rlo + w (mod kWaves) of the
// union of the queries' boxes, 16 candidates per MFMA tile.
//
// v_mfma_i32_16x16x64_i8 operands: A (16 x 64) holds candidates, lane l giving
// candidate l % 16; B (64 x 16) holds queries, lane l giving query l % 16; both
// with the same K bytes for lane group l / 16, so each product sums over all 64
// K values.  Lane l receives C[4 (l / 16) + e][l % 16], e = 0..3: candidates
// 4 g + e of the tile against its own query.
//
// K > 1 (initialisation with K temporal leaves): each lane keeps its K best
// (key, target index) per query, sorted (a candidate enters after kept ones of
// equal key, which have smaller indices); the lists are merged per query in
// LDS, each leaf gets its own cross-row search, and the combination with the
// smallest T + S + X distance wins (the earlier leaf on ties).
template <int C, int K>
__global__ void __launch_bounds__(256) init_nn_kernel(InitArgs a, SplitPlanes P) {
    __shared__ unsigned long long red[kWaves * 4][kQRows][16][K];
    __shared__ int res_u[kQRows][16][K], res_v[kQRows][16][K];
    __shared__ uint32_t res_t[kQRows][16][K];
    __shared__ int res_n[kQRows][16];
    __shared__ unsigned long long red2[4][kQRows][16];
    __shared__ unsigned long long redx[K][4][kQRows][16];
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

    const int W = a.W;
    const size_t mapsz = (size_t)a.H * W * 16 * kRecC<C>;
    const int16_t* base = a.desc + (size_t)b * 4 * mapsz;

    // queries (B operands, negated), one 16-column tile per query row
    v4i qh[kQRows], ql[kQRows];
    int best[kQRows], btile[kQRows];   // K = 1: minimum key and its first tile
    int tk[kQRows][K], ti[kQRows][K];  // K > 1: sorted keys and target indices
    const int jq = min(j0 + nq, Wk - 1);
#pragma unroll
    for (int t = 0; t < kQRows; ++t) {
        const size_t o = zR + (size_t)min(i0 + t, Hk - 1) * Wk + jq;
        qh[t] = load16(P.nhi + o * kKBytes + 16 * g);
        ql[t] = load16(P.nlo + o * kKBytes + 16 * g);
        best[t] = INT_MAX;
        btile[t] = 0;
#pragma unroll
        for (int l = 0; l < K; ++l) {
            tk[t][l] = INT_MAX;
            ti[t][l] = 0;
        }
    }
    // Scan: per query only the minimum key over this lane's candidates and the
    // first tile (in increasing target index) that reaches it are kept; the
    // target inside that tile is recovered afterwards.
    const int rlo = max(0, i0 - F), rhi = min(Hk - 1, i0 + kQRows - 1 + F);
    const int nct = (16 + 2 * F + 15) / 16;
    // candidate tiles of this wave: rows rlo + w, rlo + w + kWaves, ... and the
    // column tiles that overlap the image, visited in increasing target index
    const int ct_lo = max(0, (F - j0) >> 4);                     // first c0 + 15 >= 0
    const int ct_hi = min(nct - 1, (Wk - 1 - j0 + F) >> 4);      // last c0 < Wk
    const int ntl = ct_hi - ct_lo + 1;
    const int nrw = rlo + w <= rhi ? (rhi - rlo - w) / kWaves + 1 : 0;
    const int total = ntl > 0 ? nrw * ntl : 0;
    const v4i zero = {0, 0, 0, 0};

    struct Tile {
        v4i ah, al;
        int bsq[4];
    };
    // Loads of tile (r, ct); the scan issues those of the next tile before it
    // scores the current one.
    auto load_tile = [&](int r, int ct) {
        Tile T;
        const size_t rowT = zT + (size_t)r * Wk;
        const int c0 = j0 - F + 16 * ct;
        const size_t oa = rowT + clampi(c0 + nq, 0, Wk - 1);
        T.ah = load16(P.hi + oa * kKBytes + 16 * g);
        T.al = load16(P.lo + oa * kKBytes + 16 * g);
        const uint4 q = *reinterpret_cast<const uint4*>(P.sqx + (zTx + (size_t)r) * P.wx + P.offx + c0 + 4 * g);
        T.bsq[0] = (int)q.x;
        T.bsq[1] = (int)q.y;
        T.bsq[2] = (int)q.z;
        T.bsq[3] = (int)q.w;
        return T;
    };
    // The scan alternates between two tile buffers (scan_one(a, b) scores a
    // and loads the next tile into b), so no tile is copied between steps.
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
            if constexpr (!kInterior) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int jc = c0 + 4 * g + e;
                    ok[e] = (unsigned)(jc - jq + F) <= (unsigned)(2 * F) && (unsigned)jc < (unsigned)Wk;
                }
            }
#pragma unroll
            for (int t = 0; t < kQRows; ++t) {
                if constexpr (!kRowsIn) {
                    const int iq = i0 + t;
                    if (iq >= Hk || r < iq - F || r > iq + F) continue;
                }
                const v4i hh = __builtin_amdgcn_mfma_i32_16x16x64_i8(cur.ah, qh[t], zero, 0, 0, 0);
                v4i cr = __builtin_amdgcn_mfma_i32_16x16x64_i8(cur.ah, ql[t], zero, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_i32_16x16x64_i8(cur.al, qh[t], cr, 0, 0, 0);
                const v4i ll = __builtin_amdgcn_mfma_i32_16x16x64_i8(cur.al, ql[t], zero, 0, 0, 0);
                int k[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    // |b|^2 + 2 (-a.b), -a.b = 256 (256 hh + cr) + ll  (mod 2^32),
                    // nested so that each step is one shift-add
                    const uint32_t hc = ((uint32_t)hh[e] << 8) + (uint32_t)cr[e];
                    const uint32_t ab = (hc << 8) + (uint32_t)ll[e];
                    const uint32_t key = (ab << 1) + (uint32_t)cur.bsq[e];
                    k[e] = (int)key;
                    if constexpr (!kInterior) k[e] = ok[e] ? k[e] : INT_MAX;
                }
                if constexpr (K == 1) {
                    const int m = min(min(k[0], k[1]), min(k[2], k[3]));
                    const bool better = m < best[t];
                    btile[t] = better ? tile_id : btile[t];
                    best[t] = better ? m : best[t];
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (!__any(k[e] < tk[t][K - 1])) continue;  // wave-uniform
                        int nk = k[e], ni = r * Wk + c0 + 4 * g + e;
#pragma unroll
                        for (int l = 0; l < K; ++l) {
                            const bool lt = nk < tk[t][l];
                            const int ok_ = tk[t][l], oi = ti[t][l];
                            tk[t][l] = lt ? nk : ok_;
                            ti[t][l] = lt ? ni : oi;
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
    // the smallest target index of the winning tile that reaches the minimum
    // (exact squared distances from the int16 descriptors, equal to the MFMA
    // identity's)
    const int16_t* Tm = base + (size_t)vT * mapsz;
    const int16_t* Rm = base + (size_t)vR * mapsz;
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
            const Desc<C> qd = load_desc<C>(Rm, (size_t)(n * min(i0 + t, Hk - 1)) * W + n * jq);
            const uint32_t asq = P.sq[zR + (size_t)min(i0 + t, Hk - 1) * Wk + jq];
            bssd = (uint32_t)best[t] + asq;
            bool found = false;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int jc = c0 + 4 * g + e;
                const bool ok = (unsigned)(jc - jq + F) <= (unsigned)(2 * F) && (unsigned)jc < (unsigned)Wk;
                if (ok && !found) {
                    const uint32_t d = desc_ssd<C>(qd, load_desc<C>(Tm, (size_t)(n * r) * W + n * jc));
                    if (d == bssd) {
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

    // epipolar searches: 4 threads per query, candidates interleaved
    const int q = threadIdx.x & 15, t = (threadIdx.x >> 4) & 3, part = threadIdx.x >> 6;
    const int iq = i0 + t, jqq = j0 + q;
    const bool live = iq < Hk && jqq < Wk;
    const int x = n * min(jqq, Wk - 1), y = n * min(iq, Hk - 1);
    const Desc<C> qd = load_desc<C>(Rm, (size_t)y * W + x);
    const int16_t* Sm = base + (size_t)vS * mapsz;
    const int16_t* Xm = base + (size_t)vX * mapsz;
    // stereo partner on row y: target tx = x - s d0, increasing tx
    unsigned long long kS = ~0ull;
    if (live) {
        const int txlo = s > 0 ? x - min(a.dm, x) : x;
        const int txhi = s > 0 ? x : x + min(a.dm, ((W - 1 - x) / n) * n);
        for (int tx = txlo + n * part; tx <= txhi; tx += 4 * n) {
            const uint32_t e = desc_ssd<C>(qd, load_desc<C>(Sm, (size_t)y * W + tx));
            const unsigned long long k = ((unsigned long long)e << 32) | (uint32_t)tx;
            kS = k < kS ? k : kS;
        }
    }
    red2[part][t][q] = kS;
    __syncthreads();
    unsigned long long mS = red2[0][t][q];
#pragma unroll
    for (int k = 1; k < 4; ++k) mS = red2[k][t][q] < mS ? red2[k][t][q] : mS;
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
            for (int tx = txlo + n * part; tx <= txhi; tx += 4 * n) {
                const uint32_t e = desc_ssd<C>(qd, load_desc<C>(Xm, (size_t)yc * W + tx));
                const unsigned long long k = ((unsigned long long)e << 32) | (uint32_t)tx;
                kX = k < kX ? k : kX;
            }
        }
        redx[l][part][t][q] = kX;
    }
    __syncthreads();
    if (part != 0 || !live) return;
    // the cheapest combination (every target lies inside the image, so its
    // eq. (1) cost is the sum of the three distances); the earlier leaf on ties
    const uint32_t eS = (uint32_t)(mS >> 32);
    uint64_t bestJ = ~0ull;
    int bu = 0, bv = 0, bd1 = 0;
    for (int l = 0; l < nl; ++l) {
        unsigned long long mX = redx[l][0][t][q];
#pragma unroll
        for (int k = 1; k < 4; ++k) mX = redx[l][k][t][q] < mX ? redx[l][k][t][q] : mX;
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
    a.cost[o] = (uint32_t)bestJ;
}

template <int C>
void launch_init(int leaves, dim3 grid, hipStream_t st, const InitArgs& a, const SplitPlanes& P) {
    switch (leaves) {
        case 1: hipLaunchKernelGGL((init_nn_kernel<C, 1>), grid, dim3(256), 0, st, a, P); break;
        case 2: hipLaunchKernelGGL((init_nn_kernel<C, 2>), grid, dim3(256), 0, st, a, P); break;
        default: hipLaunchKernelGGL((init_nn_kernel<C, 4>), grid, dim3(256), 0, st, a, P); break;
    }
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct InitWs {
    size_t hi, lo, nhi, nlo, sq, sqx, total;
    int wx, offx;
};

InitWs init_ws(const sff_params& p, int batch) {
    const LevelGeom g = level_geom(p, p.levels - 1);
    const size_t cnt = (size_t)batch * 4 * g.Hk * g.Wk;
    InitWs L;
    L.hi = 0;
    L.lo = align256(cnt * kKBytes);
    L.nhi = L.lo + align256(cnt * kKBytes);
    L.nlo = L.nhi + align256(cnt * kKBytes);
    L.sq = L.nlo + align256(cnt * kKBytes);
    L.sqx = L.sq + align256(cnt * sizeof(uint32_t));
    const int F = p.fmax / g.n;
    L.offx = sqx_offset(F);
    L.wx = sqx_width(F, g.Wk);
    L.total = L.sqx + align256((size_t)batch * 4 * g.Hk * L.wx * sizeof(uint32_t));
    return L;
}

}  // namespace
}  // namespace sff

using namespace sff;

extern "C" size_t sff_init_workspace_bytes(const sff_params* p, int32_t batch) {
    if (!params_ok(p) || batch < 1 || batch > 32767) return 0;
    return init_ws(*p, batch).total;
}

extern "C" sff_status sff_init_nn_leaves(const sff_params* p, int32_t batch, int32_t dir,
                                         int32_t leaves, const int16_t* desc, int16_t* hyp,
                                         uint32_t* cost, void* workspace, size_t workspace_bytes,
                                         void* stream) {
    if (!params_ok(p) || batch < 1 || batch > 32767 || (dir != 1 && dir != -1 && dir != 0) ||
        !desc || !hyp || !cost || leaves < 1)
        return SFF_ERR_INVALID_ARG;
    if (leaves != 1 && leaves != 2 && leaves != 4) return SFF_ERR_UNSUPPORTED;
    if ((reinterpret_cast<uintptr_t>(desc) & 15) != 0 || (reinterpret_cast<uintptr_t>(hyp) & 7) != 0 ||
        (reinterpret_cast<uintptr_t>(cost) & 3) != 0)
        return SFF_ERR_INVALID_ARG;
    const InitWs L = init_ws(*p, batch);
    if (!workspace || workspace_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return SFF_ERR_WORKSPACE;
    const int level = p->levels - 1;
    const LevelGeom g = level_geom(*p, level);
    InitArgs a;
    a.desc = desc;
    a.hyp = hyp;
    a.cost = cost;
    a.H = p->H;
    a.W = p->W;
    a.n = g.n;
    a.Hk = g.Hk;
    a.Wk = g.Wk;
    a.fm = (p->fmax / g.n) * g.n;
    a.dm = (p->dmax / g.n) * g.n;
    a.batch = batch;
    a.ndir = dir == 0 ? 2 : 1;
    a.dir0 = dir == 0 ? 1 : dir;
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    SplitPlanes P;
    P.hi = reinterpret_cast<int8_t*>(ws + L.hi);
    P.lo = reinterpret_cast<int8_t*>(ws + L.lo);
    P.nhi = reinterpret_cast<int8_t*>(ws + L.nhi);
    P.nlo = reinterpret_cast<int8_t*>(ws + L.nlo);
    P.sq = reinterpret_cast<uint32_t*>(ws + L.sq);
    P.sqx = reinterpret_cast<uint32_t*>(ws + L.sqx);
    P.wx = L.wx;
    P.offx = L.offx;
    const int nz4 = 4 * batch;
    const dim3 sgrid((g.Hk * g.Wk + 255) / 256, nz4);
    const dim3 grid((g.Wk + 15) / 16, (g.Hk + kQRows - 1) / kQRows, a.ndir * batch);
    hipStream_t st = as_stream(stream);
    switch (p->C) {
        case 1:
            hipLaunchKernelGGL(split_kernel<1>, sgrid, dim3(256), 0, st, desc, P, a.H, a.W, a.n, a.Hk, a.Wk, nz4);
            launch_init<1>(leaves, grid, st, a, P);
            break;
        case 2:
            hipLaunchKernelGGL(split_kernel<2>, sgrid, dim3(256), 0, st, desc, P, a.H, a.W, a.n, a.Hk, a.Wk, nz4);
            launch_init<2>(leaves, grid, st, a, P);
            break;
        case 3:
            hipLaunchKernelGGL(split_kernel<3>, sgrid, dim3(256), 0, st, desc, P, a.H, a.W, a.n, a.Hk, a.Wk, nz4);
            launch_init<3>(leaves, grid, st, a, P);
            break;
        default:
            hipLaunchKernelGGL(split_kernel<4>, sgrid, dim3(256), 0, st, desc, P, a.H, a.W, a.n, a.Hk, a.Wk, nz4);
            launch_init<4>(leaves, grid, st, a, P);
            break;
    }
    return launch_status();
}

extern "C" sff_status sff_init_nn(const sff_params* p, int32_t batch, int32_t dir,
                                  const int16_t* desc, int16_t* hyp, uint32_t* cost,
                                  void* workspace, size_t workspace_bytes, void* stream) {
    return sff_init_nn_leaves(p, batch, dir, 1, desc, hyp, cost, workspace, workspace_bytes, stream);
}
