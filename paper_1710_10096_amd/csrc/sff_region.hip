// Region filter (SceneFlowFields, Section 3.1, "Consistency Check", second
// step; s_c in Section 5) and sparsification (Section 3.2).
//
// Regions are the connected components of the graph whose nodes are the
// consistent pixels and whose edges join 4-neighbours with every vector
// component within tau.  They are found with a lock-free union-find in which
// every union hooks the larger root under the smaller one with a
// compare-and-swap, so a component's final root is its smallest pixel index
// whatever the order of the unions.  The edges inside a 16 x 64 tile are
// united first in LDS, one block per tile; only the edges that cross tile
// borders are united in global memory.  Then each component's size is counted
// and it is flagged when an inconsistent 4-neighbour of one of its pixels is
// within tau of that pixel's vector.  A flagged component with fewer than s_c
// pixels is dropped.  The result is independent of thread order.
#include "sff_internal.hpp"

namespace sff {
namespace {

struct RegionArgs {
    const int16_t* hyp;   // [batch][H][W][4]
    const uint8_t* valid; // [batch][H][W]
    uint8_t* keep;        // [batch][H][W]
    int32_t* parent;      // [batch][H][W]  (workspace)
    int32_t* size;        // [batch][H][W]  (workspace)
    int32_t* flag;        // [batch][H][W]  (workspace)
    int H, W, tau, s_c;
};

// Parent pointers change under other threads: read and write them at device
// scope so no stale copy in a CU's cache is used.
__device__ __forceinline__ int ld(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st(int32_t* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x, halving the path on the way (every write replaces a parent by one
// of its ancestors, which is always safe).  Pointers only ever point to smaller
// indices, so the walk ends.
__device__ int find_root(int32_t* parent, int x) {
    int p = ld(parent + x);
    while (p != x) {
        const int g = ld(parent + p);
        if (g != p) st(parent + x, g);
        x = p;
        p = g;
    }
    return x;
}

// Read-only walk, for use once the unions are complete (the forest is static
// then apart from pixels being pointed straight at their roots).
__device__ int find_root_ro(const int32_t* parent, int x) {
    int p = ld(parent + x);
    while (p != x) {
        x = p;
        p = ld(parent + x);
    }
    return x;
}

__device__ void unite(int32_t* parent, int a, int b, int n) {
    // Each failed compare-and-swap means root a was hooked elsewhere, so the
    // larger root of the pair strictly decreases: at most n rounds.
    for (int round = 0; round <= n; ++round) {
        a = find_root(parent, a);
        b = find_root(parent, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(parent + a, a, b) == a) return;
    }
}

__device__ __forceinline__ bool similar(const int16_t* h, int p, int q, int tau) {
    const uint2 a = reinterpret_cast<const uint2*>(h)[p];
    const uint2 b = reinterpret_cast<const uint2*>(h)[q];
    const int d0 = (int)(int16_t)(a.x & 0xFFFFu) - (int)(int16_t)(b.x & 0xFFFFu);
    const int d1 = (int)(int16_t)(a.x >> 16) - (int)(int16_t)(b.x >> 16);
    const int d2 = (int)(int16_t)(a.y & 0xFFFFu) - (int)(int16_t)(b.y & 0xFFFFu);
    const int d3 = (int)(int16_t)(a.y >> 16) - (int)(int16_t)(b.y >> 16);
    return abs(d0) <= tau && abs(d1) <= tau && abs(d2) <= tau && abs(d3) <= tau;
}

// blockIdx.y = batch element; one thread per pixel.
__global__ void __launch_bounds__(256) rf_init_kernel(RegionArgs a) {
    const int n = a.H * a.W;
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const size_t o = (size_t)blockIdx.y * n + p;
    a.size[o] = 0;
    a.flag[o] = 0;
}

constexpr int kTH = 16, kTW = 64;  // tile of the local pass

__device__ __forceinline__ int lfind(const int* lp, int x) {
    int p = __hip_atomic_load(lp + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    while (p != x) {
        x = p;
        p = __hip_atomic_load(lp + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    return x;
}

__device__ void lunite(int* lp, int a, int b) {
    for (int round = 0; round <= kTH * kTW; ++round) {
        a = lfind(lp, a);
        b = lfind(lp, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(lp + a, a, b) == a) return;
    }
}

// One block per 16 x 64 tile (blockIdx.x = tile, blockIdx.y = batch element):
// unions of the edges inside the tile in LDS; every pixel's global parent
// becomes the global index of its tile-local root (tile rows and image rows
// are both row-major, so the smallest local index is the smallest global one).
__global__ void __launch_bounds__(256) rf_local_kernel(RegionArgs a) {
    __shared__ int lp[kTH * kTW];
    __shared__ uint8_t lv[kTH * kTW];
    const int tiles_x = (a.W + kTW - 1) / kTW;
    const int ty0 = (blockIdx.x / tiles_x) * kTH, tx0 = (blockIdx.x % tiles_x) * kTW;
    const size_t base = (size_t)blockIdx.y * a.H * a.W;
    const int16_t* h = a.hyp + base * 4;
    for (int i = threadIdx.x; i < kTH * kTW; i += 256) {
        const int y = ty0 + i / kTW, x = tx0 + i % kTW;
        lp[i] = i;
        lv[i] = (y < a.H && x < a.W) ? a.valid[base + (size_t)y * a.W + x] : 0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kTH * kTW; i += 256) {
        if (!lv[i]) continue;
        const int r = i / kTW, c = i % kTW;
        const int p = (ty0 + r) * a.W + tx0 + c;
        if (c + 1 < kTW && lv[i + 1] && similar(h, p, p + 1, a.tau)) lunite(lp, i, i + 1);
        if (r + 1 < kTH && lv[i + kTW] && similar(h, p, p + a.W, a.tau)) lunite(lp, i, i + kTW);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kTH * kTW; i += 256) {
        const int y = ty0 + i / kTW, x = tx0 + i % kTW;
        if (y >= a.H || x >= a.W) continue;
        const int r = lfind(lp, i);
        a.parent[base + (size_t)y * a.W + x] = (ty0 + r / kTW) * a.W + tx0 + r % kTW;
    }
}

// Unions of the edges that cross tile borders (right neighbour in the next
// tile column, lower neighbour in the next tile row), on the global forest.
__global__ void __launch_bounds__(256) rf_union_kernel(RegionArgs a) {
    const int n = a.H * a.W;
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const int x = p % a.W, y = p / a.W;
    const bool right = (x % kTW) == kTW - 1 && x + 1 < a.W;
    const bool down = (y % kTH) == kTH - 1 && y + 1 < a.H;
    if (!right && !down) return;
    const size_t base = (size_t)blockIdx.y * n;
    const uint8_t* v = a.valid + base;
    if (!v[p]) return;
    const int16_t* h = a.hyp + base * 4;
    int32_t* parent = a.parent + base;
    if (right && v[p + 1] && similar(h, p, p + 1, a.tau)) unite(parent, p, p + 1, n);
    if (down && v[p + a.W] && similar(h, p, p + a.W, a.tau)) unite(parent, p, p + a.W, n);
}

// Adds `val` of every active lane into arr[key], one atomic per distinct key
// of the wave (neighbouring pixels mostly share their root).  Call with the
// whole wave; the loop runs once per distinct key.
__device__ void wave_add_by_key(int32_t* arr, int key, bool active, int val) {
    unsigned long long pending = __ballot(active);
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int k0 = __shfl(key, leader);
        const bool mine = active && key == k0;
        const unsigned long long same = __ballot(mine);
        int sum = mine ? val : 0;
        // wave sum of the lanes holding k0
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) sum += __shfl_xor(sum, off);
        if ((threadIdx.x & 63) == leader) atomicAdd(arr + k0, sum);
        if (mine) active = false;
        pending &= ~same;
    }
}

// After all unions: every consistent pixel's parent becomes its root, and the
// root's pixel count is accumulated.
__global__ void __launch_bounds__(256) rf_count_kernel(RegionArgs a) {
    const int n = a.H * a.W;
    const int p = blockIdx.x * 256 + threadIdx.x;
    const size_t base = (size_t)blockIdx.y * n;
    const bool act = p < n && a.valid[base + p];
    int r = 0;
    if (act) {
        int32_t* parent = a.parent + base;
        r = find_root_ro(parent, p);
        st(parent + p, r);
    }
    wave_add_by_key(a.size + base, r, act, 1);
}

// Inconsistent pixels flag every neighbouring region they could join.  Runs
// after rf_count_kernel, so a consistent pixel's parent is its root.  Flags
// only go from 0 to 1: a flag already seen set needs no atomic.
__global__ void __launch_bounds__(256) rf_flag_kernel(RegionArgs a) {
    const int n = a.H * a.W;
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const size_t base = (size_t)blockIdx.y * n;
    const uint8_t* v = a.valid + base;
    if (v[p]) return;
    const int16_t* h = a.hyp + base * 4;
    const int32_t* parent = a.parent + base;
    int32_t* flag = a.flag + base;
    const int x = p % a.W, y = p / a.W;
    const int nb[4] = {x > 0 ? p - 1 : -1, x + 1 < a.W ? p + 1 : -1, y > 0 ? p - a.W : -1,
                       y + 1 < a.H ? p + a.W : -1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int q = nb[k];
        if (q >= 0 && v[q] && similar(h, p, q, a.tau)) {
            const int r = parent[q];
            if (flag[r] == 0) atomicOr(flag + r, 1);  // a stale 0 costs one extra atomic
        }
    }
}

__global__ void __launch_bounds__(256) rf_keep_kernel(RegionArgs a) {
    const int n = a.H * a.W;
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const size_t base = (size_t)blockIdx.y * n;
    uint8_t k = 0;
    if (a.valid[base + p]) {
        const int r = a.parent[base + p];
        k = (a.flag[base + r] != 0 && a.size[base + r] < a.s_c) ? 0 : 1;
    }
    a.keep[base + p] = k;
}

// One thread per 3 x 3 block: the kept pixel with the lowest error, ties to
// the lowest raster index; -1 for an empty block.
__global__ void __launch_bounds__(256) sparsify_kernel(const uint8_t* __restrict__ keep,
                                                       const uint32_t* __restrict__ err,
                                                       int32_t* __restrict__ seeds, int H, int W) {
    const int Hb = (H + 2) / 3, Wb = (W + 2) / 3;
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= Hb * Wb) return;
    const size_t base = (size_t)blockIdx.y * H * W;
    const int bi = b / Wb, bj = b - bi * Wb;
    int best = -1;
    uint32_t be = 0;
    for (int y = 3 * bi; y < min(3 * bi + 3, H); ++y)
        for (int x = 3 * bj; x < min(3 * bj + 3, W); ++x) {
            const int p = y * W + x;
            if (!keep[base + p]) continue;
            const uint32_t e = err[base + p];
            if (best < 0 || e < be) {
                best = p;
                be = e;
            }
        }
    seeds[(size_t)blockIdx.y * Hb * Wb + b] = best;
}

size_t region_ws_bytes(const sff_params& p, int batch) {
    const size_t words = (size_t)batch * p.H * p.W;
    const size_t one = (words * sizeof(int32_t) + 255) & ~(size_t)255;
    return 3 * one;
}

}  // namespace
}  // namespace sff

using namespace sff;

extern "C" size_t sff_region_workspace_bytes(const sff_params* p, int32_t batch) {
    if (!params_ok(p) || batch < 1 || batch > 32767) return 0;
    return region_ws_bytes(*p, batch);
}

extern "C" sff_status sff_region_filter(const sff_params* p, int32_t batch, int32_t s_c,
                                        const int16_t* hyp_fwd, const uint8_t* valid,
                                        uint8_t* keep, void* workspace, size_t workspace_bytes,
                                        void* stream) {
    if (!params_ok(p) || batch < 1 || batch > 32767 || s_c < 1 || !hyp_fwd || !valid || !keep ||
        (reinterpret_cast<uintptr_t>(hyp_fwd) & 7) != 0)
        return SFF_ERR_INVALID_ARG;
    const size_t need = region_ws_bytes(*p, batch);
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return SFF_ERR_WORKSPACE;
    RegionArgs a;
    a.hyp = hyp_fwd;
    a.valid = valid;
    a.keep = keep;
    const size_t one = need / 3;
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    a.parent = reinterpret_cast<int32_t*>(ws);
    a.size = reinterpret_cast<int32_t*>(ws + one);
    a.flag = reinterpret_cast<int32_t*>(ws + 2 * one);
    a.H = p->H;
    a.W = p->W;
    a.tau = p->tau;
    a.s_c = s_c;
    const dim3 grid((p->H * p->W + 255) / 256, batch);
    hipStream_t st = as_stream(stream);
    const int tiles = ((p->H + kTH - 1) / kTH) * ((p->W + kTW - 1) / kTW);
    hipLaunchKernelGGL(rf_init_kernel, grid, dim3(256), 0, st, a);
    hipLaunchKernelGGL(rf_local_kernel, dim3(tiles, batch), dim3(256), 0, st, a);
    hipLaunchKernelGGL(rf_union_kernel, grid, dim3(256), 0, st, a);
    hipLaunchKernelGGL(rf_count_kernel, grid, dim3(256), 0, st, a);
    hipLaunchKernelGGL(rf_flag_kernel, grid, dim3(256), 0, st, a);
    hipLaunchKernelGGL(rf_keep_kernel, grid, dim3(256), 0, st, a);
    return launch_status();
}

extern "C" sff_status sff_sparsify(const sff_params* p, int32_t batch, const uint8_t* keep,
                                   const uint32_t* err, int32_t* seeds, void* stream) {
    if (!params_ok(p) || batch < 1 || batch > 32767 || !keep || !err || !seeds ||
        (reinterpret_cast<uintptr_t>(err) & 3) != 0 || (reinterpret_cast<uintptr_t>(seeds) & 3) != 0)
        return SFF_ERR_INVALID_ARG;
    const int Hb = (p->H + 2) / 3, Wb = (p->W + 2) / 3;
    hipLaunchKernelGGL(sparsify_kernel, dim3((Hb * Wb + 255) / 256, batch), dim3(256), 0,
                       as_stream(stream), keep, err, seeds, p->H, p->W);
    return launch_status();
}
