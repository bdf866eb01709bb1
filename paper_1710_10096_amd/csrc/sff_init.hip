// Initialisation at the coarsest level (SceneFlowFields, Section 3.1,
// "Initialization"): exact nearest neighbours of each reference grid pixel's
// WHT descriptor among grid pixels of the temporal partner (box |u|,|v| <=
// fmax), the stereo partner (same row, 0 <= d0 <= dmax) and the cross partner
// (row y + v*, 0 <= d1 <= dmax), ties to the smallest target index; the
// combination's eq. (1) cost is stored with it.
//
// One thread per reference grid pixel.  A wave covers a 16 x 4 tile of grid
// pixels, so at every step of the box scan its lanes read 4 runs of 16
// consecutive candidate descriptors.
#include "sff_device.hpp"

namespace sff {
namespace {

struct InitArgs {
    const int16_t* desc;  // [batch][4][H][W][C][16]
    int16_t* hyp;         // [ndir][batch][Hk][Wk][4]
    uint32_t* cost;       // [ndir][batch][Hk][Wk]
    int H, W, n, Hk, Wk, fm, dm;
    int batch, dir0, ndir;
};

template <int C>
__global__ void __launch_bounds__(256) init_nn_kernel(InitArgs a) {
    const int j = blockIdx.x * 16 + (threadIdx.x & 15);
    const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
    const int z = blockIdx.z;  // dir_index * batch + b
    const int di = z / a.batch, b = z - di * a.batch;
    if (i >= a.Hk || j >= a.Wk) return;
    const int s = (a.ndir == 2) ? (di == 0 ? 1 : -1) : a.dir0;
    const size_t plane = (size_t)a.H * a.W;
    const size_t mapsz = plane * 16 * C;
    const int16_t* base = a.desc + (size_t)b * 4 * mapsz;
    // canonical order l0, l1, r0, r1; the inverse field permutes to r1, r0, l1, l0
    const int16_t* R = base + (size_t)(s > 0 ? 0 : 3) * mapsz;
    const int16_t* T = base + (size_t)(s > 0 ? 1 : 2) * mapsz;
    const int16_t* S = base + (size_t)(s > 0 ? 2 : 1) * mapsz;
    const int16_t* X = base + (size_t)(s > 0 ? 3 : 0) * mapsz;
    const int n = a.n, W = a.W, H = a.H;
    const int x = n * j, y = n * i;
    const Desc<C> q = load_desc<C>(R, (size_t)y * W + x);

    // temporal partner: box scan in increasing target index, strict improvement
    const int vlo = -min(a.fm, y), vhi = min(a.fm, ((H - 1 - y) / n) * n);
    const int ulo = -min(a.fm, x), uhi = min(a.fm, ((W - 1 - x) / n) * n);
    uint32_t bestT = 0xFFFFFFFFu;
    int bu = 0, bv = 0;
    for (int v = vlo; v <= vhi; v += n) {
        const size_t row = (size_t)(y + v) * W;
        for (int u = ulo; u <= uhi; u += n) {
            const uint32_t e = desc_ssd<C>(q, load_desc<C>(T, row + x + u));
            if (e < bestT) {
                bestT = e;
                bu = u;
                bv = v;
            }
        }
    }
    // stereo partner on row y: target tx = x - s d0, scanned by increasing tx
    uint32_t bestS = 0xFFFFFFFFu;
    int bd0 = 0;
    {
        const int dlim_l = min(a.dm, x);                         // towards smaller x
        const int dlim_r = min(a.dm, ((W - 1 - x) / n) * n);     // towards larger x
        const int txlo = s > 0 ? x - dlim_l : x;
        const int txhi = s > 0 ? x : x + dlim_r;
        for (int tx = txlo; tx <= txhi; tx += n) {
            const uint32_t e = desc_ssd<C>(q, load_desc<C>(S, (size_t)y * W + tx));
            if (e < bestS) {
                bestS = e;
                bd0 = s * (x - tx);
            }
        }
    }
    // cross partner on row y + v*: target tx = x + u* - s d1
    uint32_t bestX = 0xFFFFFFFFu;
    int bd1 = 0;
    {
        const int xc = x + bu, yc = y + bv;
        const int dlim_l = min(a.dm, xc);
        const int dlim_r = min(a.dm, ((W - 1 - xc) / n) * n);
        const int txlo = s > 0 ? xc - dlim_l : xc;
        const int txhi = s > 0 ? xc : xc + dlim_r;
        for (int tx = txlo; tx <= txhi; tx += n) {
            const uint32_t e = desc_ssd<C>(q, load_desc<C>(X, (size_t)yc * W + tx));
            if (e < bestX) {
                bestX = e;
                bd1 = s * (xc - tx);
            }
        }
    }
    const size_t o = ((size_t)z * a.Hk + i) * a.Wk + j;
    uint2 hv;
    hv.x = (uint32_t)(uint16_t)(int16_t)bu | ((uint32_t)(uint16_t)(int16_t)bv << 16);
    hv.y = (uint32_t)(uint16_t)(int16_t)bd0 | ((uint32_t)(uint16_t)(int16_t)bd1 << 16);
    reinterpret_cast<uint2*>(a.hyp)[o] = hv;
    a.cost[o] = bestT + bestS + bestX;  // all three targets lie inside the image
}

}  // namespace
}  // namespace sff

using namespace sff;

extern "C" sff_status sff_init_nn(const sff_params* p, int32_t batch, int32_t dir,
                                  const int16_t* desc, int16_t* hyp, uint32_t* cost,
                                  void* stream) {
    if (!params_ok(p) || batch < 1 || batch > 32767 || (dir != 1 && dir != -1 && dir != 0) ||
        !desc || !hyp || !cost)
        return SFF_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(desc) & 15) != 0 || (reinterpret_cast<uintptr_t>(hyp) & 7) != 0 ||
        (reinterpret_cast<uintptr_t>(cost) & 3) != 0)
        return SFF_ERR_INVALID_ARG;
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
    const dim3 grid((g.Wk + 15) / 16, (g.Hk + 15) / 16, a.ndir * batch);
    hipStream_t st = as_stream(stream);
    switch (p->C) {
        case 1: hipLaunchKernelGGL(init_nn_kernel<1>, grid, dim3(256), 0, st, a); break;
        case 2: hipLaunchKernelGGL(init_nn_kernel<2>, grid, dim3(256), 0, st, a); break;
        case 3: hipLaunchKernelGGL(init_nn_kernel<3>, grid, dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL(init_nn_kernel<4>, grid, dim3(256), 0, st, a); break;
    }
    return launch_status();
}
