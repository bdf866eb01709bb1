// Consistency check (SceneFlowFields, Section 3.1, "Consistency Check"; the
// threshold tau_c of Section 5).  The inverse field has reference I_r^1.  At a
// forward pixel p with vector (u, v, d0, d1) the inverse vector (u', v', d0',
// d1') at the cross target q = p + (u - d1, v) implies a disparity d1' at t0,
// d0' at t1 and a left-view flow (d0' - u' - d1', -v'); the match survives when
// all three agree with the forward vector within tau (flow as a Euclidean
// 2-vector) and all forward targets lie inside the image.
#include "sff_internal.hpp"

namespace sff {
namespace {

__global__ void __launch_bounds__(256) consistency_kernel(const int16_t* __restrict__ fwd,
                                                          const int16_t* __restrict__ inv,
                                                          uint8_t* __restrict__ valid,
                                                          uint32_t* __restrict__ err, int H, int W,
                                                          int tau) {
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int b = blockIdx.z;
    if (x >= W || y >= H) return;
    const size_t plane = (size_t)H * W;
    const size_t o = (size_t)b * plane + (size_t)y * W + x;
    const uint2 hf = reinterpret_cast<const uint2*>(fwd)[o];
    const int u = (int16_t)(hf.x & 0xFFFFu), v = (int16_t)(hf.x >> 16);
    const int d0 = (int16_t)(hf.y & 0xFFFFu), d1 = (int16_t)(hf.y >> 16);
    const int tyT = y + v, txT = x + u, txS = x - d0, txX = x + u - d1;
    const bool inb = (unsigned)txT < (unsigned)W && (unsigned)tyT < (unsigned)H &&
                     (unsigned)txS < (unsigned)W && (unsigned)txX < (unsigned)W;
    if (!inb) {
        valid[o] = 0;
        err[o] = 0xFFFFFFFFu;
        return;
    }
    const uint2 hi = reinterpret_cast<const uint2*>(inv)[(size_t)b * plane + (size_t)tyT * W + txX];
    const int ui = (int16_t)(hi.x & 0xFFFFu), vi = (int16_t)(hi.x >> 16);
    const int d0i = (int16_t)(hi.y & 0xFFFFu), d1i = (int16_t)(hi.y >> 16);
    // hypotheses are bounded by 8192 in magnitude, so every square fits 32 bits
    const int e0 = d0 - d1i, e1 = d1 - d0i;
    const int efx = u + ui + d1i - d0i, efy = v + vi;
    const uint32_t a0 = (uint32_t)(e0 * e0), a1 = (uint32_t)(e1 * e1);
    const uint32_t af = (uint32_t)(efx * efx) + (uint32_t)(efy * efy);
    const uint32_t t2 = (uint32_t)tau * (uint32_t)tau;
    valid[o] = (a0 <= t2 && a1 <= t2 && af <= t2) ? 1 : 0;
    err[o] = max(max(a0, a1), af);
}

}  // namespace
}  // namespace sff

using namespace sff;

extern "C" sff_status sff_consistency(const sff_params* p, int32_t batch, const int16_t* hyp_fwd,
                                      const int16_t* hyp_inv, uint8_t* valid, uint32_t* err,
                                      void* stream) {
    if (!params_ok(p) || batch < 1 || batch > 65535 || !hyp_fwd || !hyp_inv || !valid || !err)
        return SFF_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(hyp_fwd) & 7) != 0 ||
        (reinterpret_cast<uintptr_t>(hyp_inv) & 7) != 0 || (reinterpret_cast<uintptr_t>(err) & 3) != 0)
        return SFF_ERR_INVALID_ARG;
    hipLaunchKernelGGL(consistency_kernel, dim3((p->W + 63) / 64, (p->H + 3) / 4, batch),
                       dim3(64, 4), 0, as_stream(stream), hyp_fwd, hyp_inv, valid, err, p->H, p->W,
                       p->tau);
    return launch_status();
}
