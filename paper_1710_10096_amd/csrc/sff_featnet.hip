// Learned descriptors for the matching cost (in place of the WHT features of
// Section 3.1): per-pixel L2 normalisation of the 32-channel network output,
// quantisation to int16 records for the exact integer matcher, and the triplet
// loss used to train the network on consistent matches.
#include "sff_internal.hpp"

namespace sff {
namespace {

typedef uint16_t bf16_t;

__device__ __forceinline__ float bf2f(bf16_t v) { return __uint_as_float((uint32_t)v << 16); }

__device__ __forceinline__ bf16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (bf16_t)((u >> 16) | ((u & 0xFFFF) ? 0x40 : 0));
    return (bf16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

constexpr int kF = 32;  // feature channels

// d = round(scale * f / max(|f|, eps)), int16; one thread per pixel.
__global__ void quantise_kernel(const bf16_t* __restrict__ f, int16_t* __restrict__ d, size_t npx,
                                float scale) {
    const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= npx) return;
    float v[kF];
    const uint4* src = reinterpret_cast<const uint4*>(f + p * kF);
#pragma unroll
    for (int k = 0; k < kF / 8; ++k) {
        const uint4 w = src[k];
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[8 * k + 2 * j] = bf2f((bf16_t)(ws[j] & 0xFFFF));
            v[8 * k + 2 * j + 1] = bf2f((bf16_t)(ws[j] >> 16));
        }
    }
    float ss = 0.f;
#pragma unroll
    for (int c = 0; c < kF; ++c) ss = fmaf(v[c], v[c], ss);
    const float inv = scale / fmaxf(sqrtf(ss), 1e-12f);
    uint32_t out[kF / 2];
#pragma unroll
    for (int c = 0; c < kF / 2; ++c) {
        const int a = (int)rintf(v[2 * c] * inv), b = (int)rintf(v[2 * c + 1] * inv);
        out[c] = (uint32_t)(uint16_t)(int16_t)a | ((uint32_t)(uint16_t)(int16_t)b << 16);
    }
    uint4* dst = reinterpret_cast<uint4*>(d + p * kF);
#pragma unroll
    for (int k = 0; k < kF / 8; ++k) dst[k] = make_uint4(out[4 * k], out[4 * k + 1], out[4 * k + 2], out[4 * k + 3]);
}

__device__ __forceinline__ float load_norm(const bf16_t* f, float* v) {
    float ss = 0.f;
#pragma unroll
    for (int c = 0; c < kF; ++c) {
        v[c] = bf2f(f[c]);
        ss = fmaf(v[c], v[c], ss);
    }
    const float nrm = fmaxf(sqrtf(ss), 1e-12f);
#pragma unroll
    for (int c = 0; c < kF; ++c) v[c] /= nrm;
    return nrm;
}

// d/dx of x / |x| applied to upstream g: (g - xh (xh . g)) / |x|
__device__ __forceinline__ void norm_back(const float* xh, float nrm, float* g) {
    float dot = 0.f;
#pragma unroll
    for (int c = 0; c < kF; ++c) dot = fmaf(xh[c], g[c], dot);
#pragma unroll
    for (int c = 0; c < kF; ++c) g[c] = (g[c] - xh[c] * dot) / nrm;
}

// One thread per triple (a, p, n) of pixel indices into feat [npx][32]:
// loss = max(0, margin + |a^ - p^|^2 - |a^ - n^|^2) on normalised features;
// gradients (scaled by `weight`) are added to grad [npx][32] (FP32 atomics).
__global__ void triplet_kernel(const bf16_t* __restrict__ feat, int npx,
                               const int32_t* __restrict__ trip, int ntrip, float margin,
                               float weight, float* __restrict__ loss, float* __restrict__ grad) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= ntrip) return;
    const int ia = trip[3 * t], ip = trip[3 * t + 1], in = trip[3 * t + 2];
    if ((unsigned)ia >= (unsigned)npx || (unsigned)ip >= (unsigned)npx ||
        (unsigned)in >= (unsigned)npx) {  // invalid triple: no loss, no gradient
        loss[t] = 0.f;
        return;
    }
    float a[kF], p[kF], q[kF];
    const float na = load_norm(feat + (size_t)ia * kF, a);
    const float np_ = load_norm(feat + (size_t)ip * kF, p);
    const float nn = load_norm(feat + (size_t)in * kF, q);
    float dp = 0.f, dn = 0.f;
#pragma unroll
    for (int c = 0; c < kF; ++c) {
        dp = fmaf(a[c] - p[c], a[c] - p[c], dp);
        dn = fmaf(a[c] - q[c], a[c] - q[c], dn);
    }
    const float l = margin + dp - dn;
    loss[t] = fmaxf(l, 0.f);
    if (!(l > 0.f)) return;
    float ga[kF], gp[kF], gn[kF];
#pragma unroll
    for (int c = 0; c < kF; ++c) {
        ga[c] = 2.f * weight * (q[c] - p[c]);
        gp[c] = -2.f * weight * (a[c] - p[c]);
        gn[c] = 2.f * weight * (a[c] - q[c]);
    }
    norm_back(a, na, ga);
    norm_back(p, np_, gp);
    norm_back(q, nn, gn);
#pragma unroll
    for (int c = 0; c < kF; ++c) {
        atomicAdd(grad + (size_t)ia * kF + c, ga[c]);
        atomicAdd(grad + (size_t)ip * kF + c, gp[c]);
        atomicAdd(grad + (size_t)in * kF + c, gn[c]);
    }
}

// bf16 copy of an FP32 buffer, which is cleared for the next accumulation.
__global__ void take_grad_kernel(float* __restrict__ g, bf16_t* __restrict__ out, size_t n) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    out[i] = f2bf(g[i]);
    g[i] = 0.f;
}

}  // namespace
}  // namespace sff

using namespace sff;

extern "C" sff_status sff_quantise_features(int32_t n, int32_t H, int32_t W, const uint16_t* feat,
                                            float scale, int16_t* desc, void* stream) {
    if (n < 1 || H < 1 || W < 1 || !feat || !desc || !(scale > 0.f) || scale > 8192.f)
        return SFF_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(feat) & 15) != 0 || (reinterpret_cast<uintptr_t>(desc) & 15) != 0)
        return SFF_ERR_INVALID_ARG;
    const size_t npx = (size_t)n * H * W;
    hipLaunchKernelGGL(quantise_kernel, dim3((unsigned)((npx + 255) / 256)), dim3(256), 0,
                       as_stream(stream), feat, desc, npx, scale);
    return launch_status();
}

extern "C" sff_status sff_triplet_loss(int32_t npx, const uint16_t* feat, int32_t ntrip,
                                       const int32_t* triplets, float margin, float weight,
                                       float* loss, float* grad, void* stream) {
    if (npx < 1 || ntrip < 1 || !feat || !triplets || !loss || !grad) return SFF_ERR_INVALID_ARG;
    hipLaunchKernelGGL(triplet_kernel, dim3((ntrip + 255) / 256), dim3(256), 0, as_stream(stream),
                       feat, npx, triplets, ntrip, margin, weight, loss, grad);
    return launch_status();
}

extern "C" sff_status sff_take_grad_bf16(size_t n, float* grad, uint16_t* out, void* stream) {
    if (n < 1 || !grad || !out) return SFF_ERR_INVALID_ARG;
    hipLaunchKernelGGL(take_grad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       as_stream(stream), grad, out, n);
    return launch_status();
}
