// Calibration kernels for the roofline reported next to the matcher: a
// streaming copy (achievable HBM bandwidth) and random record gathers (the
// access pattern of the propagation / random-search cost evaluations: one
// descriptor record per lane at a data-dependent address).
#include "sff_internal.hpp"

namespace sff {
namespace {

__device__ __forceinline__ uint32_t mix(uint64_t x) {  // splitmix64 finaliser
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return (uint32_t)(x ^ (x >> 31));
}

__global__ void __launch_bounds__(256) copy_kernel(const uint4* __restrict__ src,
                                                   uint4* __restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Each thread owns `per_thread` records of `rec16` 16-byte words at
// pseudo-random record indices in [0, nrec) and folds them into one word.
// coop = 0: a thread loads its own records, one 16-byte word per instruction,
// so one wave-wide load touches 64 unrelated cache lines.  coop = 1: the 64
// records of a wave are loaded word by word by consecutive lanes (lane l of
// load k takes word (64 k + l) mod rec16 of record (64 k + l) / rec16), so one
// load touches the few lines of 64 / rec16 records.  Same records, same bytes.
__global__ void __launch_bounds__(256) gather_kernel(const uint4* __restrict__ buf, size_t nrec,
                                                     int rec16, int per_thread, uint64_t seed,
                                                     int coop, uint32_t* __restrict__ out) {
    const size_t tid = (size_t)blockIdx.x * 256 + threadIdx.x;
    const int lane = threadIdx.x & 63;
    uint32_t acc = 0;
    for (int g = 0; g < per_thread; ++g) {
        for (int k = 0; k < rec16; ++k) {
            size_t owner = tid;
            int word = k;
            if (coop) {
                const int flat = k * 64 + lane;
                owner = tid - lane + flat / rec16;
                word = flat % rec16;
            }
            const size_t r = (size_t)mix(seed ^ (owner * 0x100000001B3ull + g)) % nrec;
            const uint4 v = buf[r * rec16 + word];
            acc ^= v.x + v.y + v.z + v.w;
        }
    }
    out[tid] = acc;
}

}  // namespace
}  // namespace sff

using namespace sff;

extern "C" sff_status sff_probe_copy(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst || bytes < 16 || (bytes & 15) != 0 ||
        (reinterpret_cast<uintptr_t>(src) & 15) != 0 || (reinterpret_cast<uintptr_t>(dst) & 15) != 0)
        return SFF_ERR_INVALID_ARG;
    const size_t n = bytes / 16;
    const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 256 * 64);
    hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, as_stream(stream),
                       static_cast<const uint4*>(src), static_cast<uint4*>(dst), n);
    return launch_status();
}

extern "C" sff_status sff_probe_gather(const void* buf, size_t buf_bytes, int32_t record_bytes,
                                       int32_t threads, int32_t per_thread, uint64_t seed,
                                       int32_t coop, uint32_t* out, void* stream) {
    if (!buf || !out || record_bytes < 16 || record_bytes > 256 || (record_bytes & 15) != 0 ||
        buf_bytes < (size_t)record_bytes || threads < 256 || (threads & 255) != 0 || per_thread < 1 || (coop != 0 && coop != 1) ||
        (reinterpret_cast<uintptr_t>(buf) & 15) != 0)
        return SFF_ERR_INVALID_ARG;
    const size_t nrec = buf_bytes / (size_t)record_bytes;
    hipLaunchKernelGGL(gather_kernel, dim3(threads / 256), dim3(256), 0, as_stream(stream),
                       static_cast<const uint4*>(buf), nrec, record_bytes / 16, per_thread, seed, coop, out);
    return launch_status();
}
