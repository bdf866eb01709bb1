// The library's helper streams: one per device, with a fork and a join event,
// for calls that run two independent launch sequences concurrently (the two
// fields of a match level; the reference and target gradients of the FP32
// window cost).
#include <mutex>

#include "sff_internal.hpp"

namespace sff {
namespace {

constexpr int kMaxHelperDevices = 64;
std::mutex helper_mutex;
HelperStream helpers[kMaxHelperDevices];

}  // namespace

std::mutex& helper_lock() { return helper_mutex; }

HelperStream* helper_for_current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxHelperDevices) return nullptr;
    HelperStream& h = helpers[dev];
    if (!h.stream) {
        hipStream_t s = nullptr;
        hipEvent_t f = nullptr, j = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
        if (hipEventCreateWithFlags(&f, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&j, hipEventDisableTiming) != hipSuccess) {
            if (f) (void)hipEventDestroy(f);
            (void)hipStreamDestroy(s);
            return nullptr;
        }
        h.stream = s;
        h.fork = f;
        h.join = j;
    }
    return &h;
}

bool helper_fork(HelperStream* h, hipStream_t st) {
    return hipEventRecord(h->fork, st) == hipSuccess && hipStreamWaitEvent(h->stream, h->fork, 0) == hipSuccess;
}

bool helper_join(HelperStream* h, hipStream_t st) {
    return hipEventRecord(h->join, h->stream) == hipSuccess && hipStreamWaitEvent(st, h->join, 0) == hipSuccess;
}

}  // namespace sff
