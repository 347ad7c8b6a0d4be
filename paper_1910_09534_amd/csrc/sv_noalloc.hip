// reduce_slices for callers that cannot allocate device memory: the work
// buffers of the reduction (bitstrings, FP64 accumulators, partial sums, T
// columns) and the device copy of the queued matrices live in one
// file-scope device array of fixed size instead of the handle's pool.
//
// Host code never uses the array's name as an address (on the host it is a
// stand-in, not device memory): the device address is looked up once per
// device with hipGetSymbolAddress, with that device current, and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/sv.h"
#include "sv_state.h"

namespace {

constexpr size_t kBitsBytes = (size_t)SV_NOALLOC_MAX_BITSTRINGS * 8;
constexpr size_t kAccBytes = (size_t)SV_NOALLOC_MAX_BITSTRINGS * 16;
constexpr size_t kPartBytes = sv::kPartDoubles * 8;
constexpr int kMaxSlices = 1 << SV_NOALLOC_MAX_SLICED;
constexpr size_t kTcolBytes = (size_t)kMaxSlices * kMaxSlices * 16 + (size_t)kMaxSlices * 8;
constexpr size_t kRowmapBytes = (size_t)kMaxSlices * 4;
constexpr size_t kSmallBytes = 64;
constexpr size_t kArenaBytes = (size_t)SV_NOALLOC_MAX_QUEUED_BYTES;

constexpr size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kOffBits = 0;
constexpr size_t kOffAcc = kOffBits + up256(kBitsBytes);
constexpr size_t kOffPart = kOffAcc + up256(kAccBytes);
constexpr size_t kOffTcol = kOffPart + up256(kPartBytes);
constexpr size_t kOffRowmap = kOffTcol + up256(kTcolBytes);
constexpr size_t kOffSmall = kOffRowmap + up256(kRowmapBytes);
constexpr size_t kOffArena = kOffSmall + up256(kSmallBytes);
constexpr size_t kScratchBytes = kOffArena + up256(kArenaBytes);

constexpr int kMaxDevices = 64;
std::mutex g_mu[kMaxDevices];            // one call at a time per device: the array is shared
void* g_ptr[kMaxDevices] = {};           // device address of the array on each device

}  // namespace

__device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// The array's address on device dev (looked up once, with dev current).
int scratch_on(int dev, void** out)
{
    if (g_ptr[dev]) {
        *out = g_ptr[dev];
        return 0;
    }
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return -1;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return -1;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) return -1;
    g_ptr[dev] = p;
    *out = p;
    return 0;
}

}  // namespace

extern "C" int reduce_slices_noalloc(sv_handle h, const void* trailing_c128, int64_t count,
                                     const uint64_t* bitstrings, void* out_c128, double stats[3])
{
    if (!h) return reduce_slices(h, trailing_c128, count, bitstrings, out_c128, stats);   // NULL-handle error
    if (h->poisoned) return SV_ESTATE;
    if (h->tier) {
        h->err = "reduce_slices_noalloc: the state lives in the host tier (resident states only)";
        return SV_EINVAL;
    }
    if (h->timing) {
        h->err = "reduce_slices_noalloc: SV_OPT_TIMING is on (timing events are allocated)";
        return SV_EINVAL;
    }
    if (count > SV_NOALLOC_MAX_BITSTRINGS) {
        h->err = "reduce_slices_noalloc: more than SV_NOALLOC_MAX_BITSTRINGS bitstrings";
        return SV_EINVAL;
    }
    if (h->s > SV_NOALLOC_MAX_SLICED) {
        h->err = "reduce_slices_noalloc: more than SV_NOALLOC_MAX_SLICED sliced qubits";
        return SV_EINVAL;
    }
    if (h->arena.size() > kArenaBytes) {
        h->err = "reduce_slices_noalloc: queued matrices exceed SV_NOALLOC_MAX_QUEUED_BYTES";
        return SV_EINVAL;
    }
    hipDevice_t dev = -1;
    hipError_t e = hipStreamGetDevice(h->stream, &dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        h->err = "reduce_slices_noalloc: cannot tell the stream's device";
        return SV_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_mu[dev]);
    void* base = nullptr;
    if (scratch_on(dev, &base)) {
        h->err = "reduce_slices_noalloc: hipGetSymbolAddress of the work array failed";
        return SV_EDEVICE;
    }
    char* b = (char*)base;
    const sv::WorkBufs wb{b + kOffBits, b + kOffAcc, b + kOffPart, b + kOffTcol, b + kOffRowmap,
                          b + kOffSmall, b + kOffArena, kArenaBytes};
    return sv::reduce_with(h, trailing_c128, count, bitstrings, out_c128, stats, &wb);
}
