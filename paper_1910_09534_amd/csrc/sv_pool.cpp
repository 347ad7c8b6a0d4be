// Caching allocator for the library's small device and pinned-host work
// buffers (operation arenas, bitstring and accumulator buffers, reduction
// partials).  Freed buffers go to per-size-class free lists instead of
// hipFree / hipHostFree, which can wait for the whole device: with many
// states created and destroyed while others run (a serving loop) that wait
// would serialise otherwise independent streams.  Buffers are only returned
// to the pool after their owner synchronised its streams, so a pooled
// buffer is idle.  Sizes round up to a power of two (at least 4 KiB);
// classes above 1 GiB are not pooled.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <vector>

#include "sv_internal.h"

namespace sv {

namespace {

struct Pool {
    std::mutex mu;
    std::map<size_t, std::vector<void*>> dev, host;
};

Pool& pool()
{
    static Pool* p = new Pool();   // never destroyed: buffers live until process exit
    return *p;
}

size_t size_class(size_t bytes)
{
    size_t c = 4096;
    while (c < bytes) c <<= 1;
    return c;
}

constexpr size_t kMaxPooled = (size_t)1 << 30;

}  // namespace

void* pool_alloc(size_t bytes, bool pinned_host, size_t* got)
{
    const size_t c = size_class(bytes);
    if (c <= kMaxPooled) {
        Pool& P = pool();
        std::lock_guard<std::mutex> g(P.mu);
        auto& lst = (pinned_host ? P.host : P.dev)[c];
        if (!lst.empty()) {
            void* p = lst.back();
            lst.pop_back();
            if (got) *got = c;
            return p;
        }
    }
    void* p = nullptr;
    const hipError_t e = pinned_host ? hipHostMalloc(&p, c, hipHostMallocDefault) : hipMalloc(&p, c);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (got) *got = c;
    return p;
}

void pool_free(void* p, size_t bytes, bool pinned_host)
{
    if (!p) return;
    const size_t c = size_class(bytes);
    if (c > kMaxPooled) {
        if (pinned_host) (void)hipHostFree(p);
        else (void)hipFree(p);
        return;
    }
    Pool& P = pool();
    std::lock_guard<std::mutex> g(P.mu);
    (pinned_host ? P.host : P.dev)[c].push_back(p);
}

}  // namespace sv
