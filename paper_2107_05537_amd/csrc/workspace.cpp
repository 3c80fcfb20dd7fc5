// Device workspace of the library's calls: a caching allocator, one per
// device. A released block is kept with the stream it was released on and an
// event recorded there; it is handed out again at once to a request on the
// same stream (stream order makes that safe) and to a request on another
// stream once its event has completed. New blocks come from hipMalloc (sizes
// rounded up to 1 MiB, or 64 MiB above 256 MiB), only when no cached block
// fits, so repeated calls neither map fresh pages nor synchronise the device.
// Cached blocks are held until the process ends; the device holds at most
// the peak workspace of the calls that overlapped.
#include <map>
#include <mutex>
#include <unordered_map>

#include "internal.hpp"

namespace pmlsh {
namespace {

constexpr int kMaxDevices = 64;

struct Block {
    size_t size = 0;
    hipStream_t stream = nullptr;   // stream of the last release
    hipEvent_t ready = nullptr;     // recorded on it at the release
};

struct Cache {
    std::mutex mu;
    std::unordered_map<void*, Block> live;      // handed out
    std::multimap<size_t, std::pair<void*, Block>> free_blocks;   // by size
};

Cache g_cache[kMaxDevices];

size_t rounded(size_t bytes) {
    const size_t q = bytes > (size_t(256) << 20) ? size_t(64) << 20 : size_t(1) << 20;
    return (bytes + q - 1) / q * q;
}

Cache& cache_for_current_device() {
    int dev = 0;
    PMLSH_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(PMLSH_EDEVICE, "device ordinal out of range");
    return g_cache[dev];
}

}  // namespace

void* ws_alloc(size_t bytes, hipStream_t st) {
    Cache& c = cache_for_current_device();
    const size_t want = rounded(bytes ? bytes : 1);
    std::lock_guard<std::mutex> g(c.mu);
    // smallest cached block that fits and is free for this stream
    for (auto it = c.free_blocks.lower_bound(want); it != c.free_blocks.end(); ++it) {
        Block& b = it->second.second;
        if (b.stream == st || hipEventQuery(b.ready) == hipSuccess) {
            void* p = it->second.first;
            c.live[p] = b;
            c.free_blocks.erase(it);
            return p;
        }
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e == hipErrorOutOfMemory && !c.free_blocks.empty()) {
        // give the cached blocks that are idle back and try once more
        (void)hipGetLastError();
        for (auto it = c.free_blocks.begin(); it != c.free_blocks.end();) {
            Block& b = it->second.second;
            if (hipEventQuery(b.ready) == hipSuccess) {
                (void)hipEventDestroy(b.ready);
                (void)hipFree(it->second.first);
                it = c.free_blocks.erase(it);
            } else {
                ++it;
            }
        }
        e = hipMalloc(&p, want);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? PMLSH_ENOMEM : PMLSH_EDEVICE,
             std::string("hipMalloc of the workspace: ") + hipGetErrorString(e));
    }
    Block b;
    b.size = want;
    if (hipEventCreateWithFlags(&b.ready, hipEventDisableTiming) != hipSuccess) {
        (void)hipFree(p);
        fail(PMLSH_EDEVICE, "hipEventCreate for the workspace failed");
    }
    c.live[p] = b;
    return p;
}

void ws_free(void* p, hipStream_t st) {
    if (!p) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return;
    Cache& c = g_cache[dev];
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) return;
    Block b = it->second;
    c.live.erase(it);
    b.stream = st;
    if (hipEventRecord(b.ready, st) != hipSuccess) {
        // no event: wait for the stream so the block is idle when reused
        (void)hipStreamSynchronize(st);
        (void)hipEventRecord(b.ready, nullptr);
    }
    c.free_blocks.emplace(b.size, std::make_pair(p, b));
}

}  // namespace pmlsh
