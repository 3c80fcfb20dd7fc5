// Stream-ordered device workspace from a memory pool the library owns, one
// per device. Freed blocks stay reserved in the pool (up to kPoolKeep bytes)
// and are handed out again to later calls in stream order, so repeated calls
// neither map fresh pages nor synchronise the device to release their
// workspace. The pools live until the process ends.
#include <mutex>

#include "internal.hpp"

namespace pmlsh {
namespace {

constexpr uint64_t kPoolKeep = uint64_t(8) << 30;
constexpr int kMaxDevices = 64;

std::mutex g_pool_mu;
hipMemPool_t g_pool[kMaxDevices] = {};

hipMemPool_t pool_for_current_device() {
    int dev = 0;
    PMLSH_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(PMLSH_EDEVICE, "device ordinal out of range");
    std::lock_guard<std::mutex> g(g_pool_mu);
    if (!g_pool[dev]) {
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t p = nullptr;
        PMLSH_HIP(hipMemPoolCreate(&p, &props));
        uint64_t keep = kPoolKeep;
        PMLSH_HIP(hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &keep));
        g_pool[dev] = p;
    }
    return g_pool[dev];
}

}  // namespace

void* ws_alloc(size_t bytes, hipStream_t st) {
    void* p = nullptr;
    PMLSH_HIP(hipMallocFromPoolAsync(&p, bytes ? bytes : 1, pool_for_current_device(), st));
    return p;
}

void ws_free(void* p, hipStream_t st) {
    if (p) (void)hipFreeAsync(p, st);
}

}  // namespace pmlsh
