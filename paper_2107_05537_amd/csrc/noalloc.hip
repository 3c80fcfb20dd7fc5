// pmlsh_ann_noalloc: the (c,k)-ANN call of pmlsh_ann for callers that cannot
// allocate device memory. Its workspace is a fixed array in the library's
// code object (one copy per device, held until the process ends) instead of
// blocks from the caching allocator; the kernels and results are those of
// pmlsh_ann.
//
// The array's name is a host-side stand-in: its device address is looked up
// once per device with hipGetSymbolAddress (that device current) and only
// that address is ever handed to kernels.

#include <mutex>

#include "internal.hpp"

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[PMLSH_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of the current device's copy of the scratch array.
void* scratch_on_current_device() {
    int dev = 0;
    PMLSH_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) pmlsh::fail(PMLSH_EDEVICE, "device ordinal out of range");
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        PMLSH_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) pmlsh::fail(PMLSH_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}

}  // namespace

extern "C" int pmlsh_ann_noalloc(const pmlsh_index* index, const float* queries, int64_t nq,
                                 int32_t k, double c, double confidence, double beta,
                                 double r_min, int64_t* out_ids, float* out_dist,
                                 int32_t* out_stats, void* stream) {
    return pmlsh::guarded([&] {
        pmlsh::validate_ann(index, queries, nq, k, out_ids, out_dist, r_min);
        pmlsh::TimingOff no_events;
        pmlsh::run_ann_in(index, queries, nq, k, c, confidence, beta, r_min, out_ids, out_dist,
                          out_stats, static_cast<hipStream_t>(stream), scratch_on_current_device,
                          (int64_t)PMLSH_NOALLOC_SCRATCH_BYTES);
    });
}
