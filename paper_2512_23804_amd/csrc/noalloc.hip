// Fixed device scratch for the entry point that allocates nothing
// (sg_precond_apply_noalloc).
//
// The array below is a device symbol: host code never passes its name to a
// kernel or a copy (on the host the name is only a stand-in, not a device
// address).  Its address on each device is taken once with
// hipGetSymbolAddress, with that device current, and kept per device; every
// use goes through that address.  Each device holds its own copy until the
// process ends, and every call on a device shares it.
#include <mutex>

#include "handle.hpp"

namespace sg {

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

void* noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) throw Error(SG_ERR_INVALID, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        int cur = -1;
        SG_HIP(hipGetDevice(&cur));
        if (cur != device) throw Error(SG_ERR_INVALID, "the scratch address is resolved with its device current");
        void* p = nullptr;
        SG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error(SG_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_ptr[device] = p;
    }
    return g_ptr[device];
}

}  // namespace sg
