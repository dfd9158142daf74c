// Static device scratch of lead_decode_noalloc.
//
// The array below is a device global: each GPU the library runs on holds its
// own copy at its own address for the life of the process.  In host code its
// name denotes a host-side stand-in, never device memory, so host code uses
// only the address returned by hipGetSymbolAddress (kernel arguments and
// every other device access go through that pointer).
#include "lead_scratch.hpp"

#include <mutex>

static __device__ __align__(256) unsigned char scratch[lead::kScratchBytes];

namespace lead {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

}  // namespace

hipError_t scratch_address(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_addr[device] = p;
    }
    *out = g_addr[device];
    return hipSuccess;
}

}  // namespace lead
