// Fixed device scratch for the entry point that allocates nothing
// (hdg_residual_norm_noalloc): callers that cannot call hipMalloc, such as code under
// graph capture, tight serving loops or harnesses that forbid allocation.
//
// The array below is a file-scope device variable: each GPU the library runs on holds
// its own copy for the life of the process. In host code its name is only a host-side
// stand-in, so its device address is looked up once per device (hipGetSymbolAddress,
// with that device current, at context creation) and only that address is used from
// then on. Every call on one GPU shares that GPU's copy, so calls that overlap on one
// GPU (two contexts, two streams, two threads) race; calls on one stream do not.
#include <mutex>

#include "hdg_internal.hpp"

namespace {

static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_ptr[MAX_DEVICES] = {};

}  // namespace

// Looks up this device's copy of the scratch array (the device must be current).
hdg_status noalloc_scratch_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) return HDG_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return HDG_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        return HDG_ERR_HIP;
    }
    g_ptr[device] = (double*)p;
    return HDG_OK;
}

// The device address of `device`'s scratch array, or nullptr before noalloc_scratch_init.
double* noalloc_scratch(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[device];
}
