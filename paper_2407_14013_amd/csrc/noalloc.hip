// Scratch memory of the allocation-free wc_dsymv_noalloc (include/wcsdp_linalg.h).
//
// wc_dsymv's two passes exchange the tile partial sums through a workspace
// that it allocates and frees around every call.  Callers that must not
// allocate device memory (code under HIP graph capture, tight serving loops)
// use wc_dsymv_noalloc instead: the same kernels, with the workspace in one
// file-scope device array per GPU.  Its device address is looked up once per
// device with hipGetSymbolAddress and kept; host code never passes the
// array's own name to a kernel (on the host that name is only a stand-in).
#include <mutex>

#include "../../include/wcsdp_linalg.h"
#include "common.hpp"

namespace {

constexpr int kSymvNoAllocMaxD = WC_DSYMV_NOALLOC_MAX_D;
constexpr long kSymvTiles1D = (kSymvNoAllocMaxD + 63) / 64;
// symv_ws(d) doubles: a row-sum and a column-sum slot of 64 doubles per tile of the triangle
constexpr long kScratchDoubles = kSymvTiles1D * (kSymvTiles1D + 1) * 64;

__device__ __attribute__((aligned(256))) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on first use).
double* scratch_on_current_device() {
    int dev = -1;
    WC_HIP(hipGetDevice(&dev));
    wc::require(dev >= 0 && dev < kMaxDevices, "wc_dsymv_noalloc: device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        WC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        wc::require(p != nullptr, "wc_dsymv_noalloc: no device address for the scratch array");
        g_scratch[dev] = static_cast<double*>(p);
    }
    return g_scratch[dev];
}

}  // namespace

namespace wc {

double* symv_noalloc_scratch(int d) {
    require(d >= 0 && d <= kSymvNoAllocMaxD, "wc_dsymv_noalloc: d exceeds WC_DSYMV_NOALLOC_MAX_D");
    require(symv_ws(d) <= kScratchDoubles, "wc_dsymv_noalloc: workspace larger than the scratch array");
    return scratch_on_current_device();
}

}  // namespace wc
