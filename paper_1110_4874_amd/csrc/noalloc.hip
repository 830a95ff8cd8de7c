// Fixed device scratch for sht_synthesis_noalloc, the synthesis entry point
// for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation).
//
// The array below is the workspace that sht_synthesis_ex otherwise takes
// from the caller or allocates: the Legendre phase buffer q and, on the
// butterfly path, the level vectors.  Every GPU the library runs on holds
// its own copy for the life of the process.  In host code its name is only
// a host-side stand-in; the device address is looked up once per device
// (with that device current) and kept, and only that address is ever
// passed to kernels.  Nothing in a synthesis reads workspace memory before
// writing it, so the array needs no clearing between calls; calls that
// overlap on one GPU share it and race.
#include <mutex>

#include "internal.h"

namespace sht {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};
}  // namespace

// Device address of the scratch array on `dev`, which must be the current
// device; looked up on the first call for that device.
int noalloc_scratch(int dev, void **out) {
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return fail(SHT_EUNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(SHT_EDEVICE, std::string("scratch symbol address: ") + hipGetErrorString(e));
        }
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return SHT_OK;
}

}  // namespace sht
