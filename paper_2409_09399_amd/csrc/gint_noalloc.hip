// Static device scratch for the entry point that allocates nothing
// (gint_energy_noalloc).  The array lives in the library's code object: each
// GPU that runs the library holds its own copy until the process ends.  Host
// code never uses the array's name as an address (on the host it is only a
// stand-in for the symbol); the device address of each GPU's copy is looked
// up once per device with hipGetSymbolAddress and cached here.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gint_internal.h"

// Bytes of the static scratch: the per-system partial sums of the two-pass
// energy reduction (kParts doubles per system).
#define GINT_STATIC_SCRATCH_BYTES (1 << 20)

static __device__ __align__(256) unsigned char scratch[GINT_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of the current device's copy of `scratch` (looked up on the
// first call for that device, with the device current) and its size.
// Returns hipSuccess or the error of the lookup; *ptr is then null.
hipError_t gint_static_scratch(void **ptr, size_t *bytes) {
    *ptr = nullptr;
    *bytes = GINT_STATIC_SCRATCH_BYTES;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}
