// pa_static.hip -- pa_run_static: the plain run with its workspace in a
// fixed device array of the library instead of caller memory, for callers
// that cannot allocate device memory (code under graph capture, serving loops
// that forbid allocation).
//
// The array `scratch` is a file-scope __device__ array: every GPU the library
// runs on holds its own copy until the process ends.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in symbol);
// it uses the device address hipGetSymbolAddress returns, looked up once per
// device with that device current and kept in g_scratch.
#include "pa.h"
#include "pa_device.h"

#include <hip/hip_runtime.h>

#include <mutex>

namespace {

static __device__ __align__(256) uint8_t scratch[PA_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

}  // namespace

namespace pa {

// Device address of this device's scratch array (looked up on first use for
// the device, which must be current), or null with the HIP error in *err.
void *static_scratch(int device, hipError_t *err) {
    *err = hipSuccess;
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        g_scratch[device] = p;
    }
    return g_scratch[device];
}

}  // namespace pa
