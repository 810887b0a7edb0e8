// Entry points for callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).  Their kernels take their scratch
// memory from one static array of the library, resolved per device at set-up; they call no
// hipMalloc, hipFree or allocating library routine.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/hho.h"
#include "internal.h"

namespace {

// Scratch of the no-allocation entry points: 2 MiB per device, held until the process ends.
constexpr size_t kScratchDoubles = size_t(1) << 18;
static __device__ __align__(256) double scratch[kScratchDoubles];

// Device address of `scratch` on each device (the array's name is a host-side stand-in and must
// never be passed to a kernel or a copy); set once per device by hho::noalloc_init.
constexpr int kMaxDevices = 64;
std::mutex g_mutex;
double *g_scratch[kMaxDevices] = {};

}  // namespace

namespace hho {

std::string noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return "no-allocation scratch: device ordinal out of range";
    std::lock_guard<std::mutex> lock(g_mutex);
    if (g_scratch[device]) return "";
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return "no-allocation scratch: hipGetDevice failed";
    if (cur != device && hipSetDevice(device) != hipSuccess) return "no-allocation scratch: hipSetDevice failed";
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr)
        return std::string("no-allocation scratch: hipGetSymbolAddress: ") + hipGetErrorString(e);
    g_scratch[device] = (double *)ptr;
    return "";
}

}  // namespace hho

extern "C" hho_status hho_energy_noalloc(hho_ctx *ctx, double *E) {
    if (!ctx) return HHO_ERR_ARG;
    if (!E) {
        hho::ctx_set_error(ctx, "energy_noalloc: null output");
        return HHO_ERR_ARG;
    }
    const int dev = hho::ctx_device(ctx);
    if (hipSetDevice(dev) != hipSuccess) {
        hho::ctx_set_error(ctx, "energy_noalloc: hipSetDevice failed");
        return HHO_ERR_DEVICE;
    }
    double *part = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        part = g_scratch[dev];
    }
    if (!part) {  // set up at hho_setup; a context always has it
        hho::ctx_set_error(ctx, "energy_noalloc: scratch of the device not set up");
        return HHO_ERR_DEVICE;
    }
    return hho::energy_into(ctx, part, kScratchDoubles, E);
}
