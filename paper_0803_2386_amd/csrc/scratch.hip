// Allocation-free execution (moa_fft_exec_noalloc): the workspace of a
// plan of several levels comes from a static device array that the library
// holds on every GPU it runs on, so the call makes no device allocation and
// can run under stream capture or in a serving loop that forbids hipMalloc.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/moa_fft.h"
#include "fft_internal.h"

// The workspace array.  In host code its name is a host-side stand-in, not a
// device address: only the per-device address from hipGetSymbolAddress
// (device_scratch below) is ever passed to a kernel.
static __device__ __align__(256) unsigned char scratch[MOA_FFT_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {nullptr};

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
moa_status_t device_scratch(void** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MOA_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return MOA_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MOA_ERR_HIP;
        g_ptr[dev] = ptr;
    }
    *out = g_ptr[dev];
    return MOA_OK;
}

}  // namespace

extern "C" moa_status_t moa_fft_exec_noalloc(moa_fft_plan_t p, moa_fft_dir_t dir, const void* in, void* out,
                                             void* stream)
{
    size_t ws_bytes = 0;
    if (const moa_status_t st = moa::check_exec(p, int(dir), in, out, &ws_bytes)) return st;
    void* ws = nullptr;
    if (ws_bytes) {
        if (const moa_status_t st = device_scratch(&ws)) return st;
    }
    return moa::launch_on_workspace(p, int(dir), in, out, ws, static_cast<hipStream_t>(stream));
}
