// hsgd_refine_noalloc: the coarse-to-fine refinement with its workspace in a static device
// array, for callers that cannot allocate device memory.
//
// The array below is the library's own device memory on every GPU it runs on: the code
// object that holds it is loaded once per device, and each device's copy lives at its own
// address until the process ends. In host code `scratch` names a host-side stand-in, not a
// device address, so the kernels are never given it: each device's address comes from
// hipGetSymbolAddress, called once per device with that device current, and only that
// address is passed on.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hsgd_internal.h"

namespace hsgd {
namespace {

static_assert(HSGD_NOALLOC_SCRATCH_BYTES % kAlign == 0, "scratch size is a whole number of alignment units");

static __device__ __align__(256) unsigned char scratch[HSGD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch` per device, once looked up

// The device the caller's stream runs on (the current device for the null stream).
hipError_t stream_device(hipStream_t stream, int* dev) {
    if (stream == nullptr) return hipGetDevice(dev);
    hipDevice_t d = 0;
    const hipError_t e = hipStreamGetDevice(stream, &d);
    if (e == hipSuccess) *dev = (int)d;
    return e;
}

// Device address of `scratch` on device dev: looked up on first use with dev current (the
// caller's current device is restored afterwards), then kept.
hipError_t scratch_on(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        const hipError_t r = cur != dev ? hipSetDevice(cur) : hipSuccess;
        if (e != hipSuccess) return e;
        if (r != hipSuccess) return r;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace hsgd

using namespace hsgd;

extern "C" hsgd_status hsgd_refine_noalloc(hsgd_mpi* levels, const hsgd_views* views, int32_t L,
                                           const int32_t* iters, hsgd_select_params sel, float lr_rgb,
                                           float lr_alpha, float lambda_s, float* loss_log,
                                           hipStream_t stream) {
    clear_error();
    const char* fn = "hsgd_refine_noalloc";
    size_t need = 0;
    hsgd_status st = refine_check(fn, levels, views, L, iters, sel, lr_rgb, lr_alpha, lambda_s, &need);
    if (st) return st;
    if (need > HSGD_NOALLOC_SCRATCH_BYTES)
        return fail(HSGD_E_WORKSPACE,
                    "%s: this refine needs %zu bytes of workspace; the static scratch holds %zu "
                    "(use hsgd_refine with a caller-allocated workspace)",
                    fn, need, (size_t)HSGD_NOALLOC_SCRATCH_BYTES);
    int dev = 0;
    hipError_t e = stream_device(stream, &dev);
    if (e != hipSuccess) return hip_status(e, fn);
    void* ws = nullptr;
    e = scratch_on(dev, &ws);
    if (e != hipSuccess) return hip_status(e, fn);
    return refine_run(fn, levels, views, L, iters, sel, lr_rgb, lr_alpha, lambda_s, loss_log, ws, stream);
}
