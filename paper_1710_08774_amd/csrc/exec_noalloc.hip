// hfav_execute_noalloc: hfav_execute with the workspace taken from a static
// device array instead of a caller's buffer, for callers that cannot
// allocate device memory.
//
// In host code the name `scratch` is only the host-side stand-in the HIP
// runtime registers for the device array: it is never passed to a kernel or
// a copy.  The device address is looked up once per device, with that device
// current, and kept in `g_scratch`; each device holds its own copy of the
// array at its own address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

static __device__ __align__(256) unsigned char scratch[HFAV_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_lock;
void *g_scratch[MAX_DEVICES];       // device address of `scratch` per device (null: not looked up)

// Device address of the static array on the current device (looked up on
// the first call on that device); null after an error reported through
// hfav_fail.
void *device_scratch() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
        hfav_fail(HFAV_EDEVICE, "hfav_execute_noalloc: no current device");
        return nullptr;
    }
    if (dev >= MAX_DEVICES) {
        hfav_fail(HFAV_EDEVICE, "hfav_execute_noalloc: device index above 63");
        return nullptr;
    }
    std::lock_guard<std::mutex> hold(g_lock);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            hfav_fail(HFAV_EDEVICE, std::string("hfav_execute_noalloc: address of the static workspace: ") +
                                        hipGetErrorString(e));
            return nullptr;
        }
        g_scratch[dev] = ptr;
    }
    return g_scratch[dev];
}

}  // namespace

extern "C" int hfav_execute_noalloc(hfav_chain *c, const void *const *axioms, void *const *goals, void *stream) {
    if (!c) return hfav_fail(HFAV_EINVAL, "null chain");
    if (!c->plan.valid) return hfav_fail(HFAV_ENOPLAN, "hfav_execute_noalloc before a successful hfav_plan");
    if (c->plan.ws_bytes > HFAV_STATIC_WORKSPACE_BYTES)
        return hfav_fail(HFAV_ESIZE, "this plan needs a workspace of " + std::to_string(c->plan.ws_bytes) +
                                         " bytes; the static workspace holds " +
                                         std::to_string(HFAV_STATIC_WORKSPACE_BYTES));
    void *ws = nullptr;
    if (c->plan.ws_bytes > 0) {
        ws = device_scratch();
        if (!ws) return HFAV_EDEVICE;
    }
    return hfav_execute_ws(c, axioms, goals, ws, stream);
}
