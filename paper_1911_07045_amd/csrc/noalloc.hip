// Fixed workspace of lq_minimize_noalloc: a device array that each GPU the
// library runs on holds until the process ends, for callers that cannot
// allocate device memory.
//
// Host code must not use the array's name as an address: on the host it is a
// stand-in, not device memory.  The device address comes from
// hipGetSymbolAddress, looked up once per device with that device current,
// and only that address is passed on.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lq_aux.h"

static __device__ __align__(256) unsigned char scratch[LQ_NOALLOC_WORKSPACE_BYTES];

namespace lq {

int noalloc_workspace(int device, void** out) {
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static void* ptr[MAX_DEVICES] = {};
    if (!out || device < 0 || device >= MAX_DEVICES) return LQ_EINVAL;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return LQ_EHIP;
        }
        ptr[device] = p;
    }
    *out = ptr[device];
    return LQ_OK;
}

}  // namespace lq
