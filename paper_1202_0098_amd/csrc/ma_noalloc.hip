// Scratch of the allocation-free solve (ma_solve_columns_noalloc): a
// file-scope device array that the code object holds on every device the
// library runs on, for the life of the process.  Host code never passes the
// array's name to a kernel: its device address is looked up once per device
// (with that device current) and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ma_internal.h"

namespace ma {

namespace {

static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;

}  // namespace

hipError_t scratch_address(int device, void **ptr, size_t *bytes)
{
    static std::mutex lock;
    static void *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(lock);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;   // the caller makes it current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *ptr = addr[device];
    *bytes = kScratchBytes;
    return hipSuccess;
}

}  // namespace ma
