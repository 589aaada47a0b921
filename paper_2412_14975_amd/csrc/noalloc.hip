// ri_recognize_noalloc: the queued recognition of ri_recognize_async with
// its scratch memory in a fixed device array instead of allocated buffers,
// for callers that must not allocate (code under graph capture, serving
// loops that forbid allocation).
#include <hip/hip_runtime.h>

#include <mutex>

#include "ri.h"

namespace ri {
int set_error(int code, const char *msg);
int recognize_in_arena(const ri_handle *h, const uint8_t *text, size_t n, void *stream, int algo,
                       uint32_t chunks, int32_t *result_dev, void *arena, size_t arena_bytes);
}  // namespace ri

namespace {

constexpr size_t kScratchBytes = RI_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// The scratch of every ri_recognize_noalloc call on a device: one copy per
// device, held until the process ends.  Host code never uses the array's
// name as an address: the device address comes from hipGetSymbolAddress.
__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of the scratch array on the current device (looked up once
// per device, with that device current).
int scratch_address(int device, void **out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return ri::set_error(RI_ERR_DEVICE, "hipGetSymbolAddress of the fixed scratch array failed");
        g_scratch[device] = p;
    }
    *out = g_scratch[device];
    return RI_OK;
}

}  // namespace

extern "C" int ri_recognize_noalloc(const ri_handle *h, const uint8_t *text_dev, size_t n, void *stream, int algo,
                                    uint32_t chunks, int32_t *result_dev) {
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess || device < 0 || device >= kMaxDevices)
        return ri::set_error(RI_ERR_DEVICE, "no current device");
    void *p = nullptr;
    const int rc = scratch_address(device, &p);
    if (rc) return rc;
    return ri::recognize_in_arena(h, text_dev, n, stream, algo, chunks, result_dev, p, kScratchBytes);
}
