// Operator application that allocates nothing: the trace buffer (the one
// scratch buffer of sipdg_apply, holding both sides' (u, g) at every shared
// trace point between the trace and the apply stage) lives in a file-scope
// device array of fixed size instead of the handle's own buffer.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is looked up once per device with hipGetSymbolAddress (at
// handle creation, with the handle's device current) and only that address
// is ever handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "api_common.hpp"
#include "sipdg.h"

namespace sipdg {

namespace {

static_assert(SIPDG_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size in whole 256-byte units");

// One copy per device, held until the process ends.
static __device__ __align__(256) unsigned char scratch[SIPDG_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mutex;
void *g_ptr[MAX_DEVICES] = {};

}  // namespace

// Device address of `scratch` on `device` (the current device): looked up on
// the first call for that device, remembered afterwards.
int noalloc_setup(int device) {
    if (device < 0 || device >= MAX_DEVICES) return fail(SIPDG_EINVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (g_ptr[device]) return SIPDG_OK;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(SIPDG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_ptr[device] = p;
    return SIPDG_OK;
}

}  // namespace sipdg

using namespace sipdg;

extern "C" int sipdg_apply_noalloc(sipdg_handle h, const void *x, void *y, int precision, void *stream) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (precision != SIPDG_F64 && precision != SIPDG_F32)
        return fail(SIPDG_EINVAL, "precision must be SIPDG_F64 or SIPDG_F32");
    if (h->ndof == 0) return SIPDG_OK;
    if (!x || !y) return fail(SIPDG_EINVAL, "null argument");
    if (x == y) return fail(SIPDG_EINVAL, "x and y must not alias");
    if (h->flux != SIPDG_FLUX_SHARED)
        return fail(SIPDG_EINVAL, "the allocation-free apply takes the shared-trace flux only");
    const int64_t need = h->tbuf_len * (precision == SIPDG_F64 ? 8 : 4);
    if (need > (int64_t)SIPDG_NOALLOC_SCRATCH_BYTES)
        return fail(SIPDG_EINVAL, "trace buffer of " + std::to_string(need) + " bytes exceeds the " +
                                      std::to_string((long long)SIPDG_NOALLOC_SCRATCH_BYTES) +
                                      "-byte scratch of the allocation-free apply");
    void *p = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        if (h->device >= 0 && h->device < MAX_DEVICES) p = g_ptr[h->device];
    }
    if (!p) return fail(SIPDG_EHIP, "scratch address of the handle's device was not set up at create");
    hipStream_t st = (hipStream_t)stream;
    if (precision == SIPDG_F64) return apply_impl<double>(h, (const double *)x, (double *)y, (double *)p, nullptr, st);
    return apply_impl<float>(h, (const float *)x, (float *)y, (float *)p, nullptr, st);
}
