// pk_scratch.hip -- the library's one piece of static device memory, and the
// allocation-free entry point that uses it (pk_corr_noalloc, include/pk.h).
//
// `scratch` is a file-scope device array.  On the host its name is only a
// stand-in for the symbol, not a device address, so it is never passed to a
// kernel or a copy: pk_internal_scratch_setup takes the array's device address
// with hipGetSymbolAddress, once per device with that device current (each
// device holds its own copy at its own address), and every later use goes
// through that address.  The array lives until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pk_internal.h"

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[PK_NOALLOC_SCRATCH_BYTES];

std::once_flag g_once[kMaxDevices];
void *g_ptr[kMaxDevices];
hipError_t g_status[kMaxDevices];

}  // namespace

pk_status pk_internal_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices)
        return pk_internal_fail(PK_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::call_once(g_once[device], [device] {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_status[device] = e;
        g_ptr[device] = e == hipSuccess ? p : nullptr;
        if (e != hipSuccess)
            (void)hipGetLastError();
    });
    if (g_status[device] != hipSuccess || !g_ptr[device]) {
        char msg[256];
        snprintf(msg, sizeof msg, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                 hipGetErrorString(g_status[device]));
        return pk_internal_fail(PK_ERR_HIP, msg);
    }
    return PK_OK;
}

extern "C" pk_status pk_corr_noalloc(pk_context *ctx, pk_precision prec, int64_t n, int64_t m,
                                     const float *X, int64_t ldx, float eps, float *mean, float *std_,
                                     float *R, int64_t ldr, pk_stream stream) {
    try {
        int device = -1;
        pk_status st = pk_internal_device(ctx, &device);
        if (st != PK_OK)
            return st;
        st = pk_internal_scratch_setup(device);   // done at context creation; here it only reads
        if (st != PK_OK)
            return st;
        return pk_internal_corr(ctx, prec, n, m, X, ldx, eps, mean, std_, R, ldr, g_ptr[device],
                                PK_NOALLOC_SCRATCH_BYTES, true, (hipStream_t)stream);
    } catch (...) {
        return pk_internal_fail(PK_ERR_INVALID_ARG, "internal error");
    }
}
