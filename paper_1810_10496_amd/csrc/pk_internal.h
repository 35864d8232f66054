// pk_internal.h -- declarations shared by the runtime's own source files
// (not part of the C ABI; nothing here is exported to callers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/pk.h"

#define PK_HIDDEN __attribute__((visibility("hidden")))

// Record `msg` as the calling thread's pk_last_error and return `s`.
PK_HIDDEN pk_status pk_internal_fail(pk_status s, const char *msg);

// Check `ctx` and make its device current; *device receives the device index.
PK_HIDDEN pk_status pk_internal_device(pk_context *ctx, int *device);

// Workspace bytes pk_corr needs for (prec, n, m) (the pk_workspace_bytes figure).
PK_HIDDEN size_t pk_internal_corr_ws(pk_precision prec, int64_t n, int64_t m);

// pk_corr with its workspace given.  ws_owned: the workspace is the library's own
// device memory (no caller-allocation checks); otherwise it is checked like any
// caller pointer.
PK_HIDDEN pk_status pk_internal_corr(pk_context *ctx, pk_precision prec, int64_t n, int64_t m, const float *X,
                           int64_t ldx, float eps, float *mean, float *std_, float *R, int64_t ldr,
                           void *ws, size_t ws_bytes, bool ws_owned, hipStream_t stream);

// Per-device set-up of the allocation-free entry points' static scratch (pk_scratch.hip):
// run once per device with that device current; later calls return the first result.
PK_HIDDEN pk_status pk_internal_scratch_setup(int device);
