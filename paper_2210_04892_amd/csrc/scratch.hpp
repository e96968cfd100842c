// Internal interface between the C boundary (capi.cpp) and the
// allocation-free entry point (noalloc.hip).
#pragma once

#include "../../include/mlfma.h"

namespace mlfma {

// Device ordinal of the handle (-1 for NULL).
int handle_device(mlfma_handle h);
// Record msg as the calling thread's last error; returns code.
int set_error(int code, const char *msg);
// y = A x as mlfma_matvec_LK, with the product's scratch laid over the cap
// bytes at device address scratch (256-byte aligned); MLFMA_ERR_ARG if the
// product needs more.  Allocates nothing.
int matvec_in_scratch(mlfma_handle h, int op, int dtype, long long nrhs, const void *x, long long ldx, void *y,
                      long long ldy, void *hip_stream, void *scratch, unsigned long long cap);

}  // namespace mlfma
