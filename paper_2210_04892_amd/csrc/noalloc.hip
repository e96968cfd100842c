// Allocation-free variant of the product, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, hosts
// that forbid allocation inside the loop).
//
// The per-product scratch of mlfma_matvec_LK (internal vectors, box patterns
// of every level, the level-step intermediate) lives in one file-scope
// device array of MLFMA_NOALLOC_SCRATCH_BYTES per GPU, held by each device
// the library runs on until the process ends.  Its device address is taken
// once per device with hipGetSymbolAddress and used everywhere host code
// hands the array to the product.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/mlfma.h"
#include "scratch.hpp"

static __device__ __align__(256) unsigned char scratch[MLFMA_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_scratch_ptr[MAX_DEVICES] = {nullptr};

// Device address of this device's copy of the scratch array (taken once,
// with the device current); nullptr and an error text on failure.
void *scratch_of(int dev, std::string &why)
{
    if (dev < 0 || dev >= MAX_DEVICES) {
        why = "device ordinal out of range";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch_ptr[dev]) return g_scratch_ptr[dev];
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev && hipSetDevice(dev) != hipSuccess) {
        why = "hipSetDevice failed";
        return nullptr;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
    if (e != hipSuccess || !p) {
        why = std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(e);
        return nullptr;
    }
    g_scratch_ptr[dev] = p;
    return p;
}

}  // namespace

extern "C" int mlfma_matvec_LK_noalloc(mlfma_handle h, int op, int dtype, long long nrhs, const void *x,
                                       long long ldx, void *y, long long ldy, void *hip_stream)
{
    if (!h) return mlfma::set_error(MLFMA_ERR_ARG, "NULL handle");
    std::string why;
    void *p = scratch_of(mlfma::handle_device(h), why);
    if (!p) return mlfma::set_error(MLFMA_ERR_HIP, why.c_str());
    return mlfma::matvec_in_scratch(h, op, dtype, nrhs, x, ldx, y, ldy, hip_stream, p, MLFMA_NOALLOC_SCRATCH_BYTES);
}
