// Machine-peak probes: the ceilings the product's kernels are measured
// against, taken on the device the library runs on instead of the published
// figures alone.
//   kind 0: HBM bandwidth of a plain copy (16-byte loads and stores, every
//           byte read once and written once), GB/s counting both directions;
//   kind 1: FP32 matrix-core rate of v_mfma_f32_16x16x4f32 (2 x 16 x 16 x 4
//           flops per instruction), TFLOP/s;
//   kind 2: FP32 vector fused multiply-add rate (non-packed, as every kernel
//           of the library is compiled), TFLOP/s.
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/mlfma.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// A workgroup copies one contiguous 16 KiB block: four 16-byte elements per
// thread, consecutive threads on consecutive elements, all loads issued
// before the stores.
__global__ __launch_bounds__(256) void k_probe_copy(const f4 *__restrict__ src, f4 *__restrict__ dst, long long n)
{
    const long long base = (long long)blockIdx.x * 1024 + threadIdx.x;
    f4 v[4];
#pragma unroll
    for (int u = 0; u < 4; u++) v[u] = base + u * 256 < n ? src[base + u * 256] : f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < 4; u++)
        if (base + u * 256 < n) dst[base + u * 256] = v[u];
}

// Eight independent accumulator chains per wave keep the matrix unit busy;
// the operands change every step so nothing is hoisted.
__global__ __launch_bounds__(256) void k_probe_mfma(int iters, float seed, float *__restrict__ out)
{
    f4 acc[8];
#pragma unroll
    for (int j = 0; j < 8; j++) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
    float a = seed + threadIdx.x * 1e-3f, b = seed - threadIdx.x * 1e-3f;
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int j = 0; j < 8; j++) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[j], 0, 0, 0);
        a += 1e-7f;
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 8; j++) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    out[(long long)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Sixteen independent FMA chains per thread.
__global__ __launch_bounds__(256) void k_probe_fma(int iters, float seed, float *__restrict__ out)
{
    float v[16];
#pragma unroll
    for (int j = 0; j < 16; j++) v[j] = seed + (threadIdx.x + j) * 1e-6f;
    const float m = 0.999999f, c = 1e-7f;
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int j = 0; j < 16; j++) v[j] = __builtin_fmaf(v[j], m, c);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 16; j++) s += v[j];
    out[(long long)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" int mlfma_peak_probe(int kind, int device, double *value)
{
    if (!value || kind < 0 || kind > 2) return MLFMA_ERR_ARG;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return MLFMA_ERR_HIP;
    if (device >= 0 && hipSetDevice(device) != hipSuccess) return MLFMA_ERR_ARG;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device >= 0 ? device : prev) != hipSuccess)
        cus = 0;
    if (cus <= 0) cus = 256;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void *a = nullptr, *b = nullptr;
    int rc = MLFMA_OK;
    do {
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
            hipEventCreate(&e1) != hipSuccess) {
            rc = MLFMA_ERR_HIP;
            break;
        }
        const long long copy_bytes = 1LL << 30;
        const unsigned blocks = (unsigned)cus * 8;
        const int threads = 256;
        size_t bytes = kind == 0 ? (size_t)copy_bytes : (size_t)blocks * threads * sizeof(float);
        if (hipMalloc(&a, bytes) != hipSuccess || (kind == 0 && hipMalloc(&b, bytes) != hipSuccess)) {
            rc = MLFMA_ERR_OOM;
            break;
        }
        if (hipMemsetAsync(a, 0, bytes, st) != hipSuccess) {
            rc = MLFMA_ERR_HIP;
            break;
        }
        const int iters = 4096;
        auto launch = [&]() {
            if (kind == 0)
                hipLaunchKernelGGL(k_probe_copy, dim3((unsigned)(copy_bytes / 16 / 1024)), dim3(threads), 0, st,
                                   (const f4 *)a, (f4 *)b, copy_bytes / 16);
            else if (kind == 1)
                hipLaunchKernelGGL(k_probe_mfma, dim3(blocks), dim3(threads), 0, st, iters, 1.0f, (float *)a);
            else
                hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(threads), 0, st, iters, 1.0f, (float *)a);
        };
        launch();   // warm-up
        const int reps = 5;
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps; r++) launch();
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess || hipGetLastError() != hipSuccess) {
            rc = MLFMA_ERR_HIP;
            break;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double sec = ms * 1e-3 / reps;
        const double waves = (double)blocks * threads / 64.0;
        if (kind == 0) *value = 2.0 * copy_bytes / sec / 1e9;
        else if (kind == 1) *value = waves * iters * 8.0 * 2048.0 / sec / 1e12;
        else *value = (double)blocks * threads * iters * 16.0 * 2.0 / sec / 1e12;
    } while (false);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (prev >= 0) (void)hipSetDevice(prev);
    return rc;
}
