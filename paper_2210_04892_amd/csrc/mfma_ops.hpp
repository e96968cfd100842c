// The 16x16x4 matrix-core product of each precision (CDNA4, wave64).  Lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator slot v of
// lane l holds D[row(l / 16, v)][l % 16]: row = 4 (l / 16) + v for
// v_mfma_f32_16x16x4f32 and l / 16 + 4 v for v_mfma_f64_16x16x4f64 (both
// layouts checked on the device).  A complex product is four real ones
// (re x re and -im x im into the real sum, re x im and im x re into the
// imaginary one).
#pragma once
#include <hip/hip_runtime.h>

namespace mlfma {

template <class T>
struct Mf;
template <>
struct Mf<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ inline v4 mma(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int kk, int v) { return kk * 4 + v; }
};
template <>
struct Mf<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ inline v4 mma(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int kk, int v) { return kk + 4 * v; }
};

}  // namespace mlfma
