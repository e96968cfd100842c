// Vector kernels of the outer GMRES (restarted, one Krylov space per
// right-hand-side column).  Vectors are column-major blocks: element (n, r)
// of a block with leading dimension ld sits at r * ld + n.  Inner products
// are accumulated in double precision in a fixed order (partial sums per
// chunk of rows, then a second pass over the chunks), so results do not
// depend on the launch.
#include "device.hpp"

namespace mlfma {

namespace {

constexpr int KT = 256;

__device__ inline double wave_sum_d(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// part[(i * nchunk + c) * nrhs + r] = sum over rows of chunk c of conj(V_i(n, r)) w(n, r)
template <class T>
__global__ __launch_bounds__(KT) void k_dots(const cpx<T> *__restrict__ V, long long vstride, long long ldv, int nv,
                                             const cpx<T> *__restrict__ w, long long ldw, long long n, long long chunk,
                                             cpx<double> *__restrict__ part, int nchunk, int nrhs)
{
    __shared__ double red[2][KT / 64];
    const int c = blockIdx.x, r = blockIdx.y;
    const long long n0 = (long long)c * chunk, n1 = n0 + chunk < n ? n0 + chunk : n;
    const cpx<T> *wr = w + (long long)r * ldw;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i = 0; i < nv; i++) {
        const cpx<T> *vi = V + i * vstride + (long long)r * ldv;
        double sre = 0, sim = 0;
        for (long long k = n0 + threadIdx.x; k < n1; k += KT) {
            const cpx<T> a = vi[k], b = wr[k];
            sre += (double)a.re * (double)b.re + (double)a.im * (double)b.im;
            sim += (double)a.re * (double)b.im - (double)a.im * (double)b.re;
        }
        sre = wave_sum_d(sre);
        sim = wave_sum_d(sim);
        if (lane == 0) {
            red[0][wv] = sre;
            red[1][wv] = sim;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0, b = 0;
            for (int k = 0; k < KT / 64; k++) {
                a += red[0][k];
                b += red[1][k];
            }
            part[((long long)i * nchunk + c) * nrhs + r] = {a, b};
        }
        __syncthreads();
    }
}

// out[i * nrhs + r] = sum over chunks of part
__global__ void k_sum_parts(const cpx<double> *__restrict__ part, int nv, int nchunk, int nrhs,
                            cpx<double> *__restrict__ out)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nv * nrhs) return;
    const int i = g / nrhs, r = g % nrhs;
    double a = 0, b = 0;
    for (int c = 0; c < nchunk; c++) {
        const cpx<double> p = part[((long long)i * nchunk + c) * nrhs + r];
        a += p.re;
        b += p.im;
    }
    out[g] = {a, b};
}

// w(n, r) += sign * sum_{i < nv} V_i(n, r) h[i * nrhs + r]
template <class T>
__global__ __launch_bounds__(KT) void k_combine(const cpx<T> *__restrict__ V, long long vstride, long long ldv, int nv,
                                                const cpx<double> *__restrict__ h, double sign, cpx<T> *__restrict__ w,
                                                long long ldw, long long n, int nrhs)
{
    const long long g = (long long)blockIdx.x * KT + threadIdx.x;
    if (g >= n * nrhs) return;
    const int r = (int)(g / n);
    const long long k = g % n;
    double are = 0, aim = 0;
    for (int i = 0; i < nv; i++) {
        const cpx<T> v = V[i * vstride + (long long)r * ldv + k];
        const cpx<double> c = h[i * nrhs + r];
        are += (double)v.re * c.re - (double)v.im * c.im;
        aim += (double)v.re * c.im + (double)v.im * c.re;
    }
    cpx<T> &o = w[(long long)r * ldw + k];
    o = {(T)((double)o.re + sign * are), (T)((double)o.im + sign * aim)};
}

// y(n, r) = a[r] x(n, r) + b[r] z(n, r)  (z may be null: b ignored)
template <class T>
__global__ __launch_bounds__(KT) void k_axpby(const cpx<double> *__restrict__ a, const cpx<T> *__restrict__ x,
                                              long long ldx, const cpx<double> *__restrict__ b,
                                              const cpx<T> *__restrict__ z, long long ldz, cpx<T> *__restrict__ y,
                                              long long ldy, long long n, int nrhs)
{
    const long long g = (long long)blockIdx.x * KT + threadIdx.x;
    if (g >= n * nrhs) return;
    const int r = (int)(g / n);
    const long long k = g % n;
    const cpx<T> xv = x[(long long)r * ldx + k];
    double re = a[r].re * xv.re - a[r].im * xv.im, im = a[r].re * xv.im + a[r].im * xv.re;
    if (z) {
        const cpx<T> zv = z[(long long)r * ldz + k];
        re += b[r].re * zv.re - b[r].im * zv.im;
        im += b[r].re * zv.im + b[r].im * zv.re;
    }
    y[(long long)r * ldy + k] = {(T)re, (T)im};
}

// y(i, r) = alpha * sum_k val[k] x(col[k], r) over row i's entries of a CSR
// matrix (plus y(i, r) when accumulate); thread per (row, right-hand side),
// rows fastest so a wave writes consecutive elements of one column.
template <class T>
__global__ __launch_bounds__(KT) void k_csr_spmm(long long nrows, int nrhs, const long long *__restrict__ ptr,
                                                 const int *__restrict__ col, const cpx<T> *__restrict__ val,
                                                 const cpx<T> *__restrict__ x, long long ldx, cpx<T> *__restrict__ y,
                                                 long long ldy, double alpha, int accumulate)
{
    const long long g = (long long)blockIdx.x * KT + threadIdx.x;
    if (g >= nrows * nrhs) return;
    const int r = (int)(g / nrows);
    const long long i = g % nrows;
    const cpx<T> *xr = x + (long long)r * ldx;
    double re = 0, im = 0;
    for (long long k = ptr[i]; k < ptr[i + 1]; k++) {
        const cpx<T> a = val[k], b = xr[col[k]];
        re += (double)a.re * b.re - (double)a.im * b.im;
        im += (double)a.re * b.im + (double)a.im * b.re;
    }
    cpx<T> &o = y[(long long)r * ldy + i];
    if (accumulate) o = {(T)((double)o.re + alpha * re), (T)((double)o.im + alpha * im)};
    else o = {(T)(alpha * re), (T)(alpha * im)};
}

// b(:, r) = (complex float) a(:, r)  (rows n, leading dimensions lda, ldb)
__global__ __launch_bounds__(KT) void k_to_single(const cpx<double> *__restrict__ a, long long lda,
                                                  cpx<float> *__restrict__ b, long long ldb, long long n, int nrhs)
{
    const long long g = (long long)blockIdx.x * KT + threadIdx.x;
    if (g >= n * nrhs) return;
    const int r = (int)(g / n);
    const long long k = g % n;
    const cpx<double> v = a[(long long)r * lda + k];
    b[(long long)r * ldb + k] = {(float)v.re, (float)v.im};
}

// a(:, r) = b(:, r), or a(:, r) += b(:, r) with add  (complex double from complex float)
__global__ __launch_bounds__(KT) void k_from_single(cpx<double> *__restrict__ a, long long lda,
                                                    const cpx<float> *__restrict__ b, long long ldb, long long n,
                                                    int nrhs, int add)
{
    const long long g = (long long)blockIdx.x * KT + threadIdx.x;
    if (g >= n * nrhs) return;
    const int r = (int)(g / n);
    const long long k = g % n;
    const cpx<float> v = b[(long long)r * ldb + k];
    cpx<double> &o = a[(long long)r * lda + k];
    if (add) o = {o.re + (double)v.re, o.im + (double)v.im};
    else o = {(double)v.re, (double)v.im};
}

inline unsigned blocks(long long n) { return (unsigned)((n + KT - 1) / KT); }

}  // namespace

void launch_to_single(const cpx<double> *a, long long lda, cpx<float> *b, long long ldb, long long n, int nrhs,
                      hipStream_t s)
{
    if (n * nrhs > 0) hipLaunchKernelGGL(k_to_single, dim3(blocks(n * nrhs)), dim3(KT), 0, s, a, lda, b, ldb, n, nrhs);
}

void launch_from_single(cpx<double> *a, long long lda, const cpx<float> *b, long long ldb, long long n, int nrhs,
                        bool add, hipStream_t s)
{
    if (n * nrhs > 0)
        hipLaunchKernelGGL(k_from_single, dim3(blocks(n * nrhs)), dim3(KT), 0, s, a, lda, b, ldb, n, nrhs, add ? 1 : 0);
}

template <class T>
void launch_csr_spmm(long long nrows, int nrhs, const long long *ptr, const int *col, const cpx<T> *val,
                     const cpx<T> *x, long long ldx, cpx<T> *y, long long ldy, double alpha, bool accumulate,
                     hipStream_t s)
{
    if (nrows <= 0) return;
    hipLaunchKernelGGL(k_csr_spmm<T>, dim3(blocks(nrows * nrhs)), dim3(KT), 0, s, nrows, nrhs, ptr, col, val, x, ldx,
                       y, ldy, alpha, accumulate ? 1 : 0);
}

template <class T>
void krylov_dots(const cpx<T> *V, long long vstride, long long ldv, int nv, const cpx<T> *w, long long ldw, long long n,
                 int nrhs, cpx<double> *part, int nchunk, cpx<double> *out, hipStream_t s)
{
    const long long chunk = (n + nchunk - 1) / nchunk;
    hipLaunchKernelGGL(k_dots<T>, dim3(nchunk, nrhs), dim3(KT), 0, s, V, vstride, ldv, nv, w, ldw, n, chunk, part,
                       nchunk, nrhs);
    hipLaunchKernelGGL(k_sum_parts, dim3(blocks((long long)nv * nrhs)), dim3(KT), 0, s, part, nv, nchunk, nrhs, out);
}

template <class T>
void krylov_combine(const cpx<T> *V, long long vstride, long long ldv, int nv, const cpx<double> *h, double sign,
                    cpx<T> *w, long long ldw, long long n, int nrhs, hipStream_t s)
{
    hipLaunchKernelGGL(k_combine<T>, dim3(blocks(n * nrhs)), dim3(KT), 0, s, V, vstride, ldv, nv, h, sign, w, ldw, n,
                       nrhs);
}

template <class T>
void krylov_axpby(const cpx<double> *a, const cpx<T> *x, long long ldx, const cpx<double> *b, const cpx<T> *z,
                  long long ldz, cpx<T> *y, long long ldy, long long n, int nrhs, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpby<T>, dim3(blocks(n * nrhs)), dim3(KT), 0, s, a, x, ldx, b, z, ldz, y, ldy, n, nrhs);
}

#define KRYLOV_INST(T)                                                                                              \
    template void krylov_dots<T>(const cpx<T> *, long long, long long, int, const cpx<T> *, long long, long long,  \
                                 int, cpx<double> *, int, cpx<double> *, hipStream_t);                             \
    template void krylov_combine<T>(const cpx<T> *, long long, long long, int, const cpx<double> *, double,       \
                                    cpx<T> *, long long, long long, int, hipStream_t);                             \
    template void krylov_axpby<T>(const cpx<double> *, const cpx<T> *, long long, const cpx<double> *,           \
                                  const cpx<T> *, long long, cpx<T> *, long long, long long, int, hipStream_t);   \
    template void launch_csr_spmm<T>(long long, int, const long long *, const int *, const cpx<T> *,             \
                                     const cpx<T> *, long long, cpx<T> *, long long, double, bool, hipStream_t);
KRYLOV_INST(float)
KRYLOV_INST(double)

}  // namespace mlfma
