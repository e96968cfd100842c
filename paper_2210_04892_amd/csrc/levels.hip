// Aggregation and disaggregation between octree levels, one kernel per step.
//
// Aggregation (Sec. II-E, MLFMA outgoing patterns): for every parent P,
//   U_P(k) = sum_{c in children(P)} exp(+jk khat.(r_c - r_P)) [I U_c](k),
// with I the separable local Lagrange interpolation: first in theta (child
// theta rows -> parent theta rows, for every child phi column, across the
// poles), then in phi (periodic).  Disaggregation applies the weighted
// transposes (anterpolation) in the opposite order, after the conjugate
// shift, and adds the result to the child's incoming pattern.
//
// Both stencils are local in theta, so a workgroup owns one box and a chunk
// of theta rows: it stages the theta rows of the input pattern that the chunk
// needs in LDS with coalesced loads, forms the intermediate (parent theta x
// child phi) rows in LDS, and writes only its own outputs.  The intermediate
// never goes to memory.
#include "device.hpp"

namespace mlfma {

namespace {

constexpr int NXCD_L = 8;
__device__ inline long long xcd_block_l(long long nblk)
{
    const long long per = (nblk + NXCD_L - 1) / NXCD_L;
    const long long hw = blockIdx.x;
    const long long lb = (hw % NXCD_L) * per + hw / NXCD_L;
    return lb < nblk ? lb : -1;
}
inline unsigned xcd_grid_l(long long nblk) { return (unsigned)(((nblk + NXCD_L - 1) / NXCD_L) * NXCD_L); }

__device__ inline long long pat(long long b, int c, int r, int q, int nrhs, int K)
{
    return ((b * 2 + c) * nrhs + r) * (long long)K + q;
}

constexpr int STEP_THREADS = 256;
constexpr int STEP_OUT = 4;     // outputs per thread: a chunk has at most 4 * 256 of them

// aggregation: workgroup = (parent, chunk of parent theta rows), one rhs
template <class T, int P>
__global__ __launch_bounds__(STEP_THREADS) void k_aggregate(const LevelStep<T> a, int nrhs)
{
    extern __shared__ double step_lds_raw[];
    const long long blk = xcd_block_l((long long)a.nbox * a.nchunk);
    if (blk < 0) return;
    const int Pb = (int)(blk / a.nchunk), ch = (int)(blk % a.nchunk);
    const int r = blockIdx.y;
    const int Kc = a.nth_c * a.nph_c, Kp = a.nth_p * a.nph_p;
    const int i0 = ch * a.rows, i1 = min(a.nth_p, i0 + a.rows);
    const int w0 = a.win[2 * ch], w1 = a.win[2 * ch + 1];
    const int wlen = (w1 - w0) * a.nph_c, wmax = a.wrows * a.nph_c;
    const int mlen = (i1 - i0) * a.nph_c, mmax = a.rows * a.nph_c;
    const int olen = (i1 - i0) * a.nph_p;
    cpx<T> *cw = reinterpret_cast<cpx<T> *>(step_lds_raw);   // [2][wmax] child window
    cpx<T> *mid = cw + 2 * wmax;                              // [2][mmax] intermediate
    cpx<T> acc0[STEP_OUT], acc1[STEP_OUT];
#pragma unroll
    for (int k = 0; k < STEP_OUT; k++) acc0[k] = acc1[k] = mk<T>(0, 0);
    const int cb = a.child_start[Pb], ce = a.child_start[Pb + 1];
    for (int c = cb; c < ce; c++) {
        const cpx<T> *u0 = a.in + pat(c, 0, r, w0 * a.nph_c, nrhs, Kc);
        const cpx<T> *u1 = a.in + pat(c, 1, r, w0 * a.nph_c, nrhs, Kc);
        for (int i = threadIdx.x; i < wlen; i += STEP_THREADS) {
            cw[i] = u0[i];
            cw[wmax + i] = u1[i];
        }
        __syncthreads();
        // theta: mid row (parent theta i, child phi j) from the child window
        for (int m = threadIdx.x; m < mlen; m += STEP_THREADS) {
            const long long row = (long long)i0 * a.nph_c + m;
            int cc[P];
            T ww[P];
#pragma unroll
            for (int t = 0; t < P; t++) {
                cc[t] = a.c1[row * P + t] - w0 * a.nph_c;
                ww[t] = a.w1[row * P + t];
            }
            cpx<T> s0 = mk<T>(0, 0), s1 = mk<T>(0, 0);
#pragma unroll
            for (int t = 0; t < P; t++) {
                axpy_to(s0, ww[t], cw[cc[t]]);
                axpy_to(s1, ww[t], cw[wmax + cc[t]]);
            }
            mid[m] = s0;
            mid[mmax + m] = s1;
        }
        __syncthreads();
        // phi, then the shift to the parent centre
        const cpx<T> *sh = a.shift + (long long)a.oct[c] * Kp;
#pragma unroll
        for (int k = 0; k < STEP_OUT; k++) {
            const int o = threadIdx.x + k * STEP_THREADS;
            if (o < olen) {
                const long long q = (long long)i0 * a.nph_p + o;
                cpx<T> s0 = mk<T>(0, 0), s1 = mk<T>(0, 0);
#pragma unroll
                for (int t = 0; t < P; t++) {
                    const int j = a.c2[q * P + t] - i0 * a.nph_c;
                    const T wt = a.w2[q * P + t];
                    axpy_to(s0, wt, mid[j]);
                    axpy_to(s1, wt, mid[mmax + j]);
                }
                const cpx<T> f = sh[q];
                fma_to(acc0[k], f, s0);
                fma_to(acc1[k], f, s1);
            }
        }
        __syncthreads();   // the next child reuses the window and the intermediate
    }
#pragma unroll
    for (int k = 0; k < STEP_OUT; k++) {
        const int o = threadIdx.x + k * STEP_THREADS;
        if (o < olen) {
            const int q = i0 * a.nph_p + o;
            a.out[pat(Pb, 0, r, q, nrhs, Kp)] = acc0[k];
            a.out[pat(Pb, 1, r, q, nrhs, Kp)] = acc1[k];
        }
    }
}

// disaggregation: workgroup = (child, chunk of child theta rows), one rhs;
// out (the child's incoming pattern) += anterpolated, shifted parent pattern
template <class T>
__global__ __launch_bounds__(STEP_THREADS) void k_disaggregate(const LevelStep<T> a, int nrhs)
{
    extern __shared__ double step_lds_raw[];
    const long long blk = xcd_block_l((long long)a.nbox * a.nchunk);
    if (blk < 0) return;
    const int c = (int)(blk / a.nchunk), ch = (int)(blk % a.nchunk);
    const int r = blockIdx.y;
    const int Kc = a.nth_c * a.nph_c, Kp = a.nth_p * a.nph_p;
    const int i0 = ch * a.rows, i1 = min(a.nth_c, i0 + a.rows);
    const int w0 = a.win[2 * ch], w1 = a.win[2 * ch + 1];
    const int plen = (w1 - w0) * a.nph_p, pmax = a.wrows * a.nph_p;
    const int mlen = (w1 - w0) * a.nph_c, mmax = a.wrows * a.nph_c;
    const int olen = (i1 - i0) * a.nph_c;
    cpx<T> *pw = reinterpret_cast<cpx<T> *>(step_lds_raw);   // [2][pmax] shifted parent rows
    cpx<T> *mid = pw + 2 * pmax;                              // [2][mmax] intermediate rows
    const int Pb = a.parent[c];
    const cpx<T> *sh = a.shift + (long long)a.oct[c] * Kp + (long long)w0 * a.nph_p;
    const cpx<T> *v0 = a.in + pat(Pb, 0, r, w0 * a.nph_p, nrhs, Kp);
    const cpx<T> *v1 = a.in + pat(Pb, 1, r, w0 * a.nph_p, nrhs, Kp);
    for (int i = threadIdx.x; i < plen; i += STEP_THREADS) {
        const cpx<T> f = conjg(sh[i]);
        pw[i] = f * v0[i];
        pw[pmax + i] = f * v1[i];
    }
    __syncthreads();
    // phi anterpolation: intermediate rows from the parent rows of the window
    for (int m = threadIdx.x; m < mlen; m += STEP_THREADS) {
        const int il = m / a.nph_c, j = m % a.nph_c;
        const int *pc = a.phi_col + j * a.tphi;
        const T *pwt = a.phi_w + j * a.tphi;
        const cpx<T> *p0 = pw + il * a.nph_p, *p1 = pw + pmax + il * a.nph_p;
        cpx<T> s0 = mk<T>(0, 0), s1 = mk<T>(0, 0);
#pragma unroll 4
        for (int t = 0; t < a.tphi; t++) {
            const int jj = pc[t];
            axpy_to(s0, pwt[t], p0[jj]);
            axpy_to(s1, pwt[t], p1[jj]);
        }
        const T f = a.rowf[w0 + il];
        mid[m] = f * s0;
        mid[mmax + m] = f * s1;
    }
    __syncthreads();
    // theta anterpolation into the child's own rows
    for (int o = threadIdx.x; o < olen; o += STEP_THREADS) {
        const int ic = i0 + o / a.nph_c, j = o % a.nph_c;
        const int *tr = a.th_row + ic * a.tth, *ts = a.th_sh + ic * a.tth;
        const T *tw = a.th_w + ic * a.tth;
        cpx<T> s0 = mk<T>(0, 0), s1 = mk<T>(0, 0);
#pragma unroll 4
        for (int t = 0; t < a.tth; t++) {
            int col = j + ts[t];
            col = col >= a.nph_c ? col - a.nph_c : col;
            const int jj = (tr[t] - w0) * a.nph_c + col;
            axpy_to(s0, tw[t], mid[jj]);
            axpy_to(s1, tw[t], mid[mmax + jj]);
        }
        const long long q = (long long)ic * a.nph_c + j;
        cpx<T> &y0 = a.out[pat(c, 0, r, (int)q, nrhs, Kc)];
        cpx<T> &y1 = a.out[pat(c, 1, r, (int)q, nrhs, Kc)];
        y0 = y0 + s0;
        y1 = y1 + s1;
    }
}

}  // namespace

template <class T>
bool launch_aggregate_step(const LevelStep<T> &a, int nrhs, hipStream_t s)
{
    if (a.nchunk <= 0 || (long long)a.rows * a.nph_p > STEP_OUT * STEP_THREADS) return false;
    const size_t lds = agg_lds_bytes<T>(a.wrows, a.rows, a.nph_c);
    if (lds > STEP_LDS_MAX) return false;
    if (a.nbox <= 0 || nrhs <= 0) return true;
    const dim3 grid(xcd_grid_l((long long)a.nbox * a.nchunk), nrhs);
    switch (a.taps) {
    case 6: hipLaunchKernelGGL((k_aggregate<T, 6>), grid, dim3(STEP_THREADS), lds, s, a, nrhs); return true;
    case 8: hipLaunchKernelGGL((k_aggregate<T, 8>), grid, dim3(STEP_THREADS), lds, s, a, nrhs); return true;
    case 10: hipLaunchKernelGGL((k_aggregate<T, 10>), grid, dim3(STEP_THREADS), lds, s, a, nrhs); return true;
    default: return false;
    }
}

template <class T>
bool launch_disaggregate_step(const LevelStep<T> &a, int nrhs, hipStream_t s)
{
    if (a.nchunk <= 0 || a.tphi <= 0 || a.tth <= 0) return false;
    const size_t lds = dis_lds_bytes<T>(a.wrows, a.nph_p, a.nph_c);
    if (lds > STEP_LDS_MAX) return false;
    if (a.nbox <= 0 || nrhs <= 0) return true;
    const dim3 grid(xcd_grid_l((long long)a.nbox * a.nchunk), nrhs);
    hipLaunchKernelGGL(k_disaggregate<T>, grid, dim3(STEP_THREADS), lds, s, a, nrhs);
    return true;
}

template bool launch_aggregate_step<float>(const LevelStep<float> &, int, hipStream_t);
template bool launch_aggregate_step<double>(const LevelStep<double> &, int, hipStream_t);
template bool launch_disaggregate_step<float>(const LevelStep<float> &, int, hipStream_t);
template bool launch_disaggregate_step<double>(const LevelStep<double> &, int, hipStream_t);

}  // namespace mlfma
