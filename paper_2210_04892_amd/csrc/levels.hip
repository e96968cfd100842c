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
#include <algorithm>

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

// aggregation: workgroup = (parent, chunk of parent theta rows, one right-
// hand side); the parent's children are taken in groups of G: the group's
// windows are staged together, their intermediates formed together, then the
// phi stencil and the shift accumulate over the group (three barriers per
// group instead of per child)
template <class T, int P, bool GROUPED, int OUT>
__global__ __launch_bounds__(STEP_THREADS) void k_aggregate(const LevelStep<T> a, int nrhs, int Gr)
{
    const int G = GROUPED ? Gr : 1;
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
    cpx<T> *cw = reinterpret_cast<cpx<T> *>(step_lds_raw);   // [G][2][wmax] child windows
    cpx<T> *mid = cw + 2 * (size_t)G * wmax;                  // [G][2][mmax] intermediates
    cpx<T> acc0[OUT], acc1[OUT];
#pragma unroll
    for (int k = 0; k < OUT; k++) acc0[k] = acc1[k] = mk<T>(0, 0);
    const int cb = a.child_start[Pb], ce = a.child_start[Pb + 1];
    for (int cg = cb; cg < ce; cg += G) {
        const int ng = GROUPED ? min(G, ce - cg) : 1;
        for (int g = 0; g < ng; g++) {
            const cpx<T> *u0 = a.in + pat(cg + g, 0, r, w0 * a.nph_c, nrhs, Kc);
            const cpx<T> *u1 = u0 + (long long)nrhs * Kc;
            for (int i = threadIdx.x; i < wlen; i += STEP_THREADS) {
                cw[(2 * g) * wmax + i] = u0[i];
                cw[(2 * g + 1) * wmax + i] = u1[i];
            }
        }
        __syncthreads();
        // theta: mid row (parent theta i, child phi j) of every child of the group
        for (int m = threadIdx.x; m < mlen; m += STEP_THREADS) {
            const long long row = (long long)i0 * a.nph_c + m;
            int cc[P];
            T ww[P];
#pragma unroll
            for (int t = 0; t < P; t++) {
                cc[t] = a.c1[row * P + t] - w0 * a.nph_c;
                ww[t] = a.w1[row * P + t];
            }
            for (int g = 0; g < ng; g++) {
                const cpx<T> *c0 = cw + (2 * g) * wmax, *c1 = cw + (2 * g + 1) * wmax;
                cpx<T> s0 = mk<T>(0, 0), s1 = mk<T>(0, 0);
#pragma unroll
                for (int t = 0; t < P; t++) {
                    axpy_to(s0, ww[t], c0[cc[t]]);
                    axpy_to(s1, ww[t], c1[cc[t]]);
                }
                mid[(2 * g) * mmax + m] = s0;
                mid[(2 * g + 1) * mmax + m] = s1;
            }
        }
        __syncthreads();
        // phi and the shift to the parent centre, summed over the group
#pragma unroll
        for (int k = 0; k < OUT; k++) {
            const int o = threadIdx.x + k * STEP_THREADS;
            if (o >= olen) continue;
            const long long q = (long long)i0 * a.nph_p + o;
            int cc[P];
            T ww[P];
#pragma unroll
            for (int t = 0; t < P; t++) {
                cc[t] = a.c2[q * P + t] - i0 * a.nph_c;
                ww[t] = a.w2[q * P + t];
            }
            for (int g = 0; g < ng; g++) {
                const cpx<T> *m0 = mid + (2 * g) * mmax, *m1 = mid + (2 * g + 1) * mmax;
                cpx<T> s0 = mk<T>(0, 0), s1 = mk<T>(0, 0);
#pragma unroll
                for (int t = 0; t < P; t++) {
                    axpy_to(s0, ww[t], m0[cc[t]]);
                    axpy_to(s1, ww[t], m1[cc[t]]);
                }
                const cpx<T> f = a.shift[(long long)a.oct[cg + g] * Kp + q];
                fma_to(acc0[k], f, s0);
                fma_to(acc1[k], f, s1);
            }
        }
        __syncthreads();   // the next group reuses the windows and the intermediates
    }
#pragma unroll
    for (int k = 0; k < OUT; k++) {
        const int o = threadIdx.x + k * STEP_THREADS;
        if (o >= olen) continue;
        const int q = i0 * a.nph_p + o;
        a.out[pat(Pb, 0, r, q, nrhs, Kp)] = acc0[k];
        a.out[pat(Pb, 1, r, q, nrhs, Kp)] = acc1[k];
    }
}

// disaggregation: workgroup = (child, chunk of child theta rows, RB
// right-hand sides); out (the child's incoming pattern) += anterpolated,
// shifted parent pattern
template <class T, int RB>
__global__ __launch_bounds__(STEP_THREADS) void k_disaggregate(const LevelStep<T> a, int nrhs)
{
    extern __shared__ double step_lds_raw[];
    const long long blk = xcd_block_l((long long)a.nbox * a.nchunk);
    if (blk < 0) return;
    const int c = (int)(blk / a.nchunk), ch = (int)(blk % a.nchunk);
    const int r0 = blockIdx.y * RB;
    const int Kc = a.nth_c * a.nph_c, Kp = a.nth_p * a.nph_p;
    const int i0 = ch * a.rows, i1 = min(a.nth_c, i0 + a.rows);
    const int w0 = a.win[2 * ch], w1 = a.win[2 * ch + 1];
    const int plen = (w1 - w0) * a.nph_p, pmax = a.wrows * a.nph_p;
    const int mlen = (w1 - w0) * a.nph_c, mmax = a.wrows * a.nph_c;
    const int olen = (i1 - i0) * a.nph_c;
    cpx<T> *pw = reinterpret_cast<cpx<T> *>(step_lds_raw);   // [RB][2][pmax] shifted parent rows
    cpx<T> *mid = pw + 2 * RB * pmax;                         // [RB][2][mmax] intermediate rows
    const int Pb = a.parent[c];
    const cpx<T> *sh = a.shift + (long long)a.oct[c] * Kp + (long long)w0 * a.nph_p;
    for (int i = threadIdx.x; i < plen; i += STEP_THREADS) {
        const cpx<T> f = conjg(sh[i]);
#pragma unroll
        for (int j = 0; j < RB; j++) {
            const int r = min(r0 + j, nrhs - 1);
            pw[(2 * j) * pmax + i] = f * a.in[pat(Pb, 0, r, w0 * a.nph_p + i, nrhs, Kp)];
            pw[(2 * j + 1) * pmax + i] = f * a.in[pat(Pb, 1, r, w0 * a.nph_p + i, nrhs, Kp)];
        }
    }
    __syncthreads();
    // phi anterpolation: intermediate rows from the parent rows of the window
    for (int m = threadIdx.x; m < mlen; m += STEP_THREADS) {
        const int il = m / a.nph_c, jc = m % a.nph_c;
        const int *pc = a.phi_col + jc * a.tphi;
        const T *pwt = a.phi_w + jc * a.tphi;
        cpx<T> s0[RB], s1[RB];
#pragma unroll
        for (int j = 0; j < RB; j++) s0[j] = s1[j] = mk<T>(0, 0);
#pragma unroll 4
        for (int t = 0; t < a.tphi; t++) {
            const int jj = il * a.nph_p + pc[t];
            const T wt = pwt[t];
#pragma unroll
            for (int j = 0; j < RB; j++) {
                axpy_to(s0[j], wt, pw[(2 * j) * pmax + jj]);
                axpy_to(s1[j], wt, pw[(2 * j + 1) * pmax + jj]);
            }
        }
        const T f = a.rowf[w0 + il];
#pragma unroll
        for (int j = 0; j < RB; j++) {
            mid[(2 * j) * mmax + m] = f * s0[j];
            mid[(2 * j + 1) * mmax + m] = f * s1[j];
        }
    }
    __syncthreads();
    // theta anterpolation into the child's own rows
    for (int o = threadIdx.x; o < olen; o += STEP_THREADS) {
        const int ic = i0 + o / a.nph_c, jc = o % a.nph_c;
        const int *tr = a.th_row + ic * a.tth, *ts = a.th_sh + ic * a.tth;
        const T *tw = a.th_w + ic * a.tth;
        cpx<T> s0[RB], s1[RB];
#pragma unroll
        for (int j = 0; j < RB; j++) s0[j] = s1[j] = mk<T>(0, 0);
#pragma unroll 4
        for (int t = 0; t < a.tth; t++) {
            int col = jc + ts[t];
            col = col >= a.nph_c ? col - a.nph_c : col;
            const int jj = (tr[t] - w0) * a.nph_c + col;
            const T wt = tw[t];
#pragma unroll
            for (int j = 0; j < RB; j++) {
                axpy_to(s0[j], wt, mid[(2 * j) * mmax + jj]);
                axpy_to(s1[j], wt, mid[(2 * j + 1) * mmax + jj]);
            }
        }
        const int q = ic * a.nph_c + jc;
#pragma unroll
        for (int j = 0; j < RB; j++) {
            if (r0 + j >= nrhs) continue;
            cpx<T> &y0 = a.out[pat(c, 0, r0 + j, q, nrhs, Kc)];
            cpx<T> &y1 = a.out[pat(c, 1, r0 + j, q, nrhs, Kc)];
            y0 = y0 + s0[j];
            y1 = y1 + s1[j];
        }
    }
}

// right-hand sides per workgroup: two where the LDS allows (four would hold
// more LDS per workgroup than the sharing of the parent rows saves)
inline int step_rb(size_t lds1, int nrhs)
{
    int rb = 1;
    while (rb < 2 && rb < nrhs && 2 * rb * lds1 <= STEP_LDS_MAX) rb *= 2;
    return rb;
}

}  // namespace

// outputs per thread: two where the chunk has at most 512 of them (fewer
// registers), else four
template <class T, int P>
void agg_launch(int G, dim3 grid, dim3 block, size_t lds, hipStream_t s, const LevelStep<T> &a, int nrhs)
{
    const bool two = (long long)a.rows * a.nph_p <= 2 * STEP_THREADS;
    if (G > 1 && two) hipLaunchKernelGGL((k_aggregate<T, P, true, 2>), grid, block, lds, s, a, nrhs, G);
    else if (G > 1) hipLaunchKernelGGL((k_aggregate<T, P, true, STEP_OUT>), grid, block, lds, s, a, nrhs, G);
    else if (two) hipLaunchKernelGGL((k_aggregate<T, P, false, 2>), grid, block, lds, s, a, nrhs, 1);
    else hipLaunchKernelGGL((k_aggregate<T, P, false, STEP_OUT>), grid, block, lds, s, a, nrhs, 1);
}

template <class T>
bool launch_aggregate_step(const LevelStep<T> &a, int nrhs, hipStream_t s)
{
    if (a.nchunk <= 0 || (long long)a.rows * a.nph_p > STEP_OUT * STEP_THREADS) return false;
    if (a.taps != 6 && a.taps != 8 && a.taps != 10) return false;
    const size_t lds1 = agg_lds_bytes<T>(a.wrows, a.rows, a.nph_c);   // one child
    if (lds1 > STEP_LDS_MAX) return false;
    if (a.nbox <= 0 || nrhs <= 0) return true;
    // children per group: with few right-hand sides the grid is small and
    // the per-child barriers dominate, so several children are grouped (four
    // in single, two in double precision: a parent on a surface has about
    // four, and larger groups hold LDS that costs occupancy); with more
    // right-hand sides, one child at a time keeps the LDS per workgroup low
    const int gmax = sizeof(T) == 4 ? 4 : 2;
    const int G = nrhs < 4 ? (int)std::min<size_t>(gmax, STEP_LDS_MAX / lds1) : 1;
    const dim3 grid(xcd_grid_l((long long)a.nbox * a.nchunk), nrhs), block(STEP_THREADS);
    const size_t lds = G * lds1;
    if (a.taps == 6) agg_launch<T, 6>(G, grid, block, lds, s, a, nrhs);
    else if (a.taps == 8) agg_launch<T, 8>(G, grid, block, lds, s, a, nrhs);
    else agg_launch<T, 10>(G, grid, block, lds, s, a, nrhs);
    return true;
}

template <class T>
bool launch_disaggregate_step(const LevelStep<T> &a, int nrhs, hipStream_t s)
{
    if (a.nchunk <= 0 || a.tphi <= 0 || a.tth <= 0) return false;
    const size_t lds1 = dis_lds_bytes<T>(a.wrows, a.nph_p, a.nph_c);
    if (lds1 > STEP_LDS_MAX) return false;
    if (a.nbox <= 0 || nrhs <= 0) return true;
    const int rb = step_rb(lds1, nrhs);
    const dim3 grid(xcd_grid_l((long long)a.nbox * a.nchunk), (nrhs + rb - 1) / rb), block(STEP_THREADS);
    const size_t lds = rb * lds1;
    if (rb == 2) hipLaunchKernelGGL((k_disaggregate<T, 2>), grid, block, lds, s, a, nrhs);
    else hipLaunchKernelGGL((k_disaggregate<T, 1>), grid, block, lds, s, a, nrhs);
    return true;
}

template bool launch_aggregate_step<float>(const LevelStep<float> &, int, hipStream_t);
template bool launch_aggregate_step<double>(const LevelStep<double> &, int, hipStream_t);
template bool launch_disaggregate_step<float>(const LevelStep<float> &, int, hipStream_t);
template bool launch_disaggregate_step<double>(const LevelStep<double> &, int, hipStream_t);

}  // namespace mlfma
