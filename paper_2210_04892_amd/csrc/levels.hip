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
// never goes to memory.  Two forms of each step: blocked (a workgroup per
// chunk and block of right-hand sides) and pipelined (a workgroup walks
// several passes with the next pass's loads in flight); the autotuner picks
// per level.
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

// aggregation: workgroup = (parent, chunk of parent theta rows, RB right-
// hand sides); the parent's children are taken in groups of G: the group's
// windows are staged together, their intermediates formed together, then the
// phi stencil and the shift accumulate over the group (three barriers per
// group instead of per child).  A thread keeps OUT outputs of every one of
// the RB right-hand sides, so the stencil indices, weights and shifts it
// loads serve all of them.
template <class T, int P, bool GROUPED, int OUT, int RB>
__global__ __launch_bounds__(STEP_THREADS) void k_aggregate(const LevelStep<T> a, int nrhs, int Gr)
{
    const int G = GROUPED ? Gr : 1;
    extern __shared__ double step_lds_raw[];
    const long long blk = xcd_block_l((long long)a.nbox * a.nchunk);
    if (blk < 0) return;
    const int Pb = (int)(blk / a.nchunk), ch = (int)(blk % a.nchunk);
    const int r0 = blockIdx.y * RB;
    const int Kc = a.nth_c * a.nph_c, Kp = a.nth_p * a.nph_p;
    const int i0 = ch * a.rows, i1 = min(a.nth_p, i0 + a.rows);
    const int w0 = a.win[2 * ch], w1 = a.win[2 * ch + 1];
    const int wlen = (w1 - w0) * a.nph_c, wmax = a.wrows * a.nph_c;
    const int mlen = (i1 - i0) * a.nph_c, mmax = a.rows * a.nph_c;
    const int olen = (i1 - i0) * a.nph_p;
    cpx<T> *cw = reinterpret_cast<cpx<T> *>(step_lds_raw);   // [G][RB][2][wmax] child windows
    cpx<T> *mid = cw + 2 * (size_t)G * RB * wmax;             // [G][RB][2][mmax] intermediates
    cpx<T> acc0[OUT][RB], acc1[OUT][RB];
#pragma unroll
    for (int k = 0; k < OUT; k++)
#pragma unroll
        for (int j = 0; j < RB; j++) acc0[k][j] = acc1[k][j] = mk<T>(0, 0);
    const int cb = a.child_start[Pb], ce = a.child_start[Pb + 1];
    for (int cg = cb; cg < ce; cg += G) {
        const int ng = GROUPED ? min(G, ce - cg) : 1;
        // stage the group's windows: each thread loads up to SW samples of
        // every right-hand side and component (clamped addresses, all loads
        // in flight together) before it writes any of them to LDS
        for (int g = 0; g < ng; g++) {
            const cpx<T> *ub = a.in + pat(cg + g, 0, 0, w0 * a.nph_c, nrhs, Kc);
            if (wlen <= STEP_THREADS) {   // one slot per thread
                const int i = min((int)threadIdx.x, max(wlen - 1, 0));
                cpx<T> v0[RB], v1[RB];
#pragma unroll
                for (int j = 0; j < RB; j++) {
                    const cpx<T> *u0 = ub + (long long)min(r0 + j, nrhs - 1) * Kc;
                    v0[j] = u0[i];
                    v1[j] = u0[(long long)nrhs * Kc + i];
                }
#pragma unroll
                for (int j = 0; j < RB; j++) {
                    cpx<T> *d = cw + (size_t)(2 * (g * RB + j)) * wmax;
                    d[i] = v0[j];
                    d[wmax + i] = v1[j];
                }
                continue;
            }
            constexpr int SW = 2;
            for (int ib = threadIdx.x; ib < wlen; ib += SW * STEP_THREADS) {
                cpx<T> v0[SW][RB], v1[SW][RB];
#pragma unroll
                for (int k = 0; k < SW; k++) {
                    const int i = min(ib + k * STEP_THREADS, wlen - 1);
#pragma unroll
                    for (int j = 0; j < RB; j++) {
                        const cpx<T> *u0 = ub + (long long)min(r0 + j, nrhs - 1) * Kc;
                        v0[k][j] = u0[i];
                        v1[k][j] = u0[(long long)nrhs * Kc + i];
                    }
                }
                // slots past the window write the last sample's value to its
                // own slot again (the same value: no predicate, so the loads
                // are not moved below a branch)
#pragma unroll
                for (int k = 0; k < SW; k++) {
                    const int i = min(ib + k * STEP_THREADS, wlen - 1);
#pragma unroll
                    for (int j = 0; j < RB; j++) {
                        cpx<T> *d = cw + (size_t)(2 * (g * RB + j)) * wmax;
                        d[i] = v0[k][j];
                        d[wmax + i] = v1[k][j];
                    }
                }
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
#pragma unroll
                for (int j = 0; j < RB; j++) {
                    const cpx<T> *c0 = cw + (size_t)(2 * (g * RB + j)) * wmax, *c1 = c0 + wmax;
                    cpx<T> s0 = mk<T>(0, 0), s1 = mk<T>(0, 0);
#pragma unroll
                    for (int t = 0; t < P; t++) {
                        axpy_to(s0, ww[t], c0[cc[t]]);
                        axpy_to(s1, ww[t], c1[cc[t]]);
                    }
                    cpx<T> *d = mid + (size_t)(2 * (g * RB + j)) * mmax;
                    d[m] = s0;
                    d[mmax + m] = s1;
                }
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
                const cpx<T> f = a.shift[(long long)a.oct[cg + g] * Kp + q];
#pragma unroll
                for (int j = 0; j < RB; j++) {
                    const cpx<T> *m0 = mid + (size_t)(2 * (g * RB + j)) * mmax, *m1 = m0 + mmax;
                    cpx<T> s0 = mk<T>(0, 0), s1 = mk<T>(0, 0);
#pragma unroll
                    for (int t = 0; t < P; t++) {
                        axpy_to(s0, ww[t], m0[cc[t]]);
                        axpy_to(s1, ww[t], m1[cc[t]]);
                    }
                    fma_to(acc0[k][j], f, s0);
                    fma_to(acc1[k][j], f, s1);
                }
            }
        }
        __syncthreads();   // the next group reuses the windows and the intermediates
    }
#pragma unroll
    for (int k = 0; k < OUT; k++) {
        const int o = threadIdx.x + k * STEP_THREADS;
        if (o >= olen) continue;
        const int q = i0 * a.nph_p + o;
#pragma unroll
        for (int j = 0; j < RB; j++) {
            if (r0 + j >= nrhs) continue;
            a.out[pat(Pb, 0, r0 + j, q, nrhs, Kp)] = acc0[k][j];
            a.out[pat(Pb, 1, r0 + j, q, nrhs, Kp)] = acc1[k][j];
        }
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

// disaggregation, pipelined over the vectors: a box's patterns are 2 nrhs
// vectors of K samples (component c, right-hand side r at c nrhs + r), all
// transformed by the same stencils.  Workgroup = (child, chunk of child theta
// rows, slice of the vectors).  It walks its slice NV vectors at a time (one
// vector: half the LDS of a right-hand side's two components, for the wide
// windows of the coarse levels); while one pass anterpolates in LDS, the
// next pass's parent window (NPF samples per thread) and this pass's old
// child values (NO per thread) are in flight in registers, so the memory
// latency of one pass hides behind the arithmetic of another.  The chunk's
// stencils are staged in LDS once.  Same arithmetic as k_disaggregate, term
// for term.
template <class T, int NV, int NPF, int NO>
__global__ __launch_bounds__(STEP_THREADS) void k_disaggregate_pipe(const LevelStep<T> a, int nrhs, int per_slice)
{
    extern __shared__ double step_lds_raw[];
    const long long blk = xcd_block_l((long long)a.nbox * a.nchunk);
    if (blk < 0) return;
    const int c = (int)(blk / a.nchunk), ch = (int)(blk % a.nchunk);
    const int nvec = 2 * nrhs;
    const int vs0 = blockIdx.y * per_slice, vs1 = min(nvec, vs0 + per_slice);
    if (vs0 >= vs1) return;
    const int tid = threadIdx.x;
    const int Kc = a.nth_c * a.nph_c, Kp = a.nth_p * a.nph_p;
    const int nph_c = a.nph_c, nph_p = a.nph_p, tphi = a.tphi, tth = a.tth;
    const int i0 = ch * a.rows, i1 = min(a.nth_c, i0 + a.rows);
    const int w0 = a.win[2 * ch], w1 = a.win[2 * ch + 1];
    const int plen = (w1 - w0) * nph_p, pmax = a.wrows * nph_p;
    const int mlen = (w1 - w0) * nph_c, mmax = a.wrows * nph_c;
    const int olen = (i1 - i0) * nph_c;
    cpx<T> *pw = reinterpret_cast<cpx<T> *>(step_lds_raw);   // [NV][pmax] shifted parent rows
    cpx<T> *mid = pw + NV * pmax;                             // [NV][mmax] intermediate rows
    T *s_phw = reinterpret_cast<T *>(mid + NV * mmax);        // [nph_c][tphi]
    T *s_rowf = s_phw + nph_c * tphi;                         // [wrows]
    T *s_thw = s_rowf + a.wrows;                              // [rows][tth]
    int *s_phc = reinterpret_cast<int *>(s_thw + a.rows * tth);   // [nph_c][tphi]
    int *s_thr = s_phc + nph_c * tphi;                        // [rows][tth]: window row * nph_c
    int *s_ths = s_thr + a.rows * tth;                        // [rows][tth]: phi shift
    for (int i = tid; i < nph_c * tphi; i += STEP_THREADS) {
        s_phc[i] = a.phi_col[i];
        s_phw[i] = a.phi_w[i];
    }
    for (int i = tid; i < w1 - w0; i += STEP_THREADS) s_rowf[i] = a.rowf[w0 + i];
    for (int i = tid; i < (i1 - i0) * tth; i += STEP_THREADS) {
        const int g = i0 * tth + i;
        s_thr[i] = (a.th_row[g] - w0) * nph_c;
        s_ths[i] = a.th_sh[g];
        s_thw[i] = a.th_w[g];
    }
    const int Pb = a.parent[c];
    const cpx<T> *pin = a.in + (long long)Pb * nvec * Kp + (long long)w0 * nph_p;
    cpx<T> *pout = a.out + (long long)c * nvec * Kc + (long long)i0 * nph_c;
    const cpx<T> *sh = a.shift + (long long)a.oct[c] * Kp + (long long)w0 * nph_p;
    cpx<T> shf[NPF];
#pragma unroll
    for (int k = 0; k < NPF; k++) {
        const int i = tid + k * STEP_THREADS;
        shf[k] = i < plen ? conjg(sh[i]) : mk<T>(0, 0);
    }
    // the window and old-value loads take clamped (valid) addresses and no
    // predicate: slots past the window or the output are never written, and
    // a load whose value is not selected right away stays in flight
    cpx<T> pf[NPF][NV];
    auto load_window = [&](int v0) {
#pragma unroll
        for (int k = 0; k < NPF; k++) {
            const int i = min(tid + k * STEP_THREADS, max(plen - 1, 0));
#pragma unroll
            for (int j = 0; j < NV; j++) pf[k][j] = pin[(long long)min(v0 + j, nvec - 1) * Kp + i];
        }
    };
    load_window(vs0);
    // (row, column) of this thread's first intermediate and output slots; a
    // stride of STEP_THREADS advances them by (dq, dr)
    const int dq = STEP_THREADS / nph_c, dr = STEP_THREADS - dq * nph_c;
    const int il0 = tid / nph_c, jc0 = tid - il0 * nph_c;
    for (int v0 = vs0; v0 < vs1; v0 += NV) {
        // the previous pass's phi stage is done (second barrier): overwrite pw
#pragma unroll
        for (int k = 0; k < NPF; k++) {
            const int i = tid + k * STEP_THREADS;
            if (i < plen) {
#pragma unroll
                for (int j = 0; j < NV; j++) pw[j * pmax + i] = shf[k] * pf[k][j];
            }
        }
        load_window(min(v0 + NV, vs1 - 1));   // past the last pass: repeats a valid window
        cpx<T> old[NO][NV];
#pragma unroll
        for (int q = 0; q < NO; q++) {
            const int o = min(tid + q * STEP_THREADS, max(olen - 1, 0));
#pragma unroll
            for (int j = 0; j < NV; j++) old[q][j] = pout[(long long)min(v0 + j, vs1 - 1) * Kc + o];
        }
        __syncthreads();
        // phi anterpolation: intermediate rows from the parent rows of the window
        {
            int il = il0, jc = jc0;
            for (int m = tid; m < mlen; m += STEP_THREADS) {
                const int *pc = s_phc + jc * tphi;
                const T *pwt = s_phw + jc * tphi;
                const int rb_ = il * nph_p;
                cpx<T> sv[NV];
#pragma unroll
                for (int j = 0; j < NV; j++) sv[j] = mk<T>(0, 0);
#pragma unroll 4
                for (int t = 0; t < tphi; t++) {
                    const int jj = rb_ + pc[t];
                    const T wt = pwt[t];
#pragma unroll
                    for (int j = 0; j < NV; j++) axpy_to(sv[j], wt, pw[j * pmax + jj]);
                }
                const T f = s_rowf[il];
#pragma unroll
                for (int j = 0; j < NV; j++) mid[j * mmax + m] = f * sv[j];
                il += dq;
                jc += dr;
                if (jc >= nph_c) {
                    jc -= nph_c;
                    il++;
                }
            }
        }
        __syncthreads();
        // theta anterpolation into the child's own rows
        {
            int il = il0, jc = jc0;
#pragma unroll
            for (int q = 0; q < NO; q++) {
                const int o = tid + q * STEP_THREADS;
                if (o < olen) {
                    const int *tr = s_thr + il * tth, *ts = s_ths + il * tth;
                    const T *tw = s_thw + il * tth;
                    cpx<T> sv[NV];
#pragma unroll
                    for (int j = 0; j < NV; j++) sv[j] = mk<T>(0, 0);
#pragma unroll 4
                    for (int t = 0; t < tth; t++) {
                        int col = jc + ts[t];
                        col = col >= nph_c ? col - nph_c : col;
                        const int jj = tr[t] + col;
                        const T wt = tw[t];
#pragma unroll
                        for (int j = 0; j < NV; j++) axpy_to(sv[j], wt, mid[j * mmax + jj]);
                    }
#pragma unroll
                    for (int j = 0; j < NV; j++) {
                        if (v0 + j >= vs1) continue;
                        pout[(long long)(v0 + j) * Kc + o] = old[q][j] + sv[j];
                    }
                }
                il += dq;
                jc += dr;
                if (jc >= nph_c) {
                    jc -= nph_c;
                    il++;
                }
            }
        }
    }
}

// aggregation, pipelined over the children and the right-hand sides:
// workgroup = (parent, chunk of parent theta rows, slice of the right-hand
// sides), on the separable form of the stencils (staged in LDS once).  For
// every pass of RB right-hand sides it walks the parent's children; while
// one child is interpolated in LDS, the next child's window (NPF samples per
// thread) and shift are in flight in registers.  Two barriers per child.
// Same arithmetic as k_aggregate, term for term.
template <class T, int RB, int NPF>
__global__ __launch_bounds__(STEP_THREADS) void k_aggregate_pipe(const LevelStep<T> a, int nrhs, int per_slice)
{
    constexpr int MS = 2, NO = 2;   // intermediate and output slots per thread
    extern __shared__ double step_lds_raw[];
    const long long blk = xcd_block_l((long long)a.nbox * a.nchunk);
    if (blk < 0) return;
    const int Pb = (int)(blk / a.nchunk), ch = (int)(blk % a.nchunk);
    const int rs0 = blockIdx.y * per_slice, rs1 = min(nrhs, rs0 + per_slice);
    const int cb = a.child_start[Pb], ce = a.child_start[Pb + 1];
    if (rs0 >= rs1) return;
    const int tid = threadIdx.x;
    const int Kc = a.nth_c * a.nph_c, Kp = a.nth_p * a.nph_p;
    const int nph_c = a.nph_c, nph_p = a.nph_p, tphi = a.tphi, tth = a.tth;
    const int i0 = ch * a.rows, i1 = min(a.nth_p, i0 + a.rows);
    const int w0 = a.win[2 * ch], w1 = a.win[2 * ch + 1];
    const int wlen = (w1 - w0) * nph_c, wmax = a.wrows * nph_c;
    const int mlen = (i1 - i0) * nph_c, mmax = a.rows * nph_c;
    const int olen = (i1 - i0) * nph_p;
    cpx<T> *cw = reinterpret_cast<cpx<T> *>(step_lds_raw);   // [RB][2][wmax] child window
    cpx<T> *mid = cw + 2 * RB * wmax;                         // [RB][2][mmax] intermediate rows
    T *s_thw = reinterpret_cast<T *>(mid + 2 * RB * mmax);    // [rows][tth]
    T *s_phw = s_thw + a.rows * tth;                          // [nph_p][tphi]
    int *s_thr = reinterpret_cast<int *>(s_phw + nph_p * tphi);   // [rows][tth]: window row * nph_c
    int *s_ths = s_thr + a.rows * tth;                        // [rows][tth]: phi shift
    int *s_phc = s_ths + a.rows * tth;                        // [nph_p][tphi]
    for (int i = tid; i < (i1 - i0) * tth; i += STEP_THREADS) {
        const int g = i0 * tth + i;
        s_thr[i] = (a.th_row[g] - w0) * nph_c;
        s_ths[i] = a.th_sh[g];
        s_thw[i] = a.th_w[g];
    }
    for (int i = tid; i < nph_p * tphi; i += STEP_THREADS) {
        s_phc[i] = a.phi_col[i];
        s_phw[i] = a.phi_w[i];
    }
    const long long hc = (long long)nrhs * Kc;   // second component
    const cpx<T> *shq = a.shift + (long long)i0 * nph_p;
    // the window and shift loads take clamped (valid) addresses and no
    // predicate: slots past the window or the outputs are never used, and a
    // load whose value is not selected right away stays in flight
    cpx<T> pf0[NPF][RB], pf1[NPF][RB], sfn[NO];
    auto load = [&](int r0, int cg) {
        const cpx<T> *u = a.in + (long long)cg * 2 * nrhs * Kc + (long long)w0 * nph_c;
#pragma unroll
        for (int k = 0; k < NPF; k++) {
            const int i = min(tid + k * STEP_THREADS, max(wlen - 1, 0));
#pragma unroll
            for (int j = 0; j < RB; j++) {
                const long long o = (long long)min(r0 + j, nrhs - 1) * Kc + i;
                pf0[k][j] = u[o];
                pf1[k][j] = u[hc + o];
            }
        }
        const cpx<T> *f = shq + (long long)a.oct[cg] * Kp;
#pragma unroll
        for (int q = 0; q < NO; q++) sfn[q] = f[min(tid + q * STEP_THREADS, max(olen - 1, 0))];
    };
    if (cb < ce) load(rs0, cb);
    const int dq = STEP_THREADS / nph_c, dr = STEP_THREADS - dq * nph_c;     // intermediate slots
    const int dqo = STEP_THREADS / nph_p, dro = STEP_THREADS - dqo * nph_p;  // output slots
    const int il0 = tid / nph_c, jc0 = tid - il0 * nph_c;
    const int io0 = tid / nph_p, jo0 = tid - io0 * nph_p;
    cpx<T> *pout = a.out + (long long)Pb * 2 * nrhs * Kp + (long long)i0 * nph_p;
    const long long hp = (long long)nrhs * Kp;
    for (int r0 = rs0; r0 < rs1; r0 += RB) {
        cpx<T> acc0[NO][RB], acc1[NO][RB];
#pragma unroll
        for (int q = 0; q < NO; q++)
#pragma unroll
            for (int j = 0; j < RB; j++) acc0[q][j] = acc1[q][j] = mk<T>(0, 0);
        for (int cg = cb; cg < ce; cg++) {
            // the previous child's theta stage is done (second barrier): overwrite cw
#pragma unroll
            for (int k = 0; k < NPF; k++) {
                const int i = tid + k * STEP_THREADS;
                if (i < wlen) {
#pragma unroll
                    for (int j = 0; j < RB; j++) {
                        cw[(2 * j) * wmax + i] = pf0[k][j];
                        cw[(2 * j + 1) * wmax + i] = pf1[k][j];
                    }
                }
            }
            cpx<T> sfc[NO];
#pragma unroll
            for (int q = 0; q < NO; q++) sfc[q] = sfn[q];
            // the next child, else the next pass's first child, else this
            // child again (loads issued on every path)
            if (cg + 1 < ce) load(r0, cg + 1);
            else load(r0 + RB < rs1 ? r0 + RB : r0, r0 + RB < rs1 ? cb : cg);
            __syncthreads();
            // theta: intermediate (parent theta row, child phi column)
            {
                int il = il0, jc = jc0;
#pragma unroll
                for (int q = 0; q < MS; q++) {
                    const int m = tid + q * STEP_THREADS;
                    if (m < mlen) {
                        const int *tr = s_thr + il * tth, *ts = s_ths + il * tth;
                        const T *tw = s_thw + il * tth;
                        cpx<T> s0[RB], s1[RB];
#pragma unroll
                        for (int j = 0; j < RB; j++) s0[j] = s1[j] = mk<T>(0, 0);
#pragma unroll 4
                        for (int t = 0; t < tth; t++) {
                            int col = jc + ts[t];
                            col = col >= nph_c ? col - nph_c : col;
                            const int jj = tr[t] + col;
                            const T wt = tw[t];
#pragma unroll
                            for (int j = 0; j < RB; j++) {
                                axpy_to(s0[j], wt, cw[(2 * j) * wmax + jj]);
                                axpy_to(s1[j], wt, cw[(2 * j + 1) * wmax + jj]);
                            }
                        }
#pragma unroll
                        for (int j = 0; j < RB; j++) {
                            mid[(2 * j) * mmax + m] = s0[j];
                            mid[(2 * j + 1) * mmax + m] = s1[j];
                        }
                    }
                    il += dq;
                    jc += dr;
                    if (jc >= nph_c) {
                        jc -= nph_c;
                        il++;
                    }
                }
            }
            __syncthreads();
            // phi and the shift to the parent centre
            {
                int il = io0, jp = jo0;
#pragma unroll
                for (int q = 0; q < NO; q++) {
                    const int o = tid + q * STEP_THREADS;
                    if (o < olen) {
                        const int *pc = s_phc + jp * tphi;
                        const T *pwt = s_phw + jp * tphi;
                        const int mb = il * nph_c;
                        cpx<T> s0[RB], s1[RB];
#pragma unroll
                        for (int j = 0; j < RB; j++) s0[j] = s1[j] = mk<T>(0, 0);
#pragma unroll 4
                        for (int t = 0; t < tphi; t++) {
                            const int jj = mb + pc[t];
                            const T wt = pwt[t];
#pragma unroll
                            for (int j = 0; j < RB; j++) {
                                axpy_to(s0[j], wt, mid[(2 * j) * mmax + jj]);
                                axpy_to(s1[j], wt, mid[(2 * j + 1) * mmax + jj]);
                            }
                        }
#pragma unroll
                        for (int j = 0; j < RB; j++) {
                            fma_to(acc0[q][j], sfc[q], s0[j]);
                            fma_to(acc1[q][j], sfc[q], s1[j]);
                        }
                    }
                    il += dqo;
                    jp += dro;
                    if (jp >= nph_p) {
                        jp -= nph_p;
                        il++;
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NO; q++) {
            const int o = tid + q * STEP_THREADS;
            if (o >= olen) continue;
#pragma unroll
            for (int j = 0; j < RB; j++) {
                if (r0 + j >= rs1) continue;
                const long long e = (long long)(r0 + j) * Kp + o;
                pout[e] = acc0[q][j];
                pout[hp + e] = acc1[q][j];
            }
        }
    }
}

// right-hand sides per workgroup: the step's own choice (the autotuner's)
// where it fits the LDS, else two where the LDS allows
inline int step_rb(int want, size_t lds1, int nrhs)
{
    int rb = 1;
    const int cap = want > 0 ? want : 2;
    while (2 * rb <= cap && 2 * rb <= nrhs && 2 * rb * lds1 <= STEP_LDS_MAX) rb *= 2;
    return rb;
}

}  // namespace

// outputs per thread: two where the chunk has at most 512 of them (fewer
// registers), else four
template <class T, int P>
void agg_launch(int G, int rb, dim3 grid, dim3 block, size_t lds, hipStream_t s, const LevelStep<T> &a, int nrhs)
{
    const bool two = (long long)a.rows * a.nph_p <= 2 * STEP_THREADS;
#define AGG(GR, OUT, RB) hipLaunchKernelGGL((k_aggregate<T, P, GR, OUT, RB>), grid, block, lds, s, a, nrhs, G)
    if (G > 1) {
        if (two) AGG(true, 2, 1);
        else AGG(true, STEP_OUT, 1);
    } else if (rb == 4) {
        if (two) AGG(false, 2, 4);
        else AGG(false, STEP_OUT, 4);
    } else if (rb == 2) {
        if (two) AGG(false, 2, 2);
        else AGG(false, STEP_OUT, 2);
    } else {
        if (two) AGG(false, 2, 1);
        else AGG(false, STEP_OUT, 1);
    }
#undef AGG
}

// slices of the right-hand sides for a pipelined step: enough workgroups to
// fill the GPU (about 8192), each slice a whole number of passes of rb
inline int pipe_slices(long long nblk, int nrhs, int rb, int &per)
{
    int slices = (int)std::min<long long>((nrhs + rb - 1) / rb, std::max<long long>(1, (8192 + nblk - 1) / nblk));
    per = (nrhs + slices - 1) / slices;
    per = (per + rb - 1) / rb * rb;
    return (nrhs + per - 1) / per;
}

// the pipelined aggregation with RB right-hand sides per pass; false when the
// step is not separable or the chunk does not fit its register and LDS limits
template <class T>
bool launch_aggregate_pipe(const LevelStep<T> &a, int nrhs, hipStream_t s)
{
    if (a.tth <= 0 || a.tphi <= 0) return false;
    const long long wlen = (long long)a.wrows * a.nph_c;
    const int npf = wlen <= STEP_THREADS ? 1 : wlen <= 2 * STEP_THREADS ? 2 : wlen <= 4 * STEP_THREADS ? 4 : 0;
    if (!npf || (long long)a.rows * a.nph_p > 2 * STEP_THREADS) return false;
    const size_t tables = (size_t)a.rows * a.tth * (sizeof(T) + 2 * sizeof(int)) +
                          (size_t)a.nph_p * a.tphi * (sizeof(T) + sizeof(int));
    // two right-hand sides per pass where asked for and within the limits, else one
    int RB = a.pipe >= 2 && nrhs >= 2 && npf <= 2 ? 2 : 1;
    if (RB == 2 && 2 * agg_lds_bytes<T>(a.wrows, a.rows, a.nph_c) + tables > STEP_LDS_MAX) RB = 1;
    const size_t lds = RB * agg_lds_bytes<T>(a.wrows, a.rows, a.nph_c) + tables;
    if (lds > STEP_LDS_MAX) return false;
    if (a.nbox <= 0 || nrhs <= 0) return true;
    const long long nblk = (long long)a.nbox * a.nchunk;
    int per = 0;
    const int slices = pipe_slices(nblk, nrhs, RB, per);
    const dim3 grid(xcd_grid_l(nblk), slices), block(STEP_THREADS);
#define AGGP(RB_, NPF_) hipLaunchKernelGGL((k_aggregate_pipe<T, RB_, NPF_>), grid, block, lds, s, a, nrhs, per)
    if (RB == 2 && npf == 1) AGGP(2, 1);
    else if (RB == 2) AGGP(2, 2);
    else if (npf == 1) AGGP(1, 1);
    else if (npf == 2) AGGP(1, 2);
    else AGGP(1, 4);
#undef AGGP
    return true;
}

template <class T>
bool launch_aggregate_step(const LevelStep<T> &a, int nrhs, hipStream_t s)
{
    if (a.pipe > 0 && launch_aggregate_pipe<T>(a, nrhs, s)) return true;
    if (a.nchunk <= 0 || (long long)a.rows * a.nph_p > STEP_OUT * STEP_THREADS) return false;
    if (a.taps != 6 && a.taps != 8 && a.taps != 10) return false;
    const size_t lds1 = agg_lds_bytes<T>(a.wrows, a.rows, a.nph_c);   // one child, one right-hand side
    if (lds1 > STEP_LDS_MAX) return false;
    if (a.nbox <= 0 || nrhs <= 0) return true;
    // with few right-hand sides the grid is small and the per-child barriers
    // dominate, so several children are grouped (four in single, two in
    // double precision: a parent on a surface has about four, and larger
    // groups hold LDS that costs occupancy); with more right-hand sides, one
    // child at a time and RB right-hand sides per workgroup
    const int gmax = sizeof(T) == 4 ? 4 : 2;
    int G = nrhs < 4 ? (int)std::min<size_t>(gmax, STEP_LDS_MAX / lds1) : 1;
    int rb = G > 1 ? 1 : step_rb(a.rb > 0 ? a.rb : 1, lds1, nrhs);
    if (a.group > 1) {   // the autotuner's children per group (one right-hand side each) where the LDS allows
        G = std::min(a.group, 4);
        while (G > 1 && (size_t)G * lds1 > STEP_LDS_MAX) G /= 2;
        rb = G > 1 ? 1 : step_rb(a.rb, lds1, nrhs);
    }
    const dim3 grid(xcd_grid_l((long long)a.nbox * a.nchunk), (nrhs + rb - 1) / rb), block(STEP_THREADS);
    const size_t lds = (size_t)G * rb * lds1;
    if (a.taps == 6) agg_launch<T, 6>(G, rb, grid, block, lds, s, a, nrhs);
    else if (a.taps == 8) agg_launch<T, 8>(G, rb, grid, block, lds, s, a, nrhs);
    else agg_launch<T, 10>(G, rb, grid, block, lds, s, a, nrhs);
    return true;
}

template <class T, int NV, int NPF>
void dis_pipe_launch(int no, dim3 grid, size_t lds, hipStream_t s, const LevelStep<T> &a, int nrhs, int per)
{
    if (no == 1) hipLaunchKernelGGL((k_disaggregate_pipe<T, NV, NPF, 1>), grid, dim3(STEP_THREADS), lds, s, a, nrhs, per);
    else hipLaunchKernelGGL((k_disaggregate_pipe<T, NV, NPF, 2>), grid, dim3(STEP_THREADS), lds, s, a, nrhs, per);
}

// the pipelined disaggregation with a.pipe vectors per pass (1, 2 or 4: one
// component, one right-hand side, two right-hand sides); fewer where the
// window does not fit the registers or LDS; false when even one does not
template <class T>
bool launch_disaggregate_pipe(const LevelStep<T> &a, int nrhs, hipStream_t s)
{
    const long long plen = (long long)a.wrows * a.nph_p, olen = (long long)a.rows * a.nph_c;
    const int npf = plen <= STEP_THREADS       ? 1
                    : plen <= 2 * STEP_THREADS ? 2
                    : plen <= 4 * STEP_THREADS ? 4
                    : plen <= 8 * STEP_THREADS ? 8
                                               : 0;
    const int no = olen <= STEP_THREADS ? 1 : olen <= 2 * STEP_THREADS ? 2 : 0;
    if (!npf || !no) return false;
    const size_t tables = (size_t)a.nph_c * a.tphi * (sizeof(T) + sizeof(int)) + (size_t)a.wrows * sizeof(T) +
                          (size_t)a.rows * a.tth * (sizeof(T) + 2 * sizeof(int));
    const size_t lds1 = dis_lds_bytes<T>(a.wrows, a.nph_p, a.nph_c) / 2;   // one vector
    int nv = a.pipe >= 4 ? 4 : a.pipe >= 2 ? 2 : 1;
    nv = std::min(nv, 2 * nrhs);
    while (nv > 1 && (nv * npf > 16 || nv * lds1 + tables > STEP_LDS_MAX)) nv /= 2;
    const size_t lds = nv * lds1 + tables;
    if (lds > STEP_LDS_MAX) return false;
    if (a.nbox <= 0 || nrhs <= 0) return true;
    const long long nblk = (long long)a.nbox * a.nchunk;
    int per = 0;
    const int slices = pipe_slices(nblk, 2 * nrhs, nv, per);
    const dim3 grid(xcd_grid_l(nblk), slices);
    if (nv == 4 && npf == 1) dis_pipe_launch<T, 4, 1>(no, grid, lds, s, a, nrhs, per);
    else if (nv == 4 && npf == 2) dis_pipe_launch<T, 4, 2>(no, grid, lds, s, a, nrhs, per);
    else if (nv == 4) dis_pipe_launch<T, 4, 4>(no, grid, lds, s, a, nrhs, per);
    else if (nv == 2 && npf == 1) dis_pipe_launch<T, 2, 1>(no, grid, lds, s, a, nrhs, per);
    else if (nv == 2 && npf == 2) dis_pipe_launch<T, 2, 2>(no, grid, lds, s, a, nrhs, per);
    else if (nv == 2 && npf == 4) dis_pipe_launch<T, 2, 4>(no, grid, lds, s, a, nrhs, per);
    else if (nv == 2) dis_pipe_launch<T, 2, 8>(no, grid, lds, s, a, nrhs, per);
    else if (npf == 1) dis_pipe_launch<T, 1, 1>(no, grid, lds, s, a, nrhs, per);
    else if (npf == 2) dis_pipe_launch<T, 1, 2>(no, grid, lds, s, a, nrhs, per);
    else if (npf == 4) dis_pipe_launch<T, 1, 4>(no, grid, lds, s, a, nrhs, per);
    else dis_pipe_launch<T, 1, 8>(no, grid, lds, s, a, nrhs, per);
    return true;
}

template <class T>
bool launch_disaggregate_step(const LevelStep<T> &a, int nrhs, hipStream_t s)
{
    if (a.nchunk <= 0 || a.tphi <= 0 || a.tth <= 0) return false;
    if (a.pipe > 0 && launch_disaggregate_pipe<T>(a, nrhs, s)) return true;
    const size_t lds1 = dis_lds_bytes<T>(a.wrows, a.nph_p, a.nph_c);
    if (lds1 > STEP_LDS_MAX) return false;
    if (a.nbox <= 0 || nrhs <= 0) return true;
    const int rb = step_rb(a.rb, lds1, nrhs);
    const dim3 grid(xcd_grid_l((long long)a.nbox * a.nchunk), (nrhs + rb - 1) / rb), block(STEP_THREADS);
    const size_t lds = rb * lds1;
    if (rb == 4) hipLaunchKernelGGL((k_disaggregate<T, 4>), grid, block, lds, s, a, nrhs);
    else if (rb == 2) hipLaunchKernelGGL((k_disaggregate<T, 2>), grid, block, lds, s, a, nrhs);
    else hipLaunchKernelGGL((k_disaggregate<T, 1>), grid, block, lds, s, a, nrhs);
    return true;
}

template bool launch_aggregate_step<float>(const LevelStep<float> &, int, hipStream_t);
template bool launch_aggregate_step<double>(const LevelStep<double> &, int, hipStream_t);
template bool launch_disaggregate_step<float>(const LevelStep<float> &, int, hipStream_t);
template bool launch_disaggregate_step<double>(const LevelStep<double> &, int, hipStream_t);

}  // namespace mlfma
