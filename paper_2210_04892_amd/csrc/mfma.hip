// Radiation and receive for many right-hand sides on the matrix cores.
//
// With nrhs right-hand sides both steps are dense complex products per leaf
// box b (Sec. II-E; the single-pattern far field of the C block and the L/K
// pair):
//   radiation  U_b[c](q, r) = sum_{n in b} alpha_n(r) R_n[c](q) + beta_n(r) (khat x R_n)[c](q)
//   receive    y_(m,h)(r)   += sum_{c, q} P_(m,h)[c](q) V_b[c](q, r)
// Each complex product is four real 16x16x4 MFMAs (real part: re*re and
// -im*im, imaginary part: re*im and im*re), FP32 for complex64 and FP64 for
// complex128.  Lane layout (wave64, both checked on the device): lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; it holds D[(l / 16) * 4 +
// v][l % 16] (v_mfma_f32_16x16x4f32) or D[l / 16 + 4 v][l % 16]
// (v_mfma_f64_16x16x4f64), v = 0..3.
#include "device.hpp"
#include "mfma_ops.hpp"
#include "../../include/mlfma.h"

namespace mlfma {

namespace {

constexpr int NXCD_M = 8;
__device__ inline long long xcd_block_m(long long nblk)
{
    const long long per = (nblk + NXCD_M - 1) / NXCD_M;
    const long long hw = blockIdx.x;
    const long long lb = (hw % NXCD_M) * per + hw / NXCD_M;
    return lb < nblk ? lb : -1;
}
inline unsigned xcd_grid_m(long long nblk) { return (unsigned)(((nblk + NXCD_M - 1) / NXCD_M) * NXCD_M); }

__device__ inline long long pidx_m(long long b, int c, int r, int q, int nrhs, int K)
{
    return ((b * 2 + c) * nrhs + r) * (long long)K + q;
}

// complex D += A B on RT accumulator pairs sharing the B operand
template <class T, int RT>
__device__ inline void cmfma(typename Mf<T>::v4 (&dre)[RT], typename Mf<T>::v4 (&dim)[RT], const cpx<T> (&a)[RT],
                             cpx<T> b)
{
#pragma unroll
    for (int t = 0; t < RT; t++) dre[t] = Mf<T>::mma(a[t].re, b.re, dre[t]);
#pragma unroll
    for (int t = 0; t < RT; t++) dim[t] = Mf<T>::mma(a[t].re, b.im, dim[t]);
#pragma unroll
    for (int t = 0; t < RT; t++) dre[t] = Mf<T>::mma(-a[t].im, b.im, dre[t]);
#pragma unroll
    for (int t = 0; t < RT; t++) dim[t] = Mf<T>::mma(a[t].im, b.re, dim[t]);
}

// Radiation.  Wave = (box, component c, ST tiles of 16 samples) x RT tiles
// of 16 right-hand sides; D[i = rhs][j = sample], inner index k = (RWG,
// alpha|beta): one MFMA step covers two RWGs.  EM pair: alpha = x1, beta =
// -x2; C block: alpha = x2 / 2, beta = x1 / 2.  The x values of a step (A
// operand) serve all ST sample tiles.  Steps with both RWGs in the box load
// without predicates, the next step's operands in flight while the current
// one is multiplied (two register sets taking turns; past the last step the
// loads repeat it).
template <class T, int RT, int ST>
__global__ __launch_bounds__(256) void k_radiate_mfma(int op, int nbox, int K, int nqt,
                                                      const int *__restrict__ box_start,
                                                      const cpx<T> *__restrict__ R,
                                                      const cpx<T> *__restrict__ X, cpx<T> *__restrict__ U,
                                                      int nrhs)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nqg = (nqt + ST - 1) / ST;   // groups of ST sample tiles
    const int tiles = 2 * nqg, per_box = (tiles + 3) / 4;
    const int nrg = (nrhs + 16 * RT - 1) / (16 * RT);
    const long long blk = xcd_block_m((long long)nbox * per_box * nrg);
    if (blk < 0) return;
    const int rg = (int)(blk % nrg);
    const long long bt = blk / nrg;
    const int b = (int)(bt / per_box), t = (int)(bt % per_box) * 4 + wave;
    if (t >= tiles) return;
    const int c = t / nqg, qg = t % nqg;
    const int lo = lane & 15, kk = lane >> 4;
    int qs[ST];        // this lane's sample in each tile
    long long qo[ST];  // its pattern offset, clamped to a valid sample
#pragma unroll
    for (int st = 0; st < ST; st++) {
        qs[st] = (qg * ST + st) * 16 + lo;
        qo[st] = min(qs[st], K - 1);
    }
    const int s = kk & 1;
    // which half of X feeds this lane's alpha/beta, and its factor
    const int h = op == MLFMA_OP_EM ? s : 1 - s;
    const T fac = op == MLFMA_OP_EM ? (s ? T(-1) : T(1)) : T(0.5);
    const int rcomp = s == 0 ? c : 1 - c;
    const T rsg = (s == 1 && c == 0) ? T(-1) : T(1);
    const int n0 = box_start[b], n1 = box_start[b + 1];
    int rr[RT];   // this lane's right-hand side per tile, clamped
#pragma unroll
    for (int u = 0; u < RT; u++) rr[u] = min((rg * RT + u) * 16 + lo, nrhs - 1);
    typename Mf<T>::v4 dre[ST][RT], dim[ST][RT];
#pragma unroll
    for (int st = 0; st < ST; st++)
#pragma unroll
        for (int u = 0; u < RT; u++) dre[st][u] = dim[st][u] = typename Mf<T>::v4{0, 0, 0, 0};
    struct Step {
        cpx<T> v[ST], x[RT];
    };
    auto load = [&](int nn, Step &o) {
        const cpx<T> *rn = R + (long long)nn * K * 2 + rcomp;
#pragma unroll
        for (int st = 0; st < ST; st++) o.v[st] = rn[qo[st] * 2];
        const cpx<T> *xn = X + ((long long)nn * 2 + h) * nrhs;
#pragma unroll
        for (int u = 0; u < RT; u++) o.x[u] = xn[rr[u]];
    };
    auto mult = [&](const Step &o) {
        cpx<T> av[RT];
#pragma unroll
        for (int u = 0; u < RT; u++) av[u] = fac * o.x[u];
#pragma unroll
        for (int st = 0; st < ST; st++) {
            // alpha lanes take R[c]; beta lanes (khat x R)[c]: (-R_phi, R_theta)
            const cpx<T> bv = mk<T>(rsg * o.v[st].re, rsg * o.v[st].im);
            cmfma<T, RT>(dre[st], dim[st], av, bv);
        }
    };
    // steps with both RWGs inside the box (samples past K and right-hand
    // sides past nrhs read clamped, valid elements; only their own outputs,
    // which are never stored, see them)
    const int nfull = (n1 - n0) / 2;
    auto rwg = [&](int step) { return n0 + 2 * min(step, nfull - 1) + (kk >> 1); };
    if (nfull > 0) {
        Step s0, s1;
        load(rwg(0), s0);
        for (int step = 0; step < nfull; step += 2) {
            load(rwg(step + 1), s1);
            mult(s0);
            if (step + 1 >= nfull) break;
            load(rwg(step + 2), s0);
            mult(s1);
        }
    }
    if (n0 + 2 * nfull < n1) {   // the last RWG of an odd box: lanes of the absent second RWG feed zeros
        const int nn = n0 + 2 * nfull + (kk >> 1);
        Step o;
        load(min(nn, n1 - 1), o);
        if (nn >= n1) {
#pragma unroll
            for (int st = 0; st < ST; st++) o.v[st] = mk<T>(0, 0);
#pragma unroll
            for (int u = 0; u < RT; u++) o.x[u] = mk<T>(0, 0);
        }
        mult(o);
    }
#pragma unroll
    for (int st = 0; st < ST; st++) {
        if (qs[st] >= K) continue;
#pragma unroll
        for (int u = 0; u < RT; u++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int r = (rg * RT + u) * 16 + Mf<T>::row(kk, v);
                if (r < nrhs) U[pidx_m(b, c, r, qs[st], nrhs, K)] = mk<T>(dre[st][u][v], dim[st][u][v]);
            }
    }
}

// Receive.  Work item = (leaf box, row tile of 16 rows (RWG m, half h),
// tile of 16 right-hand sides), one per wave, right-hand-side tiles
// innermost; D[i = (m, h)][j = rhs], inner index k = (component, sample).
// Rows: h = 0 uses (Pt, Pp), h = 1 uses (Pp, -Pt), with P = conj(R) for the
// EM pair and P = Q for the C block, weights wq folded in.  The samples go
// in blocks of 16: lane group kk (lanes 16 kk .. 16 kk + 15) loads samples
// 4 kk .. 4 kk + 3 of the block for its row (both components, 64 contiguous
// bytes) and for its right-hand side (32 bytes per component), and step u
// of the block takes sample 4 kk + u in every lane group: the same order of
// the inner index for the A and B operands, so that each lane reads whole
// runs of samples.  Two blocks are in flight while one is multiplied.
template <class T>
__global__ __launch_bounds__(256) void k_receive_mfma(int op, int nitem, const int2 *__restrict__ items, int K,
                                                      const int *__restrict__ box_start,
                                                      const cpx<T> *__restrict__ R,
                                                      const cpx<T> *__restrict__ Q, const T *__restrict__ wq,
                                                      const cpx<T> *__restrict__ V, cpx<T> *__restrict__ Y,
                                                      int nrhs)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nrt = (nrhs + 15) / 16;
    const long long blk = xcd_block_m(((long long)nitem * nrt + 3) / 4);
    if (blk < 0) return;
    const long long w = blk * 4 + wave;
    if (w >= (long long)nitem * nrt) return;
    const int2 it = items[w / nrt];
    const int rt = (int)(w % nrt);
    const int b = it.x, tile = it.y;
    const int n0 = box_start[b], rows = 2 * (box_start[b + 1] - n0);
    const int lo = lane & 15, kk = lane >> 4;
    const cpx<T> *pat = op == MLFMA_OP_EM ? R : Q;
    const bool cj = op == MLFMA_OP_EM;
    const int row = tile * 16 + lo, r = rt * 16 + lo;
    const bool mok = row < rows, rok = r < nrhs;
    const int h = row & 1;
    const cpx<T> *pm = pat + (long long)(n0 + (mok ? row / 2 : 0)) * K * 2;
    const cpx<T> *v0 = V + ((long long)(b * 2) * nrhs + (rok ? r : 0)) * K;
    const long long vstep = (long long)nrhs * K;   // second component of V
    const int nblk = (K + 15) / 16;
    // the lane's A operand in component pass c is one component of its row's
    // pattern: theta for (h, c) = (0, 0), phi for (0, 1) and (1, 0), minus
    // theta for (1, 1)
    const int comp0 = h == 0 ? 0 : 1, comp1 = h == 0 ? 1 : 0;
    const T sg1 = h == 1 ? T(-1) : T(1);
    struct Blk {
        cpx<T> q[4][2];   // pattern, samples x components
        cpx<T> v[2][4];   // V, components x samples
        T w[4];
    };
    auto load = [&](int bk, Blk &o) {
        const int q0 = bk * 16 + kk * 4;
        if (bk * 16 + 16 <= K) {   // the whole block (wave-uniform: one path per block)
            // rows past the box and right-hand sides past nrhs read row 0 /
            // right-hand side 0 (pm, v0 are clamped): they feed only D rows
            // and columns that are never stored
#pragma unroll
            for (int u = 0; u < 4; u++) {
                o.w[u] = wq[q0 + u];
                o.q[u][0] = pm[2 * (q0 + u)];
                o.q[u][1] = pm[2 * (q0 + u) + 1];
                o.v[0][u] = v0[q0 + u];
                o.v[1][u] = v0[vstep + q0 + u];
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int q = q0 + u;
                const bool qok = q < K;
                o.w[u] = qok ? wq[q] : T(0);
                o.q[u][0] = mok && qok ? pm[2 * q] : mk<T>(0, 0);
                o.q[u][1] = mok && qok ? pm[2 * q + 1] : mk<T>(0, 0);
                o.v[0][u] = rok && qok ? v0[q] : mk<T>(0, 0);
                o.v[1][u] = rok && qok ? v0[vstep + q] : mk<T>(0, 0);
            }
        }
    };
    typename Mf<T>::v4 dre = {0, 0, 0, 0}, dim = {0, 0, 0, 0};
    // DEPTH blocks in flight: block bk + DEPTH is loaded while block bk is
    // multiplied (one in double precision, where a block takes 72
    // registers).  The register sets take turns (no copies), and every path
    // issues the same loads (past the last block they repeat it), so that
    // the wait before a product counts the newer blocks' loads as in flight.
    constexpr int DEPTH = sizeof(T) == 8 ? 1 : 2;
    auto mult = [&](const Blk &cur) {
#pragma unroll
        for (int c = 0; c < 2; c++)
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int cp = c == 0 ? comp0 : comp1;
                cpx<T> p = cp ? cur.q[u][1] : cur.q[u][0];   // a select, not a dynamic register index
                if (cj) p = conjg(p);
                const cpx<T> a = ((c == 1 ? sg1 : T(1)) * cur.w[u]) * p;
                const cpx<T> bv = cur.v[c][u];
                dre = Mf<T>::mma(a.re, bv.re, dre);
                dim = Mf<T>::mma(a.re, bv.im, dim);
                dre = Mf<T>::mma(-a.im, bv.im, dre);
                dim = Mf<T>::mma(a.im, bv.re, dim);
            }
    };
    auto at = [&](int bk) { return min(bk, nblk - 1); };
    Blk b0, b1, b2;
    load(0, b0);
    if constexpr (DEPTH == 2) {
        load(at(1), b1);
        for (int bk = 0; bk < nblk; bk += 3) {
            load(at(bk + 2), b2);
            mult(b0);
            if (bk + 1 >= nblk) break;
            load(at(bk + 3), b0);
            mult(b1);
            if (bk + 2 >= nblk) break;
            load(at(bk + 4), b1);
            mult(b2);
        }
    } else {
        for (int bk = 0; bk < nblk; bk += 2) {
            load(at(bk + 1), b1);
            mult(b0);
            if (bk + 1 >= nblk) break;
            load(at(bk + 2), b0);
            mult(b1);
        }
    }
#pragma unroll
    for (int v = 0; v < 4; v++) {
        const int orow = tile * 16 + Mf<T>::row(kk, v);
        if (orow < rows && rok) {
            cpx<T> &y = Y[((long long)(n0 + orow / 2) * 2 + (orow & 1)) * nrhs + r];
            y = y + mk<T>(dre[v], dim[v]);
        }
    }
}

// Near field.  Work item = (leaf box b, row tile of 16 rows (RWG m, half
// h), tile of 16 right-hand sides), one per wave, right-hand-side tiles
// innermost so that neighbouring waves share the value rows.  The box's
// columns are the RWGs of its <= 27 adjacent boxes, concatenated (the order
// the stored (A, B) rows follow), listed in cols[col_off[b] ..].
// D[i = (m, h)][j = rhs] with inner index k = (column, half h'): two columns
// per MFMA step, taken in blocks of eight columns (four steps) whose inner
// index is permuted so that each lane reads its row's entries as runs.  The
// 2 x 2 block of a pair is [[A, -B], [B, A]].  The identity
// terms of the C block (Gram and rotated Gram, same triangle only) are added
// in the epilogue; Y is overwritten.
template <class T>
__global__ __launch_bounds__(256) void k_near_mfma(int nitem, const int2 *__restrict__ items,
                                                   const int *__restrict__ box_start,
                                                   const int *__restrict__ col_off, const int *__restrict__ cols,
                                                   const long long *__restrict__ val_off,
                                                   const cpx<T> *__restrict__ vals,
                                                   const int *__restrict__ id_start, const int *__restrict__ id_col,
                                                   const T *__restrict__ id_w, const cpx<T> *__restrict__ X,
                                                   cpx<T> *__restrict__ Y, int nrhs)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nrt = (nrhs + 15) / 16;
    const long long blk = xcd_block_m(((long long)nitem * nrt + 3) / 4);
    if (blk < 0) return;
    const long long w = blk * 4 + wave;
    if (w >= (long long)nitem * nrt) return;
    const int2 it = items[w / nrt];
    const int rt = (int)(w % nrt);
    const int b = it.x, tile = it.y;
    const int n0 = box_start[b], rows = 2 * (box_start[b + 1] - n0);
    const int *cl = cols + col_off[b];
    const int ncols = col_off[b + 1] - col_off[b];
    const int lo = lane & 15, kk = lane >> 4;
    const int jc = kk >> 1, hp = kk & 1;
    const int row = tile * 16 + lo, r = rt * 16 + lo;
    const bool mok = row < rows, rok = r < nrhs;
    const int h = row & 1;
    const cpx<T> *vr = vals + 2 * (val_off[b] + (long long)(mok ? row / 2 : 0) * ncols);
    const int vsel = h == hp ? 0 : 1;
    const T vsg = (h == 0 && hp == 1) ? T(-1) : T(1);
    // column indices 64 at a time, one per lane, handed out by lane shuffles
    // (so the x load of a step does not wait for an index load)
    int cbase = -64, myc = 0;
    auto cols_for = [&](int j0) {
        if (j0 >= cbase + 64) {   // j0 is even: a step never straddles two groups
            cbase = j0 - j0 % 64;
            myc = cl[min(cbase + lane, ncols - 1)];
        }
    };
    typename Mf<T>::v4 dre = {0, 0, 0, 0}, dim = {0, 0, 0, 0};
    auto mma = [&](cpx<T> a, cpx<T> bv) {
        dre = Mf<T>::mma(a.re, bv.re, dre);
        dim = Mf<T>::mma(a.re, bv.im, dim);
        dre = Mf<T>::mma(-a.im, bv.im, dre);
        dim = Mf<T>::mma(a.im, bv.re, dim);
    };
    const int rc = rok ? r : 0;
    // Blocks of 8 columns, four MFMA steps: lane group kk takes columns
    // j = j0 + 2 kk + c (c = 0, 1) and step u = 2 c + h' feeds column
    // j0 + 2 kk + c, half h' -- the same inner index for the A and B operands
    // -- so that a lane reads the (A, B) entries of its two columns as one
    // run of its row (rows past the tile and right-hand sides past nrhs read
    // clamped, valid elements that only feed outputs never stored).  The next
    // block's operands are in flight while a block is multiplied (two
    // register sets taking turns; past the last block the loads repeat it).
    const int nb8 = ncols / 8;
    const T sgb = h == 0 ? T(-1) : T(1);   // B's sign where h' != h
    struct Blk8 {
        cpx<T> v[4];   // A, B of the lane's first column, A, B of its second
        cpx<T> x[4];   // x of (column c, half h') at 2 c + h'
    };
    auto load8 = [&](int bi, Blk8 &o) {
        const int j0 = bi * 8, j = j0 + 2 * kk;
        cols_for(j0);
#pragma unroll
        for (int e = 0; e < 4; e++) o.v[e] = vr[2 * j + e];
        const int c0 = __shfl(myc, j - cbase), c1 = __shfl(myc, j + 1 - cbase);
#pragma unroll
        for (int hh = 0; hh < 2; hh++) {
            o.x[hh] = X[((long long)c0 * 2 + hh) * nrhs + rc];
            o.x[2 + hh] = X[((long long)c1 * 2 + hh) * nrhs + rc];
        }
    };
    auto mult8 = [&](const Blk8 &o) {
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int c = u >> 1, hh = u & 1;
            const cpx<T> av = hh == h ? o.v[2 * c] : sgb * o.v[2 * c + 1];
            mma(av, o.x[u]);
        }
    };
    if (nb8 > 0) {
        Blk8 s0, s1;
        load8(0, s0);
        for (int bi = 0; bi < nb8; bi += 2) {
            load8(min(bi + 1, nb8 - 1), s1);
            mult8(s0);
            if (bi + 1 >= nb8) break;
            load8(min(bi + 2, nb8 - 1), s0);
            mult8(s1);
        }
    }
    // the last ncols % 8 columns, two per step (lane group kk: column j0 +
    // kk / 2, half kk % 2)
    auto load = [&](int j0, cpx<T> &a, cpx<T> &bv) {
        cols_for(j0);
        const int j = j0 + jc;
        const bool jok = j < ncols;
        const int col = __shfl(myc, min(j, ncols - 1) - cbase);
        a = mk<T>(0, 0);
        bv = mk<T>(0, 0);
        if (jok && mok) {
            // [[A, -B], [B, A]]: the lane needs A on the diagonal, B (or -B) off it
            const cpx<T> v = vr[2 * j + vsel];
            a = mk<T>(vsg * v.re, vsg * v.im);
        }
        if (jok && rok) bv = X[((long long)col * 2 + hp) * nrhs + r];
    };
    for (int j0 = nb8 * 8; j0 < ncols; j0 += 2) {
        cpx<T> a, bv;
        load(j0, a, bv);
        mma(a, bv);
    }
#pragma unroll
    for (int v = 0; v < 4; v++) {
        const int orow = tile * 16 + Mf<T>::row(kk, v);
        if (orow >= rows || !rok) continue;
        const int m = n0 + orow / 2, oh = orow & 1;
        cpx<T> y = mk<T>(dre[v], dim[v]);
        if (id_start) {
            for (int e = id_start[m]; e < id_start[m + 1]; e++) {
                const long long col = id_col[e];
                const T g = id_w[2 * e], gx = id_w[2 * e + 1];
                const cpx<T> x1 = X[(col * 2) * nrhs + r], x2 = X[(col * 2 + 1) * nrhs + r];
                if (oh == 0) {
                    axpy_to(y, g, x1);
                    axpy_to(y, T(0.5) * gx, x2);
                } else {
                    axpy_to(y, T(0.5) * g, x2);
                }
            }
        }
        Y[((long long)m * 2 + oh) * nrhs + r] = y;
    }
}

}  // namespace

template <class T>
bool launch_near_mfma(int nitem, const int2 *items, const int *box_start, const int *col_off, const int *cols,
                      const long long *val_off, const cpx<T> *vals, const int *id_start, const int *id_col,
                      const T *id_w, const cpx<T> *X, cpx<T> *Y, int nrhs, hipStream_t s)
{
    if (nrhs < 16 || !items || !cols) return false;
    const long long nblk = ((long long)nitem * ((nrhs + 15) / 16) + 3) / 4;
    if (nblk <= 0) return true;
    hipLaunchKernelGGL(k_near_mfma<T>, dim3(xcd_grid_m(nblk)), dim3(256), 0, s, nitem, items, box_start, col_off,
                       cols, val_off, vals, id_start, id_col, id_w, X, Y, nrhs);
    return true;
}

template <class T>
bool launch_radiate_mfma(int op, int nbox, int K, const int *box_start, const cpx<T> *R, const cpx<T> *X, cpx<T> *U,
                         int nrhs, hipStream_t s)
{
    if (nrhs < 16) return false;
    const int nqt = (K + 15) / 16;
    // right-hand-side tiles per wave (the double-precision sums take twice
    // the registers); with one, two sample tiles share each x load
    const int rt = sizeof(T) == 8 ? (nrhs >= 32 ? 2 : 1) : (nrhs >= 64 ? 4 : (nrhs >= 32 ? 2 : 1));
    const int st = rt == 1 ? 2 : 1;
    const int per_box = (2 * ((nqt + st - 1) / st) + 3) / 4;
    const long long nblk = (long long)nbox * per_box * ((nrhs + 16 * rt - 1) / (16 * rt));
    if (nblk <= 0) return true;
    const dim3 grid(xcd_grid_m(nblk)), block(256);
    if (rt == 4)
        hipLaunchKernelGGL((k_radiate_mfma<T, 4, 1>), grid, block, 0, s, op, nbox, K, nqt, box_start, R, X, U, nrhs);
    else if (rt == 2)
        hipLaunchKernelGGL((k_radiate_mfma<T, 2, 1>), grid, block, 0, s, op, nbox, K, nqt, box_start, R, X, U, nrhs);
    else hipLaunchKernelGGL((k_radiate_mfma<T, 1, 2>), grid, block, 0, s, op, nbox, K, nqt, box_start, R, X, U, nrhs);
    return true;
}

template <class T>
bool launch_receive_mfma(int op, int nitem, const int2 *items, int K, const int *box_start, const cpx<T> *R,
                         const cpx<T> *Q, const T *wq, const cpx<T> *V, cpx<T> *Y, int nrhs, hipStream_t s)
{
    if (nrhs < 16 || !items) return false;
    const long long nblk = ((long long)nitem * ((nrhs + 15) / 16) + 3) / 4;
    if (nblk <= 0) return true;
    hipLaunchKernelGGL(k_receive_mfma<T>, dim3(xcd_grid_m(nblk)), dim3(256), 0, s, op, nitem, items, K, box_start, R,
                       Q, wq, V, Y, nrhs);
    return true;
}

#define MFMA_INST(T)                                                                                                 \
    template bool launch_near_mfma<T>(int, const int2 *, const int *, const int *, const int *, const long long *,    \
                                      const cpx<T> *, const int *, const int *, const T *, const cpx<T> *, cpx<T> *,  \
                                      int, hipStream_t);                                                              \
    template bool launch_radiate_mfma<T>(int, int, int, const int *, const cpx<T> *, const cpx<T> *, cpx<T> *, int,   \
                                         hipStream_t);                                                                \
    template bool launch_receive_mfma<T>(int, int, const int2 *, int, const int *, const cpx<T> *, const cpx<T> *,    \
                                         const T *, const cpx<T> *, cpx<T> *, int, hipStream_t);
MFMA_INST(float)
MFMA_INST(double)
#undef MFMA_INST

}  // namespace mlfma
