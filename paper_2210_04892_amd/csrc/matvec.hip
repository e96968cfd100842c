// Hot-path kernels of the MLFMA matvec for CDNA4 (gfx950, wave64).
//
// Vector layout inside the library: X[rwg][half][rhs] (rwg in Morton order,
// half 0 = J or E side, 1 = M or H side, rhs innermost).  Box patterns and
// stencil intermediates are sample-innermost: U[box][component][rhs][sample]
// with component 0 = theta, 1 = phi, so that the threads of a wave, which
// take consecutive samples, read and write consecutive addresses for every
// right-hand side.
// Every kernel is templated on the arithmetic type T (double or float) and
// on NR, the number of right-hand sides handled per thread (rhs chunk).
#include <type_traits>

#include "device.hpp"

namespace mlfma {

constexpr int WAVE = 64;

template <class T>
__device__ inline cpx<T> shfl_xor(cpx<T> v, int m)
{
    return {__shfl_xor(v.re, m, WAVE), __shfl_xor(v.im, m, WAVE)};
}

template <class T>
__device__ inline cpx<T> wave_sum(cpx<T> v)
{
#pragma unroll
    for (int m = WAVE / 2; m >= 1; m >>= 1) v = v + shfl_xor(v, m);
    return v;
}

static inline int nr_for(int nrhs) { return nrhs <= 1 ? 1 : (nrhs <= 4 ? 4 : 16); }

// element (box b, component c, rhs r, sample q) of a pattern array with K
// samples per box and nrhs right-hand sides
__device__ inline long long pidx(long long b, int c, int r, int q, int nrhs, int K)
{
    return ((b * 2 + c) * nrhs + r) * (long long)K + q;
}

// Workgroups are dispatched to the 8 XCDs round-robin (hardware block b runs
// on XCD b mod 8).  Remapping gives every XCD one contiguous range of logical
// blocks, so neighbouring boxes (Morton order) share that XCD's L2.  The grid
// is padded to a multiple of 8; padding blocks return -1.
constexpr int NXCD = 8;
__device__ inline long long xcd_block(long long nblk)
{
    const long long per = (nblk + NXCD - 1) / NXCD;
    const long long hw = blockIdx.x;
    const long long lb = (hw % NXCD) * per + hw / NXCD;
    return lb < nblk ? lb : -1;
}
static inline unsigned xcd_grid(long long nblk) { return (unsigned)(((nblk + NXCD - 1) / NXCD) * NXCD); }

// ------------------------------------------------------------------ permute
template <class T>
__global__ void k_perm_in(const cpx<T> *__restrict__ x, long long ldx, cpx<T> *__restrict__ X,
                          const int *__restrict__ perm, int N, int nrhs)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long total = (long long)N * 2 * nrhs;
    if (g >= total) return;
    int r = (int)(g % nrhs);
    long long ih = g / nrhs;
    int h = (int)(ih & 1);
    int i = (int)(ih >> 1);
    X[g] = x[(long long)r * ldx + (long long)h * N + perm[i]];
}

template <class T>
__global__ void k_perm_out(const cpx<T> *__restrict__ Y, cpx<T> *__restrict__ y, long long ldy,
                           const int *__restrict__ iperm, int N, int nrhs)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long total = (long long)N * 2 * nrhs;
    if (g >= total) return;
    int u = (int)(g % N);            // user row (coalesced writes)
    long long hr = g / N;
    int h = (int)(hr & 1);
    int r = (int)(hr >> 1);
    y[(long long)r * ldy + (long long)h * N + u] = Y[((long long)iperm[u] * 2 + h) * nrhs + r];
}

// Several right-hand sides: tiles of 64 user rows x 16 right-hand sides of
// one half, transposed through LDS.  The internal side (RHS innermost) is
// read or written as whole 16-element rows, the user side (column-major) as
// runs of 64 consecutive rows per column; the permutation is applied to the
// row index of the internal side (iperm: user RWG -> tree position).
constexpr int PT_U = 64, PT_R = 16;
template <class T, bool IN>
__global__ __launch_bounds__(256) void k_perm_tile(const cpx<T> *__restrict__ src, long long ld,
                                                   cpx<T> *__restrict__ dst, const int *__restrict__ iperm, int N,
                                                   int nrhs)
{
    __shared__ cpx<T> tile[PT_U][PT_R + 1];
    const int u0 = blockIdx.x * PT_U, h = blockIdx.y, r0 = blockIdx.z * PT_R;
    const int nu = min(PT_U, N - u0), nr = min(PT_R, nrhs - r0);
    if (IN) {
        // user x (coalesced along u) -> tile -> X rows of 16 right-hand sides
        for (int k = threadIdx.x; k < PT_U * PT_R; k += 256) {
            const int rr = k / PT_U, ul = k % PT_U;
            if (rr < nr && ul < nu) tile[ul][rr] = src[(long long)(r0 + rr) * ld + (long long)h * N + u0 + ul];
        }
        __syncthreads();
        for (int k = threadIdx.x; k < PT_U * PT_R; k += 256) {
            const int ul = k / PT_R, rr = k % PT_R;
            if (rr < nr && ul < nu) dst[((long long)iperm[u0 + ul] * 2 + h) * nrhs + r0 + rr] = tile[ul][rr];
        }
    } else {
        // Y rows of 16 right-hand sides -> tile -> user y (coalesced along u)
        for (int k = threadIdx.x; k < PT_U * PT_R; k += 256) {
            const int ul = k / PT_R, rr = k % PT_R;
            if (rr < nr && ul < nu) tile[ul][rr] = src[((long long)iperm[u0 + ul] * 2 + h) * nrhs + r0 + rr];
        }
        __syncthreads();
        for (int k = threadIdx.x; k < PT_U * PT_R; k += 256) {
            const int rr = k / PT_U, ul = k % PT_U;
            if (rr < nr && ul < nu) dst[(long long)(r0 + rr) * ld + (long long)h * N + u0 + ul] = tile[ul][rr];
        }
    }
}

// ---------------------------------------------------------------- near field
// One workgroup per leaf box; each wave owns rows of the box, its lanes
// stride over the row's near columns (the concatenated RWG ranges of the
// adjacent boxes).  Values are stored row-major per box as (A, B) pairs:
//   y1 += A x1 - B x2,  y2 += A x2 + B x1
// (A, B) = (T, K) for the EM pair; (-(T + Kx)/2, (Tx - K)/2) for the C block,
// whose Gram terms are the short per-row identity list (gram, gx):
//   y1 += gram x1 + gx x2 / 2,  y2 += gram x2 / 2.
template <class T, int NR>
__global__ __launch_bounds__(256) void k_near(int N, const int *__restrict__ leaf_of, const int *__restrict__ box_start,
                                              const int *__restrict__ near_start, const int *__restrict__ near_box,
                                              const long long *__restrict__ val_off, const cpx<T> *__restrict__ vals,
                                              const int *__restrict__ id_start, const int *__restrict__ id_col,
                                              const T *__restrict__ id_w, const cpx<T> *__restrict__ X,
                                              cpx<T> *__restrict__ Y, int nrhs)
{
    // one wave per output row m; the row's columns are the concatenated RWG
    // ranges of the <= 27 boxes adjacent to its leaf box
    __shared__ int cs_all[4][32], pre_all[4][33];
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const long long blk = xcd_block((N + 3) / 4);
    if (blk < 0) return;                        // whole (padding) workgroup
    const int m = (int)(blk * 4 + wave);
    const bool valid = m < N;                   // every wave reaches the barrier
    const int r0 = blockIdx.y * NR;
    int *cstart = cs_all[wave], *pre = pre_all[wave];
    const int b = valid ? leaf_of[m] : 0;
    const int nn = valid ? near_start[b + 1] - near_start[b] : 0;
    int cnt = 0, st = 0;
    if (lane < nn) {
        const int nb = near_box[near_start[b] + lane];
        st = box_start[nb];
        cnt = box_start[nb + 1] - st;
    }
    // inclusive prefix sum of the column counts across the wave
    int inc = cnt;
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
        const int v = __shfl_up(inc, d, WAVE);
        if (lane >= d) inc += v;
    }
    if (lane < nn) {
        cstart[lane] = st;
        pre[lane + 1] = inc;
    }
    if (lane == 0) pre[0] = 0;
    __syncthreads();
    if (!valid) return;
    const int ncols = pre[nn];
    const int mr = m - box_start[b];
    const cpx<T> *vrow = vals + 2 * (val_off[b] + (long long)mr * ncols);
    cpx<T> a1[NR], a2[NR];
#pragma unroll
    for (int rr = 0; rr < NR; rr++) a1[rr] = a2[rr] = mk<T>(0, 0);
    int q = 0;
    for (int j = lane; j < ncols; j += WAVE) {
        while (j >= pre[q + 1]) q++;
        const long long col = cstart[q] + (j - pre[q]);
        const cpx<T> A = vrow[2 * j], B = vrow[2 * j + 1];
#pragma unroll
        for (int rr = 0; rr < NR; rr++) {
            if (NR > 1 && r0 + rr >= nrhs) continue;
            const cpx<T> x1 = X[(col * 2) * nrhs + r0 + rr], x2 = X[(col * 2 + 1) * nrhs + r0 + rr];
            fma_to(a1[rr], A, x1);
            fms_to(a1[rr], B, x2);
            fma_to(a2[rr], A, x2);
            fma_to(a2[rr], B, x1);
        }
    }
    if (id_start) {
        const int e = id_start[m] + lane;
        if (e < id_start[m + 1]) {
            const long long col = id_col[e];
            const T g = id_w[2 * e], gx = id_w[2 * e + 1];
#pragma unroll
            for (int rr = 0; rr < NR; rr++) {
                if (NR > 1 && r0 + rr >= nrhs) continue;
                const cpx<T> x1 = X[(col * 2) * nrhs + r0 + rr], x2 = X[(col * 2 + 1) * nrhs + r0 + rr];
                axpy_to(a1[rr], g, x1);
                axpy_to(a1[rr], T(0.5) * gx, x2);
                axpy_to(a2[rr], T(0.5) * g, x2);
            }
        }
    }
#pragma unroll
    for (int rr = 0; rr < NR; rr++) {
        const cpx<T> s1 = wave_sum(a1[rr]), s2 = wave_sum(a2[rr]);
        if (lane == 0 && (NR == 1 || r0 + rr < nrhs)) {
            Y[((long long)m * 2) * nrhs + r0 + rr] = s1;
            Y[((long long)m * 2 + 1) * nrhs + r0 + rr] = s2;
        }
    }
}

// Near field for one right-hand side.  Wave = (leaf box, RWV of the up to 8
// RWGs of one (box, 16-row tile) work item); lanes over the box's columns
// (the RWGs of its adjacent boxes, concatenated in cols), so every column's
// x is loaded once for the wave's rows and the column structure is not
// rebuilt per row.  Rows are written (=), identity terms of the C
// block added by the lane that owns the row.
template <class T, int RWV>
__global__ __launch_bounds__(256) void k_near_tile(int nitem, const int2 *__restrict__ items,
                                                   const int *__restrict__ box_start, const int *__restrict__ col_off,
                                                   const int *__restrict__ cols, const long long *__restrict__ val_off,
                                                   const cpx<T> *__restrict__ vals, const int *__restrict__ id_start,
                                                   const int *__restrict__ id_col, const T *__restrict__ id_w,
                                                   const cpx<T> *__restrict__ X, cpx<T> *__restrict__ Y)
{
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    constexpr int SUB = 8 / RWV;                 // waves per work item
    const long long blk = xcd_block(((long long)nitem * SUB + 3) / 4);
    if (blk < 0) return;
    const long long w = blk * 4 + wave;
    if (w >= (long long)nitem * SUB) return;
    const int2 it = items[w / SUB];
    const int b = it.x, m0 = it.y * 8 + (int)(w % SUB) * RWV;
    const int n0 = box_start[b], nr = min(RWV, box_start[b + 1] - n0 - m0);
    if (nr <= 0) return;
    const int *cl = cols + col_off[b];
    const int ncols = col_off[b + 1] - col_off[b];
    const cpx<T> *vr = vals + 2 * (val_off[b] + (long long)m0 * ncols);
    cpx<T> a1[RWV], a2[RWV];
#pragma unroll
    for (int i = 0; i < RWV; i++) a1[i] = a2[i] = mk<T>(0, 0);
    // rows past the tile's last re-read that row (branch-free, so that all
    // loads of an iteration are in flight together); their sums are dropped
    // one column chunk per pass (more chunks lower the occupancy more than
    // they add loads in flight); columns past the row end re-read its last
    // column with weight zero
    constexpr int CH = 1;
    for (int j0 = lane; j0 < ncols; j0 += CH * WAVE) {
        cpx<T> A[CH][RWV], B[CH][RWV], x1[CH], x2[CH];
#pragma unroll
        for (int c = 0; c < CH; c++) {
            const int j = min(j0 + c * WAVE, ncols - 1);
            const long long col = cl[j];
#pragma unroll
            for (int i = 0; i < RWV; i++) {
                const long long o = 2 * ((long long)(i < nr ? i : nr - 1) * ncols + j);
                load_pair_once(vr + o, A[c][i], B[c][i]);
            }
            const T z = j0 + c * WAVE < ncols ? T(1) : T(0);
            x1[c] = z * X[col * 2];
            x2[c] = z * X[col * 2 + 1];
        }
#pragma unroll
        for (int c = 0; c < CH; c++)
#pragma unroll
            for (int i = 0; i < RWV; i++) {
                fma_to(a1[i], A[c][i], x1[c]);
                fms_to(a1[i], B[c][i], x2[c]);
                fma_to(a2[i], A[c][i], x2[c]);
                fma_to(a2[i], B[c][i], x1[c]);
            }
    }
    cpx<T> y1 = mk<T>(0, 0), y2 = mk<T>(0, 0);
#pragma unroll
    for (int i = 0; i < RWV; i++) {
        if (i >= nr) break;
        const cpx<T> s1 = wave_sum(a1[i]), s2 = wave_sum(a2[i]);
        if (lane == i) {
            y1 = s1;
            y2 = s2;
        }
    }
    if (lane >= nr) return;
    const int m = n0 + m0 + lane;
    if (id_start) {
        for (int e = id_start[m]; e < id_start[m + 1]; e++) {
            const long long col = id_col[e];
            const T g = id_w[2 * e], gx = id_w[2 * e + 1];
            const cpx<T> x1 = X[col * 2], x2 = X[col * 2 + 1];
            axpy_to(y1, g, x1);
            axpy_to(y1, T(0.5) * gx, x2);
            axpy_to(y2, T(0.5) * g, x2);
        }
    }
    Y[(long long)m * 2] = y1;
    Y[(long long)m * 2 + 1] = y2;
}

// Broadcast lane `src` of a wave (uniform src) through the scalar unit.
__device__ inline float bcast(float v, int src)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ inline double bcast(double v, int src)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline int bcast(int v, int src) { return __builtin_amdgcn_readlane(v, src); }

// Near field for many right-hand sides: one wave per output row, lane = one
// right-hand side of a chunk of 64.  The row's (A, B) pairs and column
// indices are loaded 64 at a time (one per lane, coalesced) and broadcast
// through the scalar unit; every x load is coalesced over the lanes (rhs is
// innermost in X), and each lane accumulates its own outputs.
template <class T>
__global__ __launch_bounds__(256) void k_near_rhs(int N, const int *__restrict__ leaf_of,
                                                  const int *__restrict__ box_start, const int *__restrict__ near_start,
                                                  const int *__restrict__ near_box, const long long *__restrict__ val_off,
                                                  const cpx<T> *__restrict__ vals, const int *__restrict__ id_start,
                                                  const int *__restrict__ id_col, const T *__restrict__ id_w,
                                                  const cpx<T> *__restrict__ X, cpx<T> *__restrict__ Y, int nrhs)
{
    __shared__ int cs_all[4][32], pre_all[4][33];
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const long long blk = xcd_block((N + 3) / 4);
    if (blk < 0) return;
    const int m = (int)(blk * 4 + wave);
    const bool valid = m < N;
    int *cstart = cs_all[wave], *pre = pre_all[wave];
    const int b = valid ? leaf_of[m] : 0;
    const int nn = valid ? near_start[b + 1] - near_start[b] : 0;
    int cnt = 0, st = 0;
    if (lane < nn) {
        const int nb = near_box[near_start[b] + lane];
        st = box_start[nb];
        cnt = box_start[nb + 1] - st;
    }
    int inc = cnt;
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
        const int v = __shfl_up(inc, d, WAVE);
        if (lane >= d) inc += v;
    }
    if (lane < nn) {
        cstart[lane] = st;
        pre[lane + 1] = inc;
    }
    if (lane == 0) pre[0] = 0;
    __syncthreads();
    if (!valid) return;
    const int ncols = pre[nn];
    const int mr = m - box_start[b];
    const cpx<T> *vrow = vals + 2 * (val_off[b] + (long long)mr * ncols);
    const int r = blockIdx.y * WAVE + lane;
    const bool act = r < nrhs;
    cpx<T> y1 = mk<T>(0, 0), y2 = mk<T>(0, 0);
    int q = 0;
    for (int j0 = 0; j0 < ncols; j0 += WAVE) {
        const int j = j0 + lane;
        cpx<T> A = mk<T>(0, 0), B = mk<T>(0, 0);
        int col = 0;
        if (j < ncols) {
            while (j >= pre[q + 1]) q++;
            col = cstart[q] + (j - pre[q]);
            A = vrow[2 * j];
            B = vrow[2 * j + 1];
        }
        const int cnt_j = ncols - j0 < WAVE ? ncols - j0 : WAVE;
        for (int jj = 0; jj < cnt_j; jj++) {
            const cpx<T> a = {bcast(A.re, jj), bcast(A.im, jj)}, bb = {bcast(B.re, jj), bcast(B.im, jj)};
            const long long c = bcast(col, jj);
            if (act) {
                const cpx<T> x1 = X[(c * 2) * nrhs + r], x2 = X[(c * 2 + 1) * nrhs + r];
                fma_to(y1, a, x1);
                fms_to(y1, bb, x2);
                fma_to(y2, a, x2);
                fma_to(y2, bb, x1);
            }
        }
    }
    if (id_start && act) {
        for (int e = id_start[m]; e < id_start[m + 1]; e++) {
            const long long c = id_col[e];
            const T g = id_w[2 * e], gx = id_w[2 * e + 1];
            const cpx<T> x1 = X[(c * 2) * nrhs + r], x2 = X[(c * 2 + 1) * nrhs + r];
            axpy_to(y1, g, x1);
            axpy_to(y1, T(0.5) * gx, x2);
            axpy_to(y2, T(0.5) * g, x2);
        }
    }
    if (act) {
        Y[((long long)m * 2) * nrhs + r] = y1;
        Y[((long long)m * 2 + 1) * nrhs + r] = y2;
    }
}

// ---------------------------------------------------------------- radiation
// U_b(k) = sum_{n in b} alpha_n R_n(k) + beta_n (khat x R_n)(k),
// khat x (v_theta, v_phi) = (-v_phi, v_theta).
// EM pair: alpha = x1, beta = -x2.  C block: alpha = x2 / 2, beta = x1 / 2.
// Radiation for one right-hand side: one wave per (leaf box, chunk of 64
// samples), so that every lane of a wave belongs to the same box and the
// box's coefficients are wave-uniform (scalar loads); the patterns of eight
// RWGs (four in double precision) are loaded before they are used.
template <class T, bool PERM>
__global__ __launch_bounds__(256) void k_radiate1(int op, int nbox, int K, int nqc, const int *__restrict__ box_start,
                                                  const cpx<T> *__restrict__ R, const cpx<T> *__restrict__ X,
                                                  cpx<T> *__restrict__ U, const cpx<T> *__restrict__ xu,
                                                  const int *__restrict__ perm, int N, cpx<T> *__restrict__ Xw)
{
    constexpr int G = sizeof(T) == 4 ? 8 : 4;
    const int lane = threadIdx.x % WAVE;
    const long long blk = xcd_block(((long long)nbox * nqc + 3) / 4);
    if (blk < 0) return;
    const long long w = blk * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    if (w >= (long long)nbox * nqc) return;
    const int b = (int)(w / nqc), q = (int)(w % nqc) * WAVE + lane;
    const bool qok = q < K;
    const int qq = qok ? q : K - 1;
    const int n0 = box_start[b], n1 = box_start[b + 1];
    cpx<T> ut = mk<T>(0, 0), up = ut;
    // RWGs i0 .. i1 - 1, G at a time; xat(i, x1, x2) gives the coefficients
    auto rwgs = [&](int i0, int i1, auto xat) {
        for (int j0 = i0; j0 < i1; j0 += G) {
            cpx<T> Rt[G], Rp[G], al[G], be[G];
#pragma unroll
            for (int u = 0; u < G; u++) {
                const int i = min(j0 + u, i1 - 1);
                load_pair(R + ((long long)i * K + qq) * 2, Rt[u], Rp[u]);
                cpx<T> x1, x2;
                xat(i, x1, x2);
                const T z = j0 + u < i1 ? T(1) : T(0);   // RWGs past the box contribute nothing
                if (op == 1) {
                    al[u] = z * x1;
                    be[u] = mk<T>(-z * x2.re, -z * x2.im);
                } else {
                    al[u] = (T(0.5) * z) * x2;
                    be[u] = (T(0.5) * z) * x1;
                }
            }
#pragma unroll
            for (int u = 0; u < G; u++) {
                fma_to(ut, al[u], Rt[u]);
                fms_to(ut, be[u], Rp[u]);
                fma_to(up, al[u], Rp[u]);
                fma_to(up, be[u], Rt[u]);
            }
        }
    };
    if constexpr (PERM) {
        // coefficients taken from the caller's vector (user order) through
        // the permutation, 32 RWGs at a time: lane 2 r + h holds half h of
        // RWG c0 + r and broadcasts it; the box's first sample chunk also
        // stores them in tree order for the near field
        for (int c0 = n0; c0 < n1; c0 += WAVE / 2) {
            const int c1 = min(c0 + WAVE / 2, n1);
            cpx<T> xv = mk<T>(0, 0);
            if (lane < 2 * (c1 - c0)) {
                xv = xu[(long long)(lane & 1) * N + perm[c0 + (lane >> 1)]];
                if (w % nqc == 0) Xw[2LL * c0 + lane] = xv;
            }
            rwgs(c0, c1, [&](int i, cpx<T> &x1, cpx<T> &x2) {
                const int l = 2 * (i - c0);
                x1 = mk<T>(bcast(xv.re, l), bcast(xv.im, l));
                x2 = mk<T>(bcast(xv.re, l + 1), bcast(xv.im, l + 1));
            });
        }
    } else {
        rwgs(n0, n1, [&](int i, cpx<T> &x1, cpx<T> &x2) {
            x1 = X[(long long)i * 2];
            x2 = X[(long long)i * 2 + 1];
        });
    }
    if (qok) {
        U[pidx(b, 0, 0, q, 1, K)] = ut;
        U[pidx(b, 1, 0, q, 1, K)] = up;
    }
}

template <class T, int NR>
__global__ __launch_bounds__(256) void k_radiate(int op, int nbox, int K, const int *__restrict__ box_start,
                                                 const cpx<T> *__restrict__ R, const cpx<T> *__restrict__ X,
                                                 cpx<T> *__restrict__ U, int nrhs)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)nbox * K) return;
    const int b = (int)(g / K), q = (int)(g % K);
    const int r0 = blockIdx.y * NR;
    cpx<T> ut[NR], up[NR];
#pragma unroll
    for (int rr = 0; rr < NR; rr++) ut[rr] = up[rr] = mk<T>(0, 0);
#pragma unroll 4
    for (int i = box_start[b]; i < box_start[b + 1]; i++) {
        const cpx<T> Rt = R[((long long)i * K + q) * 2], Rp = R[((long long)i * K + q) * 2 + 1];
#pragma unroll
        for (int rr = 0; rr < NR; rr++) {
            if (NR > 1 && r0 + rr >= nrhs) continue;
            const cpx<T> x1 = X[((long long)i * 2) * nrhs + r0 + rr], x2 = X[((long long)i * 2 + 1) * nrhs + r0 + rr];
            cpx<T> al, be;
            if (op == 1) {
                al = x1;
                be = mk<T>(-x2.re, -x2.im);
            } else {
                al = T(0.5) * x2;
                be = T(0.5) * x1;
            }
            fma_to(ut[rr], al, Rt);
            fms_to(ut[rr], be, Rp);
            fma_to(up[rr], al, Rp);
            fma_to(up[rr], be, Rt);
        }
    }
#pragma unroll
    for (int rr = 0; rr < NR; rr++) {
        if (NR > 1 && r0 + rr >= nrhs) continue;
        U[pidx(b, 0, r0 + rr, q, nrhs, K)] = ut[rr];
        U[pidx(b, 1, r0 + rr, q, nrhs, K)] = up[rr];
    }
}

// ------------------------------------------------- sparse stencil (per box)
// out[box][row] (=, +=) sum_e w_e in[box][col_e], both components, all rhs
// (in has in_len samples per box, out has rows).
template <class T, int NR>
__global__ __launch_bounds__(256) void k_interp(int nbox, int rows, int in_len, const int *__restrict__ st,
                                                const int *__restrict__ col, const T *__restrict__ w,
                                                const cpx<T> *__restrict__ in, cpx<T> *__restrict__ out, int nrhs,
                                                int accumulate)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)nbox * rows) return;
    const int box = (int)(g / rows), row = (int)(g % rows);
    const int r0 = blockIdx.y * NR;
    cpx<T> a0[NR], a1[NR];
#pragma unroll
    for (int rr = 0; rr < NR; rr++) a0[rr] = a1[rr] = mk<T>(0, 0);
    const int e1 = st[row + 1];
    int e = st[row];
    for (; e + 4 <= e1; e += 4) {
        int c[4];
        T we[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            c[u] = col[e + u];
            we[u] = w[e + u];
        }
#pragma unroll
        for (int rr = 0; rr < NR; rr++) {
            if (NR > 1 && r0 + rr >= nrhs) continue;
            cpx<T> v0[4], v1[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                v0[u] = in[pidx(box, 0, r0 + rr, c[u], nrhs, in_len)];
                v1[u] = in[pidx(box, 1, r0 + rr, c[u], nrhs, in_len)];
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                axpy_to(a0[rr], we[u], v0[u]);
                axpy_to(a1[rr], we[u], v1[u]);
            }
        }
    }
    for (; e < e1; e++) {
        const T we = w[e];
        const int c = col[e];
#pragma unroll
        for (int rr = 0; rr < NR; rr++) {
            if (NR > 1 && r0 + rr >= nrhs) continue;
            axpy_to(a0[rr], we, in[pidx(box, 0, r0 + rr, c, nrhs, in_len)]);
            axpy_to(a1[rr], we, in[pidx(box, 1, r0 + rr, c, nrhs, in_len)]);
        }
    }
#pragma unroll
    for (int rr = 0; rr < NR; rr++) {
        if (NR > 1 && r0 + rr >= nrhs) continue;
        cpx<T> *o0 = &out[pidx(box, 0, r0 + rr, row, nrhs, rows)];
        cpx<T> *o1 = &out[pidx(box, 1, r0 + rr, row, nrhs, rows)];
        if (accumulate) {
            *o0 = *o0 + a0[rr];
            *o1 = *o1 + a1[rr];
        } else {
            *o0 = a0[rr];
            *o1 = a1[rr];
        }
    }
}

// Forward theta stencil with exactly P taps per row (the interpolation
// stencils are fixed-size): all P gathers are issued before the sums.
template <class T, int NR, int P>
__global__ __launch_bounds__(256) void k_interp_fixed(int nbox, int rows, int in_len, const int *__restrict__ col,
                                                      const T *__restrict__ w, const cpx<T> *__restrict__ in,
                                                      cpx<T> *__restrict__ out, int nrhs)
{
    const long long blk = xcd_block(((long long)nbox * rows + blockDim.x - 1) / blockDim.x);
    if (blk < 0) return;
    const long long g = blk * blockDim.x + threadIdx.x;
    if (g >= (long long)nbox * rows) return;
    const int box = (int)(g / rows), row = (int)(g % rows);
    const int r0 = blockIdx.y * NR;
    int c[P];
    T wt[P];
#pragma unroll
    for (int t = 0; t < P; t++) {
        c[t] = col[(long long)row * P + t];
        wt[t] = w[(long long)row * P + t];
    }
#pragma unroll
    for (int rr = 0; rr < NR; rr++) {
        if (NR > 1 && r0 + rr >= nrhs) continue;
#pragma unroll
        for (int comp = 0; comp < 2; comp++) {
            const cpx<T> *src = in + pidx(box, comp, r0 + rr, 0, nrhs, in_len);
            cpx<T> v[P];
#pragma unroll
            for (int t = 0; t < P; t++) v[t] = src[c[t]];
            cpx<T> acc = mk<T>(0, 0);
#pragma unroll
            for (int t = 0; t < P; t++) axpy_to(acc, wt[t], v[t]);
            out[pidx(box, comp, r0 + rr, row, nrhs, rows)] = acc;
        }
    }
}

// Aggregation phi stage with exactly P taps per parent sample.
template <class T, int NR, int P>
__global__ __launch_bounds__(256) void k_agg_phi_fixed(int nparent, int Kp, int mid_len,
                                                       const int *__restrict__ child_start,
                                                       const int *__restrict__ child_oct,
                                                       const cpx<T> *__restrict__ shift, const int *__restrict__ col,
                                                       const T *__restrict__ w, const cpx<T> *__restrict__ mid,
                                                       cpx<T> *__restrict__ Up, int nrhs)
{
    const long long blk = xcd_block(((long long)nparent * Kp + blockDim.x - 1) / blockDim.x);
    if (blk < 0) return;
    const long long g = blk * blockDim.x + threadIdx.x;
    if (g >= (long long)nparent * Kp) return;
    const int Pb = (int)(g / Kp), q = (int)(g % Kp);
    const int r0 = blockIdx.y * NR;
    int c[P];
    T wt[P];
#pragma unroll
    for (int t = 0; t < P; t++) {
        c[t] = col[(long long)q * P + t];
        wt[t] = w[(long long)q * P + t];
    }
    cpx<T> a0[NR], a1[NR];
#pragma unroll
    for (int rr = 0; rr < NR; rr++) a0[rr] = a1[rr] = mk<T>(0, 0);
    for (int ch = child_start[Pb]; ch < child_start[Pb + 1]; ch++) {
        const cpx<T> sh = shift[(long long)child_oct[ch] * Kp + q];
#pragma unroll
        for (int rr = 0; rr < NR; rr++) {
            if (NR > 1 && r0 + rr >= nrhs) continue;
            const cpx<T> *m0 = mid + pidx(ch, 0, r0 + rr, 0, nrhs, mid_len);
            const cpx<T> *m1 = mid + pidx(ch, 1, r0 + rr, 0, nrhs, mid_len);
            cpx<T> v0[P], v1[P];
#pragma unroll
            for (int t = 0; t < P; t++) {
                v0[t] = m0[c[t]];
                v1[t] = m1[c[t]];
            }
            cpx<T> s0 = mk<T>(0, 0), s1 = mk<T>(0, 0);
#pragma unroll
            for (int t = 0; t < P; t++) {
                axpy_to(s0, wt[t], v0[t]);
                axpy_to(s1, wt[t], v1[t]);
            }
            fma_to(a0[rr], sh, s0);
            fma_to(a1[rr], sh, s1);
        }
    }
#pragma unroll
    for (int rr = 0; rr < NR; rr++) {
        if (NR > 1 && r0 + rr >= nrhs) continue;
        Up[pidx(Pb, 0, r0 + rr, q, nrhs, Kp)] = a0[rr];
        Up[pidx(Pb, 1, r0 + rr, q, nrhs, Kp)] = a1[rr];
    }
}

// ----------------------------------------- aggregation: phi stage + shift
// U_P(k) = sum_{children c} exp(+jk khat.(r_c - r_P)) [A_phi mid_c](k)
template <class T, int NR>
__global__ __launch_bounds__(256) void k_agg_phi(int nparent, int Kp, int mid_len, const int *__restrict__ child_start,
                                                 const int *__restrict__ child_oct, const cpx<T> *__restrict__ shift,
                                                 const int *__restrict__ st, const int *__restrict__ col,
                                                 const T *__restrict__ w, const cpx<T> *__restrict__ mid,
                                                 cpx<T> *__restrict__ Up, int nrhs)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)nparent * Kp) return;
    const int P = (int)(g / Kp), q = (int)(g % Kp);
    const int r0 = blockIdx.y * NR;
    cpx<T> a0[NR], a1[NR];
#pragma unroll
    for (int rr = 0; rr < NR; rr++) a0[rr] = a1[rr] = mk<T>(0, 0);
    for (int c = child_start[P]; c < child_start[P + 1]; c++) {
        cpx<T> s0[NR], s1[NR];
#pragma unroll
        for (int rr = 0; rr < NR; rr++) s0[rr] = s1[rr] = mk<T>(0, 0);
        for (int e = st[q]; e < st[q + 1]; e++) {
            const T we = w[e];
            const int cc = col[e];
#pragma unroll
            for (int rr = 0; rr < NR; rr++) {
                if (NR > 1 && r0 + rr >= nrhs) continue;
                axpy_to(s0[rr], we, mid[pidx(c, 0, r0 + rr, cc, nrhs, mid_len)]);
                axpy_to(s1[rr], we, mid[pidx(c, 1, r0 + rr, cc, nrhs, mid_len)]);
            }
        }
        const cpx<T> sh = shift[(long long)child_oct[c] * Kp + q];
#pragma unroll
        for (int rr = 0; rr < NR; rr++) {
            fma_to(a0[rr], sh, s0[rr]);
            fma_to(a1[rr], sh, s1[rr]);
        }
    }
#pragma unroll
    for (int rr = 0; rr < NR; rr++) {
        if (NR > 1 && r0 + rr >= nrhs) continue;
        Up[pidx(P, 0, r0 + rr, q, nrhs, Kp)] = a0[rr];
        Up[pidx(P, 1, r0 + rr, q, nrhs, Kp)] = a1[rr];
    }
}

// ---------------------------------------------------------------- translation
// V_A(k) = sum_{(B, o) in IL(A)} T_o(k) U_B(k)   (diagonal in k)
//
// Workgroup = (tile, chunk of samples, group of right-hand sides), all levels
// in one grid; wave j of the workgroup owns the tile's j-th target box.  The
// lanes of a wave take QW consecutive samples for each of RW right-hand sides
// (QW * RW = 64).  The source patterns of the tile (both components, the
// chunk's samples and right-hand sides) are staged in LDS one batch at a time
// and every wave sums T(offset, q) U_source(q) over its target's entries in
// the batch, so each staged pattern is read from memory once per tile instead
// of once per target.  The sums stay in registers across batches.

// read-only index tables in the constant address space: loads at
// wave-uniform addresses become scalar loads
typedef const __attribute__((address_space(4))) int cint;
__device__ inline int ld_uniform(const int *p, int i) { return ((cint *)p)[i]; }

template <class T, int RW, int RB>
__global__ __launch_bounds__(TRANS_TMAX_MAX * WAVE) void k_translate_tiled(const TransArgs<T> a, int nrhs)
{
    constexpr int QW = WAVE / RW;
    constexpr int UNR = (sizeof(T) == 4 ? 16 : 8) / (RB > 2 ? 2 : 1);   // operator loads in flight
    constexpr int SRC = 2 * RB * WAVE;                                  // LDS elements per staged source
    extern __shared__ double trans_lds_raw[];
    cpx<T> *lds = reinterpret_cast<cpx<T> *>(trans_lds_raw);
    // every XCD takes an eighth of every level, coarse levels first (their
    // few, long workgroups then overlap the many short ones of the leaf
    // level), each eighth a contiguous range of tiles for the XCD's L2
    const int xcd = blockIdx.x % NXCD, pos = blockIdx.x / NXCD;
    if (pos >= a.nblocks) return;
    int l = 0;
    while (l + 1 < a.nlev && pos >= a.lv[l + 1].first) l++;
    const TransLevel<T> &L = a.lv[l];
    const int nblk = L.ntile * L.nqc, per = (nblk + NXCD - 1) / NXCD;
    const int lb = xcd * per + (pos - L.first);
    if (lb >= nblk) return;
    const int tile = lb % L.ntile, qc = lb / L.ntile;
    const int K = L.K;
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int nwave = blockDim.x / WAVE;
    const int qi = lane % QW, ri = lane / QW;
    const int q = qc * QW + qi;
    const int rbase = blockIdx.y * RW * RB + ri;   // this lane's right-hand sides: rbase + j RW, j < RB
    const bool qok = q < K;
    const cpx<T> *tq = L.trans + (qok ? q : K - 1);
    const cpx<T> *Uq = L.U + (qok ? q : K - 1);
    const int t0 = ld_uniform(L.tile_tgt, tile), nt = ld_uniform(L.tile_tgt, tile + 1) - t0;
    const int b0 = ld_uniform(L.tile_bat, tile), b1 = ld_uniform(L.tile_bat, tile + 1);
    cpx<T> a0[RB], a1[RB];
#pragma unroll
    for (int j = 0; j < RB; j++) a0[j] = a1[j] = mk<T>(0, 0);
    // stage: LDS row (source s, component c, register j) holds 64 lanes; wave
    // w copies rows w, w + nwave, ...; every load of a batch is issued before
    // the first store.  With several right-hand sides per lane (PIPE) the
    // loads of batch b + 1 are issued right after batch b is in LDS, so they
    // are in flight while batch b is summed; with one, the registers this
    // holds would cost more occupancy than the overlap gains.
    constexpr bool PIPE = RW == 4;
    const int S = 2 * nrhs * K;   // elements of one box's patterns
    cpx<T> st[TRANS_ROWS];
    // the batch's source boxes, lane i holding the i-th: one vector load per
    // batch, issued a batch ahead, instead of a dependent scalar load per
    // staged row
    auto batch_sources = [&](int b) {
        const int s0 = ld_uniform(L.bat_src, b), ns = ld_uniform(L.bat_src, b + 1) - s0;
        return lane < ns ? L.src[s0 + lane] : 0;
    };
    // lanes past the last sample or right-hand side stage a duplicate of a
    // valid element: a staged element is read only by the lane that staged
    // it, and the sums of those lanes are never stored
    auto stage_load = [&](int b, int srcv) {
        const int ns = ld_uniform(L.bat_src, b + 1) - ld_uniform(L.bat_src, b);
        // every row's source is taken from srcv before the first load, so
        // that no row waits for the loads of the rows before it
        int src[TRANS_ROWS];
#pragma unroll
        for (int i = 0; i < TRANS_ROWS; i++)
            src[i] = __builtin_amdgcn_readlane(srcv, ((wave + i * nwave) / (2 * RB)) & (WAVE - 1));
        // the row offsets are formed where they are used, not held in
        // registers across the batch loop: a uniform offset stays whole in
        // scalar registers, and with several right-hand sides per lane the
        // lane's base is taken afresh for every batch
        int rb = rbase;
        if constexpr (RW > 1) asm volatile("" : "+v"(rb));
#pragma unroll
        for (int i = 0; i < TRANS_ROWS; i++) {
            const int sc = wave + i * nwave;
            st[i] = mk<T>(0, 0);   // not carried over from the previous batch
            if (sc < 2 * RB * ns) {
                const int j = sc % RB, c = (sc / RB) & 1, rr = min(rb + j * RW, nrhs - 1);
                long long off = (long long)src[i] * S + (long long)(c * nrhs + rr) * K;
                if constexpr (RW == 1) asm volatile("" : "+s"(off));
                st[i] = Uq[off];
            }
        }
    };
    int srcv = b0 < b1 ? batch_sources(b0) : 0;
    if (PIPE && b0 < b1) stage_load(b0, srcv);
    for (int b = b0; b < b1; b++) {
        const int ns = ld_uniform(L.bat_src, b + 1) - ld_uniform(L.bat_src, b);
        if (!PIPE) {
            stage_load(b, srcv);
            if (b + 1 < b1) srcv = batch_sources(b + 1);   // in flight while this batch is summed
        }
        // this wave's entries of the batch (n <= ns <= 64), loaded before the
        // barriers so that their latency overlaps the staging (without PIPE;
        // with it the registers would cost occupancy)
        int n = 0, mine = 0;
        auto entries = [&]() {
            const int *rw = L.row + ld_uniform(L.bat_row, b);
            const int e0 = ld_uniform(rw, wave);
            n = ld_uniform(rw, wave + 1) - e0;
            mine = lane < n ? L.ent[e0 + lane] : 0;
        };
        if (!PIPE && wave < nt) entries();
        if (b > b0) __syncthreads();   // every wave is done with the previous batch
#pragma unroll
        for (int i = 0; i < TRANS_ROWS; i++) {
            const int sc = wave + i * nwave;
            if (sc < 2 * RB * ns) lds[sc * WAVE + lane] = st[i];
        }
        // with PIPE the next batch's sources are loaded here, where the
        // staged registers are free, and arrive during the barrier
        if (PIPE && b + 1 < b1) srcv = batch_sources(b + 1);
        __syncthreads();
        if (PIPE && b + 1 < b1) stage_load(b + 1, srcv);
        if (wave >= nt) continue;
        if (PIPE) entries();
        int e = 0;
        // entry = (operator element offset << 8) | staged source.  With four
        // right-hand sides per lane the batch's entries are decoded at once,
        // as byte offsets of the operator sample and of the staged source
        // (two vector instructions per batch instead of four scalar ones per
        // entry); with one right-hand side per lane that measured slower
        constexpr bool VDEC = RW == 4;
        const unsigned opb = ((unsigned)mine >> 8) * (unsigned)sizeof(cpx<T>);
        const unsigned ldb = (unsigned)(mine & 0xff) * (unsigned)(SRC * sizeof(cpx<T>));
        auto op_at = [&](int i) {
            if constexpr (VDEC)
                return *reinterpret_cast<const cpx<T> *>(reinterpret_cast<const char *>(tq) +
                                                         (unsigned)__builtin_amdgcn_readlane((int)opb, i));
            else
                return tq[(unsigned)__builtin_amdgcn_readlane(mine, i) >> 8];
        };
        auto src_at = [&](int i) {
            if constexpr (VDEC)
                return reinterpret_cast<const cpx<T> *>(reinterpret_cast<const char *>(lds + lane) +
                                                        (unsigned)__builtin_amdgcn_readlane((int)ldb, i));
            else
                return lds + (__builtin_amdgcn_readlane(mine, i) & 0xff) * SRC + lane;
        };
        for (; e + UNR <= n; e += UNR) {
            cpx<T> t[UNR];
#pragma unroll
            for (int u = 0; u < UNR; u++) t[u] = op_at(e + u);
            if constexpr (VDEC) __builtin_amdgcn_sched_barrier(0);   // every operator load issued before the sums
#pragma unroll
            for (int u = 0; u < UNR; u++) {
                const cpx<T> *p = src_at(e + u);
#pragma unroll
                for (int j = 0; j < RB; j++) {
                    fma_to(a0[j], t[u], p[j * WAVE]);
                    fma_to(a1[j], t[u], p[(RB + j) * WAVE]);
                }
            }
        }
        // one right-hand side per lane: the remaining n - e < UNR entries in
        // blocks of 8, 4, 2 and 1, each with all its operator loads issued
        // before its sums (a wave has about ten entries per batch: one by one,
        // every load latency would be exposed; padding to a full block costs
        // redundant loads).  With several right-hand sides per lane the
        // registers of the blocks cost more occupancy than they save.
        auto block = [&](auto width) {
            constexpr int NB = decltype(width)::value;
            cpx<T> t[NB];
#pragma unroll
            for (int u = 0; u < NB; u++) t[u] = op_at(e + u);
            if constexpr (VDEC) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < NB; u++) {
                const cpx<T> *p = src_at(e + u);
#pragma unroll
                for (int j = 0; j < RB; j++) {
                    fma_to(a0[j], t[u], p[j * WAVE]);
                    fma_to(a1[j], t[u], p[(RB + j) * WAVE]);
                }
            }
            e += NB;
        };
        if constexpr (RW == 1) {
            if (UNR > 8 && n - e >= 8) block(std::integral_constant<int, 8>());
            if (UNR > 4 && n - e >= 4) block(std::integral_constant<int, 4>());
            if (n - e >= 2) block(std::integral_constant<int, 2>());
            if (n - e >= 1) block(std::integral_constant<int, 1>());
        } else {
            for (; e < n; e++) {
                const cpx<T> t = op_at(e);
                const cpx<T> *p = src_at(e);
#pragma unroll
                for (int j = 0; j < RB; j++) {
                    fma_to(a0[j], t, p[j * WAVE]);
                    fma_to(a1[j], t, p[(RB + j) * WAVE]);
                }
            }
        }
    }
    if (wave < nt && qok) {
#pragma unroll
        for (int j = 0; j < RB; j++) {
            const int rr = rbase + j * RW;
            if (rr < nrhs) {
                L.V[pidx(t0 + wave, 0, rr, q, nrhs, K)] = a0[j];
                L.V[pidx(t0 + wave, 1, rr, q, nrhs, K)] = a1[j];
            }
        }
    }
}

// ------------------------------ disaggregation: shift + transposed phi stage
// mid_c = (A_phi^T W_P) [exp(-jk khat.(r_c - r_P)) V_P]
template <class T, int NR>
__global__ __launch_bounds__(256) void k_disagg_mid(int nchild, int mid_len, int Kp, const int *__restrict__ parent,
                                                    const int *__restrict__ oct, const cpx<T> *__restrict__ shift,
                                                    const int *__restrict__ st, const int *__restrict__ col,
                                                    const T *__restrict__ w, const cpx<T> *__restrict__ Vp,
                                                    cpx<T> *__restrict__ mid, int nrhs)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)nchild * mid_len) return;
    const int c = (int)(g / mid_len), row = (int)(g % mid_len);
    const int r0 = blockIdx.y * NR;
    const int P = parent[c];
    const cpx<T> *sh = shift + (long long)oct[c] * Kp;
    cpx<T> a0[NR], a1[NR];
#pragma unroll
    for (int rr = 0; rr < NR; rr++) a0[rr] = a1[rr] = mk<T>(0, 0);
    const int e1 = st[row + 1];
    int e = st[row];
    for (; e + 4 <= e1; e += 4) {
        int kp[4];
        cpx<T> f[4];
#pragma unroll
        for (int u = 0; u < 4; u++) kp[u] = col[e + u];
#pragma unroll
        for (int u = 0; u < 4; u++) f[u] = w[e + u] * conjg(sh[kp[u]]);
#pragma unroll
        for (int rr = 0; rr < NR; rr++) {
            if (NR > 1 && r0 + rr >= nrhs) continue;
            cpx<T> v0[4], v1[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                v0[u] = Vp[pidx(P, 0, r0 + rr, kp[u], nrhs, Kp)];
                v1[u] = Vp[pidx(P, 1, r0 + rr, kp[u], nrhs, Kp)];
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                fma_to(a0[rr], f[u], v0[u]);
                fma_to(a1[rr], f[u], v1[u]);
            }
        }
    }
    for (; e < e1; e++) {
        const int kp = col[e];
        const cpx<T> f = w[e] * conjg(sh[kp]);
#pragma unroll
        for (int rr = 0; rr < NR; rr++) {
            if (NR > 1 && r0 + rr >= nrhs) continue;
            fma_to(a0[rr], f, Vp[pidx(P, 0, r0 + rr, kp, nrhs, Kp)]);
            fma_to(a1[rr], f, Vp[pidx(P, 1, r0 + rr, kp, nrhs, Kp)]);
        }
    }
#pragma unroll
    for (int rr = 0; rr < NR; rr++) {
        if (NR > 1 && r0 + rr >= nrhs) continue;
        mid[pidx(c, 0, r0 + rr, row, nrhs, mid_len)] = a0[rr];
        mid[pidx(c, 1, r0 + rr, row, nrhs, mid_len)] = a1[rr];
    }
}

// ---------------------------------------------------------------- receive
// y1 += c0 sum_k w_k P_m(k) . V_b(k),  y2 += c0 sum_k w_k P_m(k) . (khat x V_b(k))
// with P = conj(R) for the EM pair and P = Q for the C block; c0 and the
// sphere weights are folded into wq.  One wave per RWG, lanes over samples.
// Receive for one right-hand side: wave per RWG row, lanes over samples,
// the row's pattern and the box's incoming pattern loaded for four chunks of
// 64 samples (two in double precision) before they are used.
template <class T, bool PERM>
__global__ __launch_bounds__(256) void k_receive1(int op, int N, int K, const int *__restrict__ leaf_of,
                                                  const cpx<T> *__restrict__ R, const cpx<T> *__restrict__ Q,
                                                  const T *__restrict__ wq, const cpx<T> *__restrict__ V,
                                                  cpx<T> *__restrict__ Y, cpx<T> *__restrict__ yu,
                                                  const int *__restrict__ perm)
{
    constexpr int CH = sizeof(T) == 4 ? 4 : 2;
    const int m = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    if (m >= N) return;
    const int b = leaf_of[m];
    const cpx<T> *pat = op == 1 ? R : Q;
    cpx<T> a1 = mk<T>(0, 0), a2 = a1;
    for (int q0 = lane; q0 < K; q0 += CH * WAVE) {
        cpx<T> Pt[CH], Pp[CH], Vt[CH], Vp[CH];
        T wk[CH];
#pragma unroll
        for (int c = 0; c < CH; c++) {
            const int q = min(q0 + c * WAVE, K - 1);
            load_pair(pat + ((long long)m * K + q) * 2, Pt[c], Pp[c]);
            Vt[c] = V[pidx(b, 0, 0, q, 1, K)];
            Vp[c] = V[pidx(b, 1, 0, q, 1, K)];
            wk[c] = q0 + c * WAVE < K ? wq[q] : T(0);    // samples past K contribute nothing
        }
#pragma unroll
        for (int c = 0; c < CH; c++) {
            cpx<T> pt = Pt[c], pp = Pp[c];
            if (op == 1) {
                pt = conjg(pt);
                pp = conjg(pp);
            }
            pt = wk[c] * pt;
            pp = wk[c] * pp;
            fma_to(a1, pt, Vt[c]);
            fma_to(a1, pp, Vp[c]);
            fma_to(a2, pp, Vt[c]);
            fms_to(a2, pt, Vp[c]);
        }
    }
    const cpx<T> s1 = wave_sum(a1), s2 = wave_sum(a2);
    if (lane == 0) {
        const cpx<T> r1 = Y[(long long)m * 2] + s1, r2 = Y[(long long)m * 2 + 1] + s2;
        if constexpr (PERM) {
            // the caller's vector in user order: J half, then M half
            const long long u = perm[m];
            yu[u] = r1;
            yu[N + u] = r2;
        } else {
            Y[(long long)m * 2] = r1;
            Y[(long long)m * 2 + 1] = r2;
        }
    }
}

template <class T, int NR>
__global__ __launch_bounds__(256) void k_receive(int op, int N, int K, const int *__restrict__ leaf_of,
                                                 const cpx<T> *__restrict__ R, const cpx<T> *__restrict__ Q,
                                                 const T *__restrict__ wq, const cpx<T> *__restrict__ V,
                                                 cpx<T> *__restrict__ Y, int nrhs)
{
    const int m = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    if (m >= N) return;
    const int r0 = blockIdx.y * NR;
    const int b = leaf_of[m];
    cpx<T> a1[NR], a2[NR];
#pragma unroll
    for (int rr = 0; rr < NR; rr++) a1[rr] = a2[rr] = mk<T>(0, 0);
    const cpx<T> *pat = op == 1 ? R : Q;
    for (int q = lane; q < K; q += WAVE) {
        cpx<T> Pt = pat[((long long)m * K + q) * 2], Pp = pat[((long long)m * K + q) * 2 + 1];
        if (op == 1) {
            Pt = conjg(Pt);
            Pp = conjg(Pp);
        }
        const T wk = wq[q];
        Pt = wk * Pt;
        Pp = wk * Pp;
#pragma unroll
        for (int rr = 0; rr < NR; rr++) {
            if (NR > 1 && r0 + rr >= nrhs) continue;
            const cpx<T> Vt = V[pidx(b, 0, r0 + rr, q, nrhs, K)], Vp = V[pidx(b, 1, r0 + rr, q, nrhs, K)];
            fma_to(a1[rr], Pt, Vt);
            fma_to(a1[rr], Pp, Vp);
            fma_to(a2[rr], Pp, Vt);
            fms_to(a2[rr], Pt, Vp);
        }
    }
#pragma unroll
    for (int rr = 0; rr < NR; rr++) {
        const cpx<T> s1 = wave_sum(a1[rr]), s2 = wave_sum(a2[rr]);
        if (lane == 0 && (NR == 1 || r0 + rr < nrhs)) {
            cpx<T> &y1 = Y[((long long)m * 2) * nrhs + r0 + rr];
            cpx<T> &y2 = Y[((long long)m * 2 + 1) * nrhs + r0 + rr];
            y1 = y1 + s1;
            y2 = y2 + s2;
        }
    }
}

// fill with zeros (used instead of a memset so the sequence stays capturable)
template <class T>
__global__ void k_zero(cpx<T> *__restrict__ p, long long n)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) p[g] = mk<T>(0, 0);
}

// ---------------------------------------------------------------- launchers
static inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <class T>
void launch_perm_in(const cpx<T> *x, long long ldx, cpx<T> *X, const int *perm, const int *iperm, int N, int nrhs,
                    hipStream_t s)
{
    if (nrhs >= 4) {
        const dim3 grid((N + PT_U - 1) / PT_U, 2, (nrhs + PT_R - 1) / PT_R);
        hipLaunchKernelGGL((k_perm_tile<T, true>), grid, dim3(256), 0, s, x, ldx, X, iperm, N, nrhs);
        return;
    }
    long long n = (long long)N * 2 * nrhs;
    hipLaunchKernelGGL(k_perm_in<T>, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, ldx, X, perm, N, nrhs);
}
template <class T>
void launch_perm_out(const cpx<T> *Y, cpx<T> *y, long long ldy, const int *iperm, int N, int nrhs, hipStream_t s)
{
    if (nrhs >= 4) {
        const dim3 grid((N + PT_U - 1) / PT_U, 2, (nrhs + PT_R - 1) / PT_R);
        hipLaunchKernelGGL((k_perm_tile<T, false>), grid, dim3(256), 0, s, Y, ldy, y, iperm, N, nrhs);
        return;
    }
    long long n = (long long)N * 2 * nrhs;
    hipLaunchKernelGGL(k_perm_out<T>, dim3(blocks_for(n, 256)), dim3(256), 0, s, Y, y, ldy, iperm, N, nrhs);
}

#define DISPATCH_NR(nrhs, KERNEL_CALL)            \
    do {                                          \
        int nr_ = nr_for(nrhs);                   \
        if (nr_ == 1) { constexpr int NR = 1; KERNEL_CALL; } \
        else if (nr_ == 4) { constexpr int NR = 4; KERNEL_CALL; } \
        else { constexpr int NR = 16; KERNEL_CALL; } \
    } while (0)

template <class T>
void launch_near_tile(int nitem, const int2 *items, const int *box_start, const int *col_off, const int *cols,
                      const long long *val_off, const cpx<T> *vals, const int *id_start, const int *id_col,
                      const T *id_w, const cpx<T> *X, cpx<T> *Y, hipStream_t s)
{
    if (nitem <= 0) return;
    // rows per wave: four in single and two in double precision (a wave per
    // 8-RWG item holds registers that cut the occupancy, most in double)
    constexpr int RWV = sizeof(T) == 4 ? 4 : 2;
    hipLaunchKernelGGL((k_near_tile<T, RWV>), dim3(xcd_grid(((long long)nitem * (8 / RWV) + 3) / 4)), dim3(256), 0, s,
                       nitem, items, box_start, col_off, cols, val_off, vals, id_start, id_col, id_w, X, Y);
}

template <class T>
void launch_near(int N, const int *leaf_of, const int *box_start, const int *near_start, const int *near_box,
                 const long long *val_off, const cpx<T> *vals, const int *id_start, const int *id_col, const T *id_w,
                 const cpx<T> *X, cpx<T> *Y, int nrhs, hipStream_t s)
{
    if (nrhs >= 16) {
        dim3 grid(xcd_grid((N + 3) / 4), (nrhs + WAVE - 1) / WAVE);
        hipLaunchKernelGGL(k_near_rhs<T>, grid, dim3(256), 0, s, N, leaf_of, box_start, near_start, near_box,
                           val_off, vals, id_start, id_col, id_w, X, Y, nrhs);
        return;
    }
    DISPATCH_NR(nrhs, {
        dim3 grid(xcd_grid((N + 3) / 4), (nrhs + NR - 1) / NR);
        hipLaunchKernelGGL((k_near<T, NR>), grid, dim3(256), 0, s, N, leaf_of, box_start, near_start, near_box,
                           val_off, vals, id_start, id_col, id_w, X, Y, nrhs);
    });
}

template <class T>
void launch_radiate(int op, int nbox, int K, const int *box_start, const cpx<T> *R, const cpx<T> *X, cpx<T> *U,
                    int nrhs, hipStream_t s)
{
    if (nrhs == 1) {
        const int nqc = (K + WAVE - 1) / WAVE;
        const long long nw = (long long)nbox * nqc;
        if (nw > 0)
            hipLaunchKernelGGL((k_radiate1<T, false>), dim3(xcd_grid((nw + 3) / 4)), dim3(256), 0, s, op, nbox, K, nqc,
                               box_start, R, X, U, nullptr, nullptr, 0, nullptr);
        return;
    }
    DISPATCH_NR(nrhs, {
        dim3 grid(blocks_for((long long)nbox * K, 256), (nrhs + NR - 1) / NR);
        hipLaunchKernelGGL((k_radiate<T, NR>), grid, dim3(256), 0, s, op, nbox, K, box_start, R, X, U, nrhs);
    });
}

template <class T>
void launch_interp(int nbox, int rows, int in_len, const int *st, const int *col, const T *w, const cpx<T> *in,
                   cpx<T> *out, int nrhs, bool accumulate, hipStream_t s)
{
    DISPATCH_NR(nrhs, {
        dim3 grid(blocks_for((long long)nbox * rows, 256), (nrhs + NR - 1) / NR);
        hipLaunchKernelGGL((k_interp<T, NR>), grid, dim3(256), 0, s, nbox, rows, in_len, st, col, w, in, out, nrhs,
                           accumulate ? 1 : 0);
    });
}

template <class T>
bool launch_interp_fixed(int taps, int nbox, int rows, int in_len, const int *col, const T *w, const cpx<T> *in,
                         cpx<T> *out, int nrhs, hipStream_t s)
{
    if (taps != 6 && taps != 8 && taps != 10) return false;
    DISPATCH_NR(nrhs, {
        dim3 grid(xcd_grid(blocks_for((long long)nbox * rows, 256)), (nrhs + NR - 1) / NR);
        if (taps == 6)
            hipLaunchKernelGGL((k_interp_fixed<T, NR, 6>), grid, dim3(256), 0, s, nbox, rows, in_len, col, w, in, out,
                               nrhs);
        else if (taps == 8)
            hipLaunchKernelGGL((k_interp_fixed<T, NR, 8>), grid, dim3(256), 0, s, nbox, rows, in_len, col, w, in, out,
                               nrhs);
        else
            hipLaunchKernelGGL((k_interp_fixed<T, NR, 10>), grid, dim3(256), 0, s, nbox, rows, in_len, col, w, in,
                               out, nrhs);
    });
    return true;
}

template <class T>
bool launch_agg_phi_fixed(int taps, int nparent, int Kp, int mid_len, const int *child_start, const int *child_oct,
                          const cpx<T> *shift, const int *col, const T *w, const cpx<T> *mid, cpx<T> *Up, int nrhs,
                          hipStream_t s)
{
    if (taps != 6 && taps != 8 && taps != 10) return false;
    DISPATCH_NR(nrhs, {
        dim3 grid(xcd_grid(blocks_for((long long)nparent * Kp, 256)), (nrhs + NR - 1) / NR);
        if (taps == 6)
            hipLaunchKernelGGL((k_agg_phi_fixed<T, NR, 6>), grid, dim3(256), 0, s, nparent, Kp, mid_len, child_start,
                               child_oct, shift, col, w, mid, Up, nrhs);
        else if (taps == 8)
            hipLaunchKernelGGL((k_agg_phi_fixed<T, NR, 8>), grid, dim3(256), 0, s, nparent, Kp, mid_len, child_start,
                               child_oct, shift, col, w, mid, Up, nrhs);
        else
            hipLaunchKernelGGL((k_agg_phi_fixed<T, NR, 10>), grid, dim3(256), 0, s, nparent, Kp, mid_len,
                               child_start, child_oct, shift, col, w, mid, Up, nrhs);
    });
    return true;
}

template <class T>
void launch_agg_phi(int nparent, int Kp, int mid_len, const int *child_start, const int *child_oct,
                    const cpx<T> *shift, const int *st, const int *col, const T *w, const cpx<T> *mid, cpx<T> *Up,
                    int nrhs, hipStream_t s)
{
    DISPATCH_NR(nrhs, {
        dim3 grid(blocks_for((long long)nparent * Kp, 256), (nrhs + NR - 1) / NR);
        hipLaunchKernelGGL((k_agg_phi<T, NR>), grid, dim3(256), 0, s, nparent, Kp, mid_len, child_start, child_oct,
                           shift, st, col, w, mid, Up, nrhs);
    });
}


template <class T>
bool launch_translate_tiled(const TransArgs<T> &args, int nrhs, hipStream_t s)
{
    if (!trans_shape_ok(args.tmax, args.smax, args.rb)) return false;
    if (args.nlev <= 0 || nrhs <= 0) return true;
    // right-hand sides per lane only when four of them span the lanes (the
    // tiles do not depend on it, and one per lane needs less LDS)
    const int rw = trans_rw(nrhs), qw = WAVE / rw, rb = rw == 4 ? args.rb : 1;
    TransArgs<T> a = args;
    a.rb = rb;
    // nblocks: workgroups per XCD over all levels; first: a level's first
    // position in that per-XCD sequence
    a.nblocks = 0;
    for (int l = 0; l < a.nlev; l++) {
        a.lv[l].nqc = (a.lv[l].K + qw - 1) / qw;
        a.lv[l].first = a.nblocks;
        a.nblocks += (a.lv[l].ntile * a.lv[l].nqc + NXCD - 1) / NXCD;
    }
    if (a.nblocks <= 0) return true;
    const size_t lds = trans_lds_bytes<T>(a.smax, rb);
    const dim3 grid((unsigned)a.nblocks * NXCD, (nrhs + rw * rb - 1) / (rw * rb)), block(a.tmax * WAVE);
    if (rw == 4 && rb == 4)
        hipLaunchKernelGGL((k_translate_tiled<T, 4, 4>), grid, block, lds, s, a, nrhs);
    else if (rw == 4 && rb == 2)
        hipLaunchKernelGGL((k_translate_tiled<T, 4, 2>), grid, block, lds, s, a, nrhs);
    else if (rw == 4)
        hipLaunchKernelGGL((k_translate_tiled<T, 4, 1>), grid, block, lds, s, a, nrhs);
    else if (rw == 2)
        hipLaunchKernelGGL((k_translate_tiled<T, 2, 1>), grid, block, lds, s, a, nrhs);
    else
        hipLaunchKernelGGL((k_translate_tiled<T, 1, 1>), grid, block, lds, s, a, nrhs);
    return true;
}

template <class T>
void launch_disagg_mid(int nchild, int mid_len, int Kp, const int *parent, const int *oct, const cpx<T> *shift,
                       const int *st, const int *col, const T *w, const cpx<T> *Vp, cpx<T> *mid, int nrhs,
                       hipStream_t s)
{
    DISPATCH_NR(nrhs, {
        dim3 grid(blocks_for((long long)nchild * mid_len, 256), (nrhs + NR - 1) / NR);
        hipLaunchKernelGGL((k_disagg_mid<T, NR>), grid, dim3(256), 0, s, nchild, mid_len, Kp, parent, oct, shift, st,
                           col, w, Vp, mid, nrhs);
    });
}

template <class T>
void launch_zero(cpx<T> *p, long long n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_zero<T>, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n);
}

template <class T>
void launch_receive(int op, int N, int K, const int *leaf_of, const cpx<T> *R, const cpx<T> *Q, const T *wq,
                    const cpx<T> *V, cpx<T> *Y, int nrhs, hipStream_t s)
{
    if (nrhs == 1) {
        if (N > 0)
            hipLaunchKernelGGL((k_receive1<T, false>), dim3(blocks_for(N, 4)), dim3(256), 0, s, op, N, K, leaf_of, R,
                               Q, wq, V, Y, nullptr, nullptr);
        return;
    }
    DISPATCH_NR(nrhs, {
        dim3 grid(blocks_for(N, 4), (nrhs + NR - 1) / NR);
        hipLaunchKernelGGL((k_receive<T, NR>), grid, dim3(256), 0, s, op, N, K, leaf_of, R, Q, wq, V, Y, nrhs);
    });
}

template <class T>
void launch_radiate1_user(int op, int nbox, int K, const int *box_start, const cpx<T> *R, const cpx<T> *x,
                          const int *perm, int N, cpx<T> *X, cpx<T> *U, hipStream_t s)
{
    const int nqc = (K + WAVE - 1) / WAVE;
    const long long nw = (long long)nbox * nqc;
    if (nw > 0)
        hipLaunchKernelGGL((k_radiate1<T, true>), dim3(xcd_grid((nw + 3) / 4)), dim3(256), 0, s, op, nbox, K, nqc,
                           box_start, R, (const cpx<T> *)nullptr, U, x, perm, N, X);
}

template <class T>
void launch_receive1_user(int op, int N, int K, const int *leaf_of, const cpx<T> *R, const cpx<T> *Q, const T *wq,
                          const cpx<T> *V, const cpx<T> *Y, cpx<T> *y, const int *perm, hipStream_t s)
{
    if (N > 0)
        hipLaunchKernelGGL((k_receive1<T, true>), dim3(blocks_for(N, 4)), dim3(256), 0, s, op, N, K, leaf_of, R, Q,
                           wq, V, const_cast<cpx<T> *>(Y), y, perm);
}

#define INSTANTIATE(T)                                                                                              \
    template void launch_radiate1_user<T>(int, int, int, const int *, const cpx<T> *, const cpx<T> *, const int *, \
                                          int, cpx<T> *, cpx<T> *, hipStream_t);                                  \
    template void launch_receive1_user<T>(int, int, int, const int *, const cpx<T> *, const cpx<T> *, const T *,  \
                                          const cpx<T> *, const cpx<T> *, cpx<T> *, const int *, hipStream_t);    \
    template void launch_perm_in<T>(const cpx<T> *, long long, cpx<T> *, const int *, const int *, int, int,     \
                                    hipStream_t);                                                                 \
    template void launch_perm_out<T>(const cpx<T> *, cpx<T> *, long long, const int *, int, int, hipStream_t);    \
    template void launch_near_tile<T>(int, const int2 *, const int *, const int *, const int *, const long long *, \
                                      const cpx<T> *, const int *, const int *, const T *, const cpx<T> *, cpx<T> *, \
                                      hipStream_t);                                                               \
    template void launch_near<T>(int, const int *, const int *, const int *, const int *, const long long *,     \
                                 const cpx<T> *, const int *, const int *, const T *, const cpx<T> *, cpx<T> *, \
                                 int, hipStream_t);                                                               \
    template bool launch_interp_fixed<T>(int, int, int, int, const int *, const T *, const cpx<T> *, cpx<T> *,    \
                                         int, hipStream_t);                                                       \
    template bool launch_agg_phi_fixed<T>(int, int, int, int, const int *, const int *, const cpx<T> *,          \
                                          const int *, const T *, const cpx<T> *, cpx<T> *, int, hipStream_t);   \
    template void launch_radiate<T>(int, int, int, const int *, const cpx<T> *, const cpx<T> *, cpx<T> *, int,   \
                                    hipStream_t);                                                                 \
    template void launch_interp<T>(int, int, int, const int *, const int *, const T *, const cpx<T> *, cpx<T> *, \
                                   int, bool, hipStream_t);                                                       \
    template void launch_agg_phi<T>(int, int, int, const int *, const int *, const cpx<T> *, const int *,        \
                                    const int *, const T *, const cpx<T> *, cpx<T> *, int, hipStream_t);          \
    template bool launch_translate_tiled<T>(const TransArgs<T> &, int, hipStream_t);                             \
    template void launch_disagg_mid<T>(int, int, int, const int *, const int *, const cpx<T> *, const int *,     \
                                       const int *, const T *, const cpx<T> *, cpx<T> *, int, hipStream_t);       \
    template void launch_zero<T>(cpx<T> *, long long, hipStream_t);                                               \
    template void launch_receive<T>(int, int, int, const int *, const cpx<T> *, const cpx<T> *, const T *,       \
                                    const cpx<T> *, cpx<T> *, int, hipStream_t);

INSTANTIATE(double)
INSTANTIATE(float)

}  // namespace mlfma
