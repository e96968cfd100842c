// Sparse approximate inverse of the BI block's near field (build and apply).
// The paper preconditions its outer GMRES with an SAI built from C alone
// (Sec. III, dielectric-plate example); the Frobenius-norm definition of the
// SAI literature it cites is used over the near field (see sai.hpp).
#include "sai.hpp"

namespace mlfma {
namespace {

constexpr int SAI_ROWS = 16;                          // RWG rows staged per pass
constexpr int SAI_TRI = SAI_D * (SAI_D + 1) / 2;      // packed lower triangle of G

__device__ inline int tri_idx(int i, int j) { return i * (i + 1) / 2 + j; }   // j <= i

// One workgroup (4 waves) per RWG u.  Pass over every leaf box B that holds
// rows of C_near touching the pattern: stage the rows of B (SAI_ROWS RWGs at a
// time, both halves) restricted to the pattern's unknowns in LDS, then every
// thread adds their contribution to its 16 entries of G = A^H A (thread t owns
// row t % 64 and columns 16 (t / 64) .. + 15).  The right-hand sides A^H e of
// the two columns (u, J) and (u, M) are the conjugated rows of u itself.
// Then G is written to LDS (packed lower triangle), factored by Cholesky and
// two waves solve for the two columns, one lane per unknown.
__global__ __launch_bounds__(256) void k_sai_build(int u0, const int *__restrict__ pat_start,
                                                   const int *__restrict__ pat, const int *__restrict__ rb_start,
                                                   const int *__restrict__ rb, const int *__restrict__ leaf_of,
                                                   const int *__restrict__ box_start, const int *__restrict__ near_start,
                                                   const int *__restrict__ near_box,
                                                   const long long *__restrict__ val_off,
                                                   const cpx<double> *__restrict__ vals,
                                                   const int *__restrict__ id_start, const int *__restrict__ id_col,
                                                   const double *__restrict__ id_w, cpx<double> *__restrict__ M,
                                                   int *__restrict__ status)
{
    constexpr int STAGE = 2 * SAI_ROWS * SAI_D;
    constexpr int BUF = STAGE > SAI_TRI ? STAGE : SAI_TRI;
    __shared__ cpx<double> buf[BUF];              // staged rows, later the packed G
    __shared__ cpx<double> rhs[2][SAI_D];
    __shared__ int sp[SAI_MAXP], sbox[SAI_MAXP], colpos[SAI_MAXP];
    __shared__ int adj_box[27], adj_pre[28];
    __shared__ int bad;
    const int u = u0 + (int)blockIdx.x, tid = threadIdx.x;
    const int p0 = pat_start[u], np = pat_start[u + 1] - p0, D = 2 * np;
    if (tid < np) {
        sp[tid] = pat[p0 + tid];
        sbox[tid] = leaf_of[sp[tid]];
    }
    if (tid < 2 * SAI_D) rhs[tid / SAI_D][tid % SAI_D] = mk<double>(0, 0);
    if (tid == 0) bad = 0;
    const int a = tid & 63, g = tid >> 6;
    cpx<double> acc[16];
#pragma unroll
    for (int j = 0; j < 16; j++) acc[j] = mk<double>(0, 0);
    __syncthreads();
    for (int e = rb_start[u]; e < rb_start[u + 1]; e++) {
        const int B = rb[e];
        const int nadj = near_start[B + 1] - near_start[B];
        if (tid == 0) {
            int run = 0;
            for (int l = 0; l < nadj; l++) {
                const int nb = near_box[near_start[B] + l];
                adj_box[l] = nb;
                adj_pre[l] = run;
                run += box_start[nb + 1] - box_start[nb];
            }
            adj_pre[nadj] = run;
        }
        __syncthreads();
        if (tid < np) {
            int pos = -1;
            for (int l = 0; l < nadj; l++)
                if (adj_box[l] == sbox[tid]) pos = adj_pre[l] + (sp[tid] - box_start[sbox[tid]]);
            colpos[tid] = pos;
        }
        __syncthreads();
        const int ncols = adj_pre[nadj];
        const int r0 = box_start[B], r1 = box_start[B + 1];
        for (int c0 = r0; c0 < r1; c0 += SAI_ROWS) {
            const int nr = min(SAI_ROWS, r1 - c0);
            for (int idx = tid; idx < SAI_ROWS * SAI_MAXP; idx += 256) {
                const int ri = idx / SAI_MAXP, pc = idx % SAI_MAXP;
                cpx<double> jj = mk<double>(0, 0), jm = jj, mj = jj, mm = jj;
                if (ri < nr && pc < np && colpos[pc] >= 0) {
                    const int i = c0 + ri;
                    const cpx<double> *v = vals + 2 * (val_off[B] + (long long)(i - r0) * ncols + colpos[pc]);
                    const cpx<double> A = v[0], Bv = v[1];
                    double gr = 0, gx = 0;
                    if (id_start)
                        for (int q = id_start[i]; q < id_start[i + 1]; q++)
                            if (id_col[q] == sp[pc]) {
                                gr = id_w[2 * q];
                                gx = id_w[2 * q + 1];
                            }
                    // [[A + gram, -B + gx / 2], [B, A + gram / 2]] (op EM: no Gram terms)
                    jj = mk<double>(A.re + gr, A.im);
                    jm = mk<double>(-Bv.re + 0.5 * gx, -Bv.im);
                    mj = Bv;
                    mm = mk<double>(A.re + 0.5 * gr, A.im);
                }
                buf[(2 * ri) * SAI_D + 2 * pc] = jj;
                buf[(2 * ri) * SAI_D + 2 * pc + 1] = jm;
                buf[(2 * ri + 1) * SAI_D + 2 * pc] = mj;
                buf[(2 * ri + 1) * SAI_D + 2 * pc + 1] = mm;
            }
            __syncthreads();
            if (u >= c0 && u < c0 + nr && tid < 2 * SAI_D) {
                const int h = tid / SAI_D, c = tid % SAI_D;
                rhs[h][c] = conjg(buf[(2 * (u - c0) + h) * SAI_D + c]);
            }
            for (int r = 0; r < 2 * nr; r++) {
                const cpx<double> av = conjg(buf[r * SAI_D + a]);
#pragma unroll
                for (int j = 0; j < 16; j++) fma_to(acc[j], av, buf[r * SAI_D + g * 16 + j]);
            }
            __syncthreads();
        }
    }
    // packed lower triangle of G
#pragma unroll
    for (int j = 0; j < 16; j++) {
        const int b = g * 16 + j;
        if (b <= a) buf[tri_idx(a, b)] = acc[j];
    }
    __syncthreads();
    // Cholesky G = L L^H in place
    for (int k = 0; k < D; k++) {
        if (tid == 0) {
            double d = buf[tri_idx(k, k)].re;
            if (!(d > 0)) {
                bad = 1;
                d = 1;
            }
            buf[tri_idx(k, k)] = mk<double>(sqrt(d), 0);
        }
        __syncthreads();
        const double inv = 1.0 / buf[tri_idx(k, k)].re;
        if (tid > k && tid < D) {
            const cpx<double> v = buf[tri_idx(tid, k)];
            buf[tri_idx(tid, k)] = mk<double>(v.re * inv, v.im * inv);
        }
        __syncthreads();
        const int m = D - k - 1;
        for (int idx = tid; idx < m * m; idx += 256) {
            const int i = k + 1 + idx / m, j = k + 1 + idx % m;
            if (j <= i) fms_to(buf[tri_idx(i, j)], buf[tri_idx(i, k)], conjg(buf[tri_idx(j, k)]));
        }
        __syncthreads();
    }
    if (tid < 128) {
        // wave h solves L L^H m = rhs[h]; lane l holds unknown l
        const int h = tid >> 6, l = tid & 63;
        cpx<double> y = l < D ? rhs[h][l] : mk<double>(0, 0);
        for (int k = 0; k < D; k++) {
            const double dk = buf[tri_idx(k, k)].re;
            const cpx<double> yk = mk<double>(__shfl(y.re, k) / dk, __shfl(y.im, k) / dk);
            if (l == k) y = yk;
            else if (l > k && l < D) fms_to(y, buf[tri_idx(l, k)], yk);
        }
        for (int k = D - 1; k >= 0; k--) {
            const double dk = buf[tri_idx(k, k)].re;
            const cpx<double> xk = mk<double>(__shfl(y.re, k) / dk, __shfl(y.im, k) / dk);
            if (l == k) y = xk;
            else if (l < k) fms_to(y, conjg(buf[tri_idx(k, l)]), xk);
        }
        M[((long long)u * 2 + h) * SAI_D + l] = l < D ? y : mk<double>(0, 0);
    }
    if (tid == 0 && bad) status[0] = 1;
}

// y = M x, thread per (row RWG p, right-hand side r), p fastest.
template <class T>
__global__ __launch_bounds__(256) void k_sai_apply(int N, int nrhs, const int *__restrict__ row_start,
                                                   const int *__restrict__ ent_col, const int *__restrict__ ent_val,
                                                   const cpx<T> *__restrict__ M, const cpx<T> *__restrict__ x,
                                                   long long ldx, cpx<T> *__restrict__ y, long long ldy)
{
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)N * nrhs) return;
    const int p = (int)(t % N), r = (int)(t / N);
    const cpx<T> *xr = x + (long long)r * ldx;
    cpx<T> sJ = mk<T>(0, 0), sM = sJ;
    for (int e = row_start[p]; e < row_start[p + 1]; e++) {
        const int n = ent_col[e];
        const cpx<T> *m = M + ent_val[e];
        const cpx<T> xJ = xr[n], xM = xr[N + n];
        fma_to(sJ, m[0], xJ);
        fma_to(sJ, m[SAI_D], xM);
        fma_to(sM, m[1], xJ);
        fma_to(sM, m[SAI_D + 1], xM);
    }
    y[(long long)r * ldy + p] = sJ;
    y[(long long)r * ldy + N + p] = sM;
}

}  // namespace

void launch_sai_build(int u0, int count, const int *pat_start, const int *pat, const int *rb_start, const int *rb,
                      const int *leaf_of, const int *box_start, const int *near_start, const int *near_box,
                      const long long *val_off, const cpx<double> *vals, const int *id_start, const int *id_col,
                      const double *id_w, cpx<double> *M, int *status, hipStream_t s)
{
    if (count > 0)
        hipLaunchKernelGGL(k_sai_build, dim3(count), dim3(256), 0, s, u0, pat_start, pat, rb_start, rb, leaf_of,
                           box_start, near_start, near_box, val_off, vals, id_start, id_col, id_w, M, status);
}

template <class T>
void launch_sai_apply(int N, int nrhs, const int *row_start, const int *ent_col, const int *ent_val,
                      const cpx<T> *M, const cpx<T> *x, long long ldx, cpx<T> *y, long long ldy, hipStream_t s)
{
    const long long n = (long long)N * nrhs;
    if (n > 0)
        hipLaunchKernelGGL(k_sai_apply<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, nrhs, row_start,
                           ent_col, ent_val, M, x, ldx, y, ldy);
}

template void launch_sai_apply<float>(int, int, const int *, const int *, const int *, const cpx<float> *,
                                      const cpx<float> *, long long, cpx<float> *, long long, hipStream_t);
template void launch_sai_apply<double>(int, int, const int *, const int *, const int *, const cpx<double> *,
                                       const cpx<double> *, long long, cpx<double> *, long long, hipStream_t);

}  // namespace mlfma
