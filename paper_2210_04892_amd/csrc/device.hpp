// Device-side types and kernel launchers shared by the HIP sources.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace mlfma {

template <class T>
struct alignas(2 * sizeof(T)) cpx {
    T re, im;
};

template <class T>
__host__ __device__ inline cpx<T> mk(T r, T i) { return cpx<T>{r, i}; }
template <class T>
__host__ __device__ inline cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T>
__host__ __device__ inline cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T>
__host__ __device__ inline cpx<T> operator*(cpx<T> a, cpx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T>
__host__ __device__ inline cpx<T> operator*(T s, cpx<T> a) { return {s * a.re, s * a.im}; }
template <class T>
__host__ __device__ inline cpx<T> conjg(cpx<T> a) { return {a.re, -a.im}; }
// fused multiply-add a b + c, rounded once
template <class T>
__host__ __device__ inline T fmad(T a, T b, T c);
template <>
__host__ __device__ inline float fmad<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__host__ __device__ inline double fmad<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// p[0], p[1] with one 16-byte load in single precision (p must be 16-byte
// aligned there: an even index into a buffer from the allocator)
__device__ inline void load_pair(const cpx<float> *p, cpx<float> &a, cpx<float> &b)
{
    const float4 v = *reinterpret_cast<const float4 *>(p);
    a = {v.x, v.y};
    b = {v.z, v.w};
}
__device__ inline void load_pair(const cpx<double> *p, cpx<double> &a, cpx<double> &b)
{
    a = p[0];
    b = p[1];
}
// the same for data read once (non-temporal: streamed past the caches)
typedef float nt_f4 __attribute__((ext_vector_type(4)));
__device__ inline void load_pair_once(const cpx<float> *p, cpx<float> &a, cpx<float> &b)
{
    const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(p));
    a = {v.x, v.y};
    b = {v.z, v.w};
}
// (double pairs: plain loads measured faster)
__device__ inline void load_pair_once(const cpx<double> *p, cpx<double> &a, cpx<double> &b) { load_pair(p, a, b); }

// acc += a b (four fused multiply-adds)
template <class T>
__host__ __device__ inline void fma_to(cpx<T> &acc, cpx<T> a, cpx<T> b)
{
    acc.re = fmad(a.re, b.re, acc.re);
    acc.re = fmad(-a.im, b.im, acc.re);
    acc.im = fmad(a.re, b.im, acc.im);
    acc.im = fmad(a.im, b.re, acc.im);
}
// acc -= a b
template <class T>
__host__ __device__ inline void fms_to(cpx<T> &acc, cpx<T> a, cpx<T> b)
{
    acc.re = fmad(-a.re, b.re, acc.re);
    acc.re = fmad(a.im, b.im, acc.re);
    acc.im = fmad(-a.re, b.im, acc.im);
    acc.im = fmad(-a.im, b.re, acc.im);
}
// acc += s x for real s
template <class T>
__host__ __device__ inline void axpy_to(cpx<T> &acc, T s, cpx<T> x)
{
    acc.re = fmad(s, x.re, acc.re);
    acc.im = fmad(s, x.im, acc.im);
}

// Launchers of the hot path (matvec.hip).  X, Y internal vectors
// [rwg][half][rhs]; U, V patterns [box][sample][component][rhs].
template <class T>
void launch_perm_in(const cpx<T> *x, long long ldx, cpx<T> *X, const int *perm, const int *iperm, int N, int nrhs,
                    hipStream_t s);
template <class T>
void launch_perm_out(const cpx<T> *Y, cpx<T> *y, long long ldy, const int *iperm, int N, int nrhs, hipStream_t s);
template <class T>
void launch_near(int N, const int *leaf_of, const int *box_start, const int *near_start, const int *near_box,
                 const long long *val_off, const cpx<T> *vals, const int *id_start, const int *id_col, const T *id_w,
                 const cpx<T> *X, cpx<T> *Y, int nrhs, hipStream_t s);
// near field, one right-hand side: wave per (leaf box, tile of 8 RWGs) work
// item, columns of the box from cols[col_off[b] ..]
template <class T>
void launch_near_tile(int nitem, const int2 *items, const int *box_start, const int *col_off, const int *cols,
                      const long long *val_off, const cpx<T> *vals, const int *id_start, const int *id_col,
                      const T *id_w, const cpx<T> *X, cpx<T> *Y, hipStream_t s);
template <class T>
void launch_radiate(int op, int nbox, int K, const int *box_start, const cpx<T> *R, const cpx<T> *X, cpx<T> *U,
                    int nrhs, hipStream_t s);
template <class T>
void launch_interp(int nbox, int rows, int in_len, const int *st, const int *col, const T *w, const cpx<T> *in,
                   cpx<T> *out, int nrhs, bool accumulate, hipStream_t s);
// fixed-size forward stencils (taps = interpolation order 6, 8 or 10);
// return false when the order has no fixed-size kernel
template <class T>
bool launch_interp_fixed(int taps, int nbox, int rows, int in_len, const int *col, const T *w, const cpx<T> *in,
                         cpx<T> *out, int nrhs, hipStream_t s);
template <class T>
bool launch_agg_phi_fixed(int taps, int nparent, int Kp, int mid_len, const int *child_start, const int *child_oct,
                          const cpx<T> *shift, const int *col, const T *w, const cpx<T> *mid, cpx<T> *Up, int nrhs,
                          hipStream_t s);
template <class T>
void launch_agg_phi(int nparent, int Kp, int mid_len, const int *child_start, const int *child_oct,
                    const cpx<T> *shift, const int *st, const int *col, const T *w, const cpx<T> *mid, cpx<T> *Up,
                    int nrhs, hipStream_t s);
// Tiled translation of every level in one launch.  Per level: the tile
// tables of build_translation_tiles (device copies), the level's translation
// operators (343 offsets x K samples) and its outgoing/incoming patterns.
constexpr int TRANS_MAXLEV = 20;   // the octree has at most 20 levels
// Tile shape of the translation: tmax targets per tile (= waves per
// workgroup, at most TRANS_TMAX_MAX), smax sources per LDS batch and rb
// right-hand sides per lane (1, 2 or 4; above 1 only with four right-hand
// sides across the lanes of a wave).  A target's entries in one batch are
// fetched by the lanes of one wave, so smax <= 64, and each wave stages at
// most TRANS_ROWS rows of 64 lanes, so 2 smax rb <= TRANS_ROWS tmax.
constexpr int TRANS_TMAX_MAX = 16;
constexpr int TRANS_ROWS = 8;
inline bool trans_shape_ok(int tmax, int smax, int rb)
{
    return tmax >= 1 && tmax <= TRANS_TMAX_MAX && smax >= 1 && smax <= 64 && (rb == 1 || rb == 2 || rb == 4) &&
           2 * smax * rb <= TRANS_ROWS * tmax;
}
template <class T>
inline size_t trans_lds_bytes(int smax, int rb) { return (size_t)smax * 2 * 64 * rb * sizeof(cpx<T>); }
// right-hand sides across the lanes of a wave
inline int trans_rw(int nrhs) { return nrhs >= 4 ? 4 : (nrhs >= 2 ? 2 : 1); }
template <class T>
struct TransLevel {
    int K = 0, ntile = 0;
    int nqc = 0, first = 0;     // sample chunks; first position in each XCD's workgroup sequence (launcher)
    const int *tile_tgt = nullptr, *tile_bat = nullptr, *bat_src = nullptr, *src = nullptr;
    const int *bat_row = nullptr, *row = nullptr, *ent = nullptr;
    const cpx<T> *trans = nullptr, *U = nullptr;
    cpx<T> *V = nullptr;
};
template <class T>
struct TransArgs {
    int nlev = 0, nblocks = 0, smax = 0, tmax = 0, rb = 1;   // nblocks: workgroups per XCD
    TransLevel<T> lv[TRANS_MAXLEV];
};
// false when the tile shape is invalid
template <class T>
bool launch_translate_tiled(const TransArgs<T> &a, int nrhs, hipStream_t s);

// Register-blocked translation over sibling groups (translate.hip; tables
// of GroupTiles in setup.hpp): every lane keeps the sums of all targets of
// its group and streams the group's source records, so a source value is
// loaded once for all the targets whose interaction lists hold it.
template <class T>
struct GroupLevel {
    int K = 0, ngroup = 0;
    int nqc = 0, first = 0;     // sample chunks of a workgroup; first position per XCD (launcher)
    const int *first_tgt = nullptr, *count = nullptr, *rec_start = nullptr, *src = nullptr;
    const int *off = nullptr;   // per record tg offset ids, -1 = not in that target's list
    const cpx<T> *trans = nullptr, *U = nullptr;
    cpx<T> *V = nullptr;
};
template <class T>
struct GroupArgs {
    int nlev = 0, nblocks = 0, tg = 4, rb = 1;   // tg: targets per group (4 or 8); rb: RHS per lane
    int rw = 0;                                  // lanes over the RHS (1, 2, 4, 8, 16; 0: trans_rw(nrhs))
    int lds = 0;                                 // 1: operator values staged in LDS (k_translate_lds)
    GroupLevel<T> lv[TRANS_MAXLEV];
};
// false when (tg, rw, rb) has no kernel
template <class T>
bool launch_translate_groups(const GroupArgs<T> &a, int nrhs, hipStream_t s);
// One octree step of aggregation (children at level l+1 -> parents at l) or
// disaggregation (parents -> children), done per box and chunk of theta rows
// in LDS (levels.hip).  Sample index = theta row * nph + phi column.
//  aggregation: workgroup = (parent, chunk of `rows` parent theta rows); the
//    chunk needs child theta rows win[2 c] .. win[2 c + 1] (exclusive);
//  disaggregation: workgroup = (child, chunk of `rows` child theta rows); the
//    chunk needs parent (and intermediate) theta rows win[2 c] .. win[2 c + 1].
// `wrows` is the largest window of any chunk.
template <class T>
struct LevelStep {
    int nbox = 0;                       // parents (aggregation) or children (disaggregation)
    int nth_p = 0, nph_p = 0, nth_c = 0, nph_c = 0;
    int rows = 0, nchunk = 0, wrows = 0, taps = 0;
    int rb = 0;                         // right-hand sides per workgroup (0: the launcher's choice)
    int group = 0;                      // aggregation: children staged together (0: the launcher's choice)
    int pipe = 0;                       // > 0: the pipelined kernel; per pass this many vectors (component x
                                        // right-hand side; 1, 2, 4) in the disaggregation, right-hand sides
                                        // (1, 2; 4 counts as 2) in the aggregation
    const int *win = nullptr;
    const int *child_start = nullptr;   // aggregation: children of each parent
    const int *parent = nullptr;        // disaggregation: parent of each child
    const int *oct = nullptr;           // octant of each child in its parent
    // aggregation: theta and phi stencils with `taps` entries per row
    const int *c1 = nullptr, *c2 = nullptr;
    const T *w1 = nullptr, *w2 = nullptr;
    // disaggregation: separable transposed stencils (SepStencil on the host)
    int tphi = 0, tth = 0;
    const int *phi_col = nullptr, *th_row = nullptr, *th_sh = nullptr;
    const T *phi_w = nullptr, *rowf = nullptr, *th_w = nullptr;
    const cpx<T> *shift = nullptr;      // exp(+jk khat.(r_child - r_parent)), 8 x Kp
    const cpx<T> *in = nullptr;
    cpx<T> *out = nullptr;
};
// LDS bytes of a step (both components of the window and of the intermediate)
template <class T>
inline size_t agg_lds_bytes(int wrows, int rows, int nph_c) { return 2 * (size_t)(wrows + rows) * nph_c * sizeof(cpx<T>); }
template <class T>
inline size_t dis_lds_bytes(int wrows, int nph_p, int nph_c) { return 2 * (size_t)wrows * (nph_p + nph_c) * sizeof(cpx<T>); }
constexpr size_t STEP_LDS_MAX = 64 * 1024;
// One level step on the matrix cores (levels_mfma.hip, complex64): the
// stencils as dense, zero-padded real matrices (see the kernels).  ok = 0
// when the step's stencils are not separable in that form or exceed the
// kernels' tile limits (16 x 8 parent phi columns, 16 x 4 parent theta rows).
struct StepMfma {
    int ok = 0;
    int nbox = 0;                       // parents (aggregation) or children (disaggregation)
    int nth_p = 0, nph_p = 0, nth_c = 0, nph_c = 0;
    const int *child_start = nullptr, *parent = nullptr, *oct = nullptr;
    const cpx<float> *shift = nullptr;
    int njt = 0;                        // tiles of 16 child phi columns
    // aggregation: theta over the child rows extended across the poles
    int nit = 0, ne = 0, e_pad = 0, jc_pad = 0;
    const int *ext_row = nullptr, *ext_sh = nullptr, *ks_lo = nullptr, *ks_hi = nullptr;
    const float *ath = nullptr;         // [nit * 16][e_pad]
    const float *bph = nullptr;         // [16 * ceil(nph_p / 16)][jc_pad]
    const unsigned *bmask = nullptr;    // per child phi tile: bit p = block p of bph is non-zero
    // disaggregation
    int nks = 0, jp_pad = 0, nict = 0, ip_pad = 0;
    unsigned rmask = 0;                 // parent theta tiles reached across a pole
    const unsigned long long *kmask = nullptr, *kmask_s = nullptr;   // per child phi tile: non-zero k-steps
    const float *dph = nullptr;         // [njt * 16][jp_pad]
    const float *rowf = nullptr;        // [ip_pad]
    const float *dthd = nullptr, *dthr = nullptr;   // [nict * 16][ip_pad]
    const unsigned *dmask = nullptr, *rmask_c = nullptr;   // per child theta tile
};
bool launch_aggregate_mfma(const StepMfma &a, const cpx<float> *in, cpx<float> *out, int nrhs, hipStream_t s);
bool launch_disaggregate_mfma(const StepMfma &a, const cpx<float> *in, cpx<float> *out, int nrhs, hipStream_t s);

// return false when the step has no fused kernel (taps or LDS size)
template <class T>
bool launch_aggregate_step(const LevelStep<T> &a, int nrhs, hipStream_t s);
template <class T>
bool launch_disaggregate_step(const LevelStep<T> &a, int nrhs, hipStream_t s);

// Radiation on the matrix cores (mfma.hip): FP32 MFMAs for complex float,
// FP64 MFMAs for complex double, at least 16 right-hand sides; return false
// otherwise
template <class T>
bool launch_radiate_mfma(int op, int nbox, int K, const int *box_start, const cpx<T> *R, const cpx<T> *X, cpx<T> *U,
                         int nrhs, hipStream_t s);
// Near field and receive on the matrix cores (16+ right-hand sides).
// items = (leaf box, row tile of 16 rows) pairs; cols[col_off[b] ..] = the
// RWGs of leaf box b's adjacent boxes in block-row order.
template <class T>
bool launch_near_mfma(int nitem, const int2 *items, const int *box_start, const int *col_off, const int *cols,
                      const long long *val_off, const cpx<T> *vals, const int *id_start, const int *id_col,
                      const T *id_w, const cpx<T> *X, cpx<T> *Y, int nrhs, hipStream_t s);
template <class T>
bool launch_receive_mfma(int op, int nitem, const int2 *items, int K, const int *box_start, const cpx<T> *R,
                         const cpx<T> *Q, const T *wq, const cpx<T> *V, cpx<T> *Y, int nrhs, hipStream_t s);

// Outer GMRES vector kernels (krylov.hip); column-major blocks, element
// (n, r) at r * ld + n; basis vector i of V starts at V + i * vstride.
// out[i * nrhs + r] = <V_i(:, r), w(:, r)> (conjugate-linear in V), i < nv,
// accumulated in double; part holds nv x nchunk x nrhs partial sums.
template <class T>
void krylov_dots(const cpx<T> *V, long long vstride, long long ldv, int nv, const cpx<T> *w, long long ldw, long long n,
                 int nrhs, cpx<double> *part, int nchunk, cpx<double> *out, hipStream_t s);
// w(:, r) += sign * sum_i V_i(:, r) h[i * nrhs + r]
template <class T>
void krylov_combine(const cpx<T> *V, long long vstride, long long ldv, int nv, const cpx<double> *h, double sign,
                    cpx<T> *w, long long ldw, long long n, int nrhs, hipStream_t s);
// y(:, r) = a[r] x(:, r) + b[r] z(:, r)  (z = null: the second term is dropped)
template <class T>
void krylov_axpby(const cpx<double> *a, const cpx<T> *x, long long ldx, const cpx<double> *b, const cpx<T> *z,
                  long long ldz, cpx<T> *y, long long ldy, long long n, int nrhs, hipStream_t s);

// Column-major blocks between precisions: b = (complex float) a; a = b, or
// a += b with add.
void launch_to_single(const cpx<double> *a, long long lda, cpx<float> *b, long long ldb, long long n, int nrhs,
                      hipStream_t s);
void launch_from_single(cpx<double> *a, long long lda, const cpx<float> *b, long long ldb, long long n, int nrhs,
                        bool add, hipStream_t s);

// Sparse (CSR) times a column-major block: y(i, r) = alpha * sum_k val[k]
// x(col[k], r) (+ y(i, r) with accumulate), rows i < nrows.
template <class T>
void launch_csr_spmm(long long nrows, int nrhs, const long long *ptr, const int *col, const cpx<T> *val,
                     const cpx<T> *x, long long ldx, cpx<T> *y, long long ldy, double alpha, bool accumulate,
                     hipStream_t s);

template <class T>
void launch_disagg_mid(int nchild, int mid_len, int Kp, const int *parent, const int *oct, const cpx<T> *shift,
                       const int *st, const int *col, const T *w, const cpx<T> *Vp, cpx<T> *mid, int nrhs,
                       hipStream_t s);
template <class T>
void launch_zero(cpx<T> *p, long long n, hipStream_t s);
template <class T>
void launch_receive(int op, int N, int K, const int *leaf_of, const cpx<T> *R, const cpx<T> *Q, const T *wq,
                    const cpx<T> *V, cpx<T> *Y, int nrhs, hipStream_t s);
// One right-hand side with the permutations folded in: the radiation reads
// the caller's vector x (user order, J half then M half) through perm (tree
// position -> user RWG) and also stores it in tree order in X; the receive
// adds the far field to the tree-order near field Y and writes the sum to y
// in user order.
template <class T>
void launch_radiate1_user(int op, int nbox, int K, const int *box_start, const cpx<T> *R, const cpx<T> *x,
                          const int *perm, int N, cpx<T> *X, cpx<T> *U, hipStream_t s);
template <class T>
void launch_receive1_user(int op, int N, int K, const int *leaf_of, const cpx<T> *R, const cpx<T> *Q, const T *wq,
                          const cpx<T> *V, const cpx<T> *Y, cpx<T> *y, const int *perm, hipStream_t s);

}  // namespace mlfma
