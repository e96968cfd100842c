// Sparse approximate inverse (SAI) of the near-field part of the BI block.
//
// The paper preconditions GMRES with an SAI built from the BI block C alone
// (Sec. III, dielectric-plate example).  Here M minimises || I - C_near M ||_F
// column by column: the columns (n, J) and (n, M) of M live on the J and M
// unknowns of pattern(n), the SAI_MAXP or fewer RWGs nearest to RWG n inside
// the leaf boxes adjacent to n's, and solve the least-squares problem
// min || C_near m - e ||_2 over all rows of C_near (C_near = the stored near
// blocks plus, for op C, the Gram terms).
#pragma once
#include "device.hpp"

namespace mlfma {

constexpr int SAI_MAXP = 32;             // RWGs per pattern at most
constexpr int SAI_D = 2 * SAI_MAXP;      // unknowns per pattern (J and M halves); stride of M

// Build, one workgroup per RWG u in [u0, u0 + count) (internal order), in
// double precision: the normal equations G m = A^H e of the least-squares
// problem, accumulated over the rows of every leaf box in rb[rb_start[u] ..]
// (the boxes adjacent to a box of the pattern), then a Cholesky solve.
// pat[pat_start[u] ..]: pattern (internal RWG indices, at most SAI_MAXP).
// vals: near blocks (A, B) per slot in the layout of the near-field product;
// id_*: Gram terms of op C (id_start = nullptr for op EM).
// Output M[(u * 2 + h) * SAI_D + 2 j + h'] = entry of column (u, h) on the
// unknown (pattern[j], h'); status[0] is set to 1 if some Gram matrix is not
// numerically positive definite.
void launch_sai_build(int u0, int count, const int *pat_start, const int *pat, const int *rb_start, const int *rb,
                      const int *leaf_of, const int *box_start, const int *near_start, const int *near_box,
                      const long long *val_off, const cpx<double> *vals, const int *id_start, const int *id_col,
                      const double *id_w, cpx<double> *M, int *status, hipStream_t s);

// y = M x on user-ordered column-major vectors (2N x nrhs, J rows then M
// rows): row p of M holds the entries row_start[p] .. row_start[p + 1]; entry
// e belongs to column RWG ent_col[e] (user index) and its four values are
// M[ent_val[e] + {0, 1, SAI_D, SAI_D + 1}] = (row J, col J), (row M, col J),
// (row J, col M), (row M, col M).
template <class T>
void launch_sai_apply(int N, int nrhs, const int *row_start, const int *ent_col, const int *ent_val,
                      const cpx<T> *M, const cpx<T> *x, long long ldx, cpx<T> *y, long long ldy, hipStream_t s);

}  // namespace mlfma
