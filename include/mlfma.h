/*
 * mlfma.h -- C ABI of the MI355X library for the boundary-integral (BI)
 * matrix-vector product of the coupled HDG-BI method (arXiv 2210.04892),
 * accelerated by the multilevel fast multipole algorithm (MLFMA).
 *
 * The product is the step of the hybrid solver's matrix-vector subroutine
 * that multiplies the guess vector by the dense BI block (Sec. II-E, step
 * 2(a), "Hybrid Solver"): y = C x with C = [[C^JJ, C^JM], [C^MJ, C^MM]]
 * (entries eqs. 43-46, alpha = 1/2 as fixed in Sec. II-C), or the plain
 * operator pair of the Stratton-Chu representation (eqs. 22a/b tested as in
 * the EFIE/MFIE eqs. 24a/b).  Unknowns are the RWG coefficients of the
 * equivalent currents J and M (expansions eqs. exp4-exp5); 2N of them for N
 * RWG functions.
 *
 * Conventions (fixed readings where the paper is silent):
 *  - time dependence e^{+j w t}; Green's function exp(-jkR)/(4 pi R);
 *    fields normalised so that the EFIE operator L carries -jk and the MFIE
 *    operator K carries 1 (Sec. II-A normalisation by sqrt(eps0/mu0));
 *  - the surface is closed and its triangles are counter-clockwise seen
 *    from outside (outward normal, Sec. II-A);
 *  - RWG n lives on the edge (a,b), a < b, numbered in lexicographic order of
 *    (a,b); T+ is the triangle in which a->b runs counter-clockwise;
 *    f = (l/2A+)(r - p+) on T+ and (l/2A-)(p- - r) on T-;
 *  - triangle pairs that share no vertex are integrated with the 7-point
 *    degree-5 rule on both triangles; pairs that share a vertex, an edge or
 *    the whole triangle are integrated to ~1e-12 relative accuracy.
 *
 * Vectors are complex, interleaved (re, im), column-major 2N x nrhs with a
 * leading dimension; rows [0, N) hold J (op C) or the E-side (op EM)
 * coefficients, rows [N, 2N) hold M (op C) or the H-side (op EM), in the RWG
 * order above.  All functions return MLFMA_OK (0) or a negative error code;
 * mlfma_last_error() then describes the failure (thread-local text).  No
 * C++ exception crosses this boundary.
 */
#ifndef MLFMA_H
#define MLFMA_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mlfma_ctx *mlfma_handle;

enum {
    MLFMA_OK = 0,
    MLFMA_ERR_ARG = -1,          /* bad argument (null pointer, size, enum)        */
    MLFMA_ERR_MESH = -2,         /* open, non-manifold, mis-oriented, degenerate   */
    MLFMA_ERR_OOM = -3,          /* device memory exhausted or over the budget     */
    MLFMA_ERR_HIP = -4,          /* HIP runtime error (launch or asynchronous)     */
    MLFMA_ERR_STATE = -5,        /* call out of order (e.g. matvec before nearfield) */
    MLFMA_ERR_TREE = -6,         /* touching triangles whose RWGs are not near     */
    MLFMA_ERR_UNSUPPORTED = -7
};

enum { MLFMA_C128 = 0, MLFMA_C64 = 1 };     /* vector element type = arithmetic  */
enum {
    MLFMA_OP_C = 0,    /* y = C x, the BI block of eq. 42 (entries eqs. 43-46)        */
    MLFMA_OP_EM = 1    /* y = [T xJ - K xM ; T xM + K xJ], T = <f,L f>, K = <f,Kbar f> */
};

typedef struct {
    double wavenumber;   /* k in rad per length unit (k = 2 pi / lambda)            */
    double leaf_size;    /* edge of the finest octree boxes, length units           */
    int digits;          /* MLFMA accuracy parameter d0 of the truncation rule (3)  */
    int interp_order;    /* Lagrange points per angular dimension (8)               */
    int leaf_extra_L;    /* extra multipoles added at the leaf level (2)            */
    int max_rhs;         /* right-hand sides the workspace is sized for (1)         */
    int device;          /* HIP device ordinal (-1: the current device)             */
    unsigned long long hbm_budget_bytes;   /* 0 = no limit                          */
    int trans_kernel;    /* translation kernel: MLFMA_TRANS_AUTO (autotuner picks)   */
    int level_kernel;    /* level steps: MLFMA_LEVELS_AUTO (autotuner picks)         */
    int near_precision;  /* arithmetic of the near part of complex128 products      */
    int far_precision;   /* and of their MLFMA far part: MLFMA_PREC_* (as the dtype) */
} mlfma_options;
/* Precision of a part of complex128 products (complex64 products always
 * compute in FP32): MLFMA_PREC_DTYPE = the vector's (FP64), MLFMA_PREC_FP32
 * = complex FP32 accumulated in FP32 on tables precomputed in FP64 (the
 * input is rounded to complex64 for that part, its result added to the
 * other part in FP64). */
enum { MLFMA_PREC_DTYPE = 0, MLFMA_PREC_FP64 = 1, MLFMA_PREC_FP32 = 2 };
/* Translation kernels.  TILED: LDS tiles of targets; GROUPS: sibling groups
 * with the sums in registers (vector FMAs), the operator values loaded per
 * lane or staged in LDS per workgroup; LDS: only the latter; AUTO: the
 * autotuner times the shapes of TILED and GROUPS and keeps the fastest;
 * MATRIX: groups of 16 targets whose sums per sample are a complex product
 * on the matrix cores (FP32 MFMAs for complex64, FP64 for complex128), its
 * shapes timed.  MATRIX pays where the targets of a group share most of
 * their sources (volumes); on surface meshes most of its operand is zero and
 * GROUPS is faster. */
enum {
    MLFMA_TRANS_AUTO = 0,
    MLFMA_TRANS_TILED = 1,
    MLFMA_TRANS_GROUPS = 2,
    MLFMA_TRANS_MATRIX = 3,
    MLFMA_TRANS_LDS = 4
};
/* Level-step kernels.  AUTO: the autotuner picks (complex64: vector or
 * matrix cores; the vector kernels' shape per level and precision).  VECTOR:
 * vector kernels of autotuned shape.  MATRIX: complex64 steps on the matrix
 * cores.  BLOCKED: vector kernels with right-hand sides blocked per
 * workgroup only.  PIPELINED: vector kernels pipelined over the right-hand
 * sides (and children) wherever a step fits their limits, for products of
 * four or more right-hand sides. */
enum {
    MLFMA_LEVELS_AUTO = 0,
    MLFMA_LEVELS_VECTOR = 1,
    MLFMA_LEVELS_MATRIX = 2,
    MLFMA_LEVELS_BLOCKED = 3,
    MLFMA_LEVELS_PIPELINED = 4
};

/* Fill *opt with defaults: k = 2 pi, leaf 0.25, d0 = 3, order 8, extra 2,
 * one RHS, current device, no budget, autotuned translation and level-step
 * kernels, both parts of complex128 products in FP64.  The paper cites MLFMA
 * without its parameters: the truncation rule (d0), the Lagrange order and
 * the leaf size are this library's, chosen to reach 3 digits (Sec. II-E
 * asks for the product, not for a parameter set).  Returns MLFMA_ERR_ARG on
 * NULL. */
int mlfma_options_default(mlfma_options *opt);

/*
 * Validate the closed surface (Sec. II-B: the triangles of Gamma_h), build
 * the RWG table, the octree over RWG centres (edge midpoints), the k-space
 * sampling, interpolation stencils and translation operators of every level,
 * and the leaf radiation/receive patterns on the device.
 *   verts: n_verts x 3 doubles, row-major (host memory, copied);
 *   tris : n_tris x 3 ints, row-major, counter-clockwise from outside.
 * On success *out owns all device memory of the geometry.  Errors:
 * MLFMA_ERR_MESH, MLFMA_ERR_TREE, MLFMA_ERR_OOM, MLFMA_ERR_HIP, MLFMA_ERR_ARG.
 * Blocking (synchronises the device).
 */
int mlfma_build_tree(const double *verts, long long n_verts, const int *tris, long long n_tris,
                     const mlfma_options *opt, mlfma_handle *out);

/*
 * Compute the near-field blocks in double precision on the device: for every
 * pair of RWGs whose leaf boxes are adjacent, the entries of T, K, n x L and
 * n x Kbar (the operators of eqs. 22-27 and 43-46), the identity terms of
 * eqs. 43, 44, 46 (Gram matrices), and a single-precision copy.  Blocking.
 * Errors: MLFMA_ERR_OOM, MLFMA_ERR_HIP, MLFMA_ERR_ARG.
 */
int mlfma_precompute_nearfield(mlfma_handle h);

/*
 * y = A x for A = C (op MLFMA_OP_C) or the EM pair (op MLFMA_OP_EM): the near
 * part from the stored blocks, the far part by MLFMA (radiation, aggregation
 * with Lagrange interpolation, diagonal translation, anterpolation and
 * disaggregation, receive).  Sec. II-E step 2(a).
 *   dtype: MLFMA_C128 (complex double in/out, double arithmetic unless the
 *          handle's near_precision / far_precision options ask for FP32
 *          parts) or MLFMA_C64 (complex float in/out, single arithmetic on
 *          tables precomputed in double);
 *   x, y : DEVICE pointers, 2N x nrhs column-major, leading dimensions ldx,
 *          ldy >= 2N (elements); y is overwritten; x and y must not overlap;
 *   hip_stream: hipStream_t to enqueue on (NULL = default stream).
 * Asynchronous: returns after enqueueing.  Enqueue-time errors are returned;
 * an asynchronous device error is reported by the next call on the handle.
 * Grows the workspace (a blocking allocation) if nrhs exceeds what it was
 * sized for.  Not thread-safe for concurrent calls on one handle; products
 * on one handle share its workspace, so products enqueued on different
 * streams must be ordered by the caller.  The near part runs on a second
 * stream of the handle, forked from and joined back into hip_stream (so the
 * call is also valid inside a stream capture of hip_stream).
 * Errors: MLFMA_ERR_STATE (near field not computed), MLFMA_ERR_ARG,
 * MLFMA_ERR_OOM, MLFMA_ERR_HIP.
 */
int mlfma_matvec_LK(mlfma_handle h, int op, int dtype, long long nrhs, const void *x, long long ldx,
                    void *y, long long ldy, void *hip_stream);

/* ------------------------------------------------------------------------
 * Allocation-free product, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, hosts that forbid
 * allocation inside the loop).  Same arguments, result and asynchrony as
 * mlfma_matvec_LK, but the product's scratch (internal vectors, box
 * patterns of every level, level-step intermediate) lives in one static
 * device array of MLFMA_NOALLOC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends; nothing is allocated or
 * freed, and the near field runs on hip_stream itself (no second stream).
 * A product whose scratch exceeds the array (about (4N + sum over levels of
 * 4 boxes K + the largest level-step intermediate) x nrhs complex elements,
 * each padded to 256 bytes) is refused with MLFMA_ERR_ARG, nothing enqueued.
 * Every call on one GPU uses that GPU's one array: calls whose products may
 * overlap on the device (other streams, other threads) race and must be
 * ordered by the caller.  The array keeps the last call's contents; the
 * product writes every scratch element before reading it.
 * ------------------------------------------------------------------------ */
#define MLFMA_NOALLOC_SCRATCH_BYTES (256ULL << 20)
int mlfma_matvec_LK_noalloc(mlfma_handle h, int op, int dtype, long long nrhs, const void *x, long long ldx,
                            void *y, long long ldy, void *hip_stream);

/* ------------------------------------------------------------------------
 * Several products in one call (the batched form of Sec. II-E step 2(a) for
 * many geometries or operators): every item is y = A x as in
 * mlfma_matvec_LK.  Items of different geometries run concurrently on
 * streams of their handles, forked from and joined back into hip_stream;
 * items of one geometry run in list order (they share its workspace).  All
 * items are checked before anything is enqueued (the first bad one is
 * reported, "item i: ..."); all handles must live on one device.
 * Asynchronous like mlfma_matvec_LK; valid inside a stream capture of
 * hip_stream.  Grows workspaces as mlfma_matvec_LK does.
 * ------------------------------------------------------------------------ */
typedef struct {
    mlfma_handle h;
    int op, dtype;           /* MLFMA_OP_*, MLFMA_C128 / MLFMA_C64              */
    long long nrhs;
    const void *x;           /* device, 2N x nrhs column-major, ldx >= 2N        */
    long long ldx;
    void *y;                 /* device, overwritten; must not overlap x          */
    long long ldy;
} mlfma_batch_item;
int mlfma_matvec_batch(const mlfma_batch_item *items, int n_items, void *hip_stream);

/* Products of several geometries in lockstep with shared translation
 * launches (the batched form of Sec. II-E step 2(a) for many uneven
 * geometries): the diagonal translations of every level of every item run
 * as one work list over (geometry, level, group of target boxes, sample
 * chunk, right-hand-side slice), at most 20 levels per launch, in the
 * sibling-group kernel shape the autotuner picked for the item with the most
 * translation work; the other stages run concurrently on the handles' own
 * streams, forked from hip_stream before and after the shared translations
 * (each near field on its handle's side stream).  Items: distinct handles on one
 * device, one dtype and one nrhs for all, no handle with FP32 parts of
 * complex128 products; otherwise MLFMA_ERR_ARG ("item i: ...") and nothing
 * is enqueued.  The results equal the single products bit for bit where a
 * handle's own translation is the sibling-group kernel (every target sums
 * its sources in the same order in every shape), else to rounding.
 * Asynchronous; grows workspaces as mlfma_matvec_LK does. */
int mlfma_matvec_batch_fused(const mlfma_batch_item *items, int n_items, void *hip_stream);

/*
 * Diagnostic split of mlfma_matvec_LK (same arguments, same asynchrony):
 *   part = MLFMA_PART_NEAR : near-field blocks (and identity terms) only;
 *   part = MLFMA_PART_FAR  : MLFMA far field only;
 *   part = MLFMA_PART_ALL  : both (identical to mlfma_matvec_LK);
 *   part = MLFMA_PART_LEVEL + l : far field restricted to the translations
 *          at octree level l (2 <= l < levels), the per-level error split.
 * Errors as mlfma_matvec_LK, plus MLFMA_ERR_ARG for an unknown part.
 */
enum { MLFMA_PART_NEAR = 1, MLFMA_PART_FAR = 2, MLFMA_PART_ALL = 3, MLFMA_PART_LEVEL = 16 };
int mlfma_matvec_part(mlfma_handle h, int op, int dtype, int part, long long nrhs, const void *x, long long ldx,
                      void *y, long long ldy, void *hip_stream);

/*
 * Right-hand sides of the coupled system for incident plane waves (eqs. 49,
 * 50, excitation of Sec. III with E0 = 1 in the normalised units):
 *   b^J_m = <f_m, E/2 + n x H/2>,  b^M_m = <f_m, H/2 - n x E/2>,
 *   E = pol exp(-jk khat.r),  H = khat x pol exp(-jk khat.r),
 * 7-point rule per triangle.  khat, pol: host arrays nrhs x 3 (unit vectors,
 * pol perpendicular to khat); b: DEVICE, 2N x nrhs column-major (ldb >= 2N),
 * complex128 or complex64 by dtype.  Blocking on hip_stream.
 */
int mlfma_plane_wave_rhs(mlfma_handle h, int dtype, long long nrhs, const double *khat, const double *pol, void *b,
                         long long ldb, void *hip_stream);

/* Far field of the surface currents x (radar cross section, Sec. III):
 * with E = L{J} - K{M} (the operators of Sec. II-C) the scattered field is
 * exp(-jkr)/r F(khat) far away, F = (-jk/4pi)[P_J - khat (khat . P_J) -
 * khat x P_M], P_X = Int X exp(+jk khat . r) ds (7-point rule on every
 * triangle, double-precision sums); sigma = 4 pi |F|^2 for a unit incident
 * field.
 *   x:    device, column-major 2N x nrhs (ldx >= 2N), J rows then M rows
 *   dirs: host, ndir x 3 unit vectors (observation directions khat)
 *   F:    device, ndir x 2 x nrhs complex of dtype (row-major):
 *         F . theta_hat and F . phi_hat, theta_hat = (cos t cos p, cos t
 *         sin p, -sin t), phi_hat = (-sin p, cos p, 0), t = acos(khat_z),
 *         p = atan2(khat_y, khat_x)
 * Enqueued on hip_stream and waited for before returning.  MLFMA_ERR_ARG for
 * a null pointer, a bad count or a direction that is not a unit vector. */
int mlfma_far_field(mlfma_handle h, int dtype, long long nrhs, const void *x, long long ldx, long long ndir,
                    const double *dirs, void *F, void *hip_stream);

/* ------------------------------------------------------------------------
 * Captured products (HIP graphs).  mlfma_graph_create records the whole
 * product y = A x of mlfma_matvec_LK (same arguments and checks; op, dtype,
 * nrhs and the x / y pointers are fixed in the graph) into an instantiated
 * HIP graph; mlfma_graph_launch replays it on hip_stream with no further
 * host work per kernel.  The graph uses the handle's workspace: replays and
 * products on the same handle must not overlap, the handle must outlive the
 * graph, and a replay returns MLFMA_ERR_STATE once a product with more
 * right-hand sides has reallocated that workspace.  The captured sequence
 * contains kernels only (memory is cleared by kernels, not memset nodes).
 * ------------------------------------------------------------------------ */
typedef struct mlfma_graph_s *mlfma_graph;
int mlfma_graph_create(mlfma_handle h, int op, int dtype, long long nrhs, const void *x, long long ldx, void *y,
                       long long ldy, mlfma_graph *out);
int mlfma_graph_launch(mlfma_graph g, void *hip_stream);
/* NULL accepted. */
int mlfma_graph_destroy(mlfma_graph g);

/* ------------------------------------------------------------------------
 * Outer Krylov solver.  The hybrid solver of Sec. II-E wraps the product in
 * GMRES (its experiments stop at a relative residual of 1e-3).  mlfma_gmres
 * solves A x = b for the operator op (MLFMA_OP_C: the BI block C of eqs.
 * 43-46 alone; MLFMA_OP_EM: the L/K pair) with restarted GMRES(restart), one
 * Krylov space per right-hand-side column, every Arnoldi step one batched
 * product of all columns (classical Gram-Schmidt applied twice, inner
 * products in double precision, on hip_stream; rotations on the host).
 *   b, x: device, column-major 2N x nrhs (ldb, ldx >= 2N), must not overlap;
 *         x holds the initial guess on entry and the solution on return.
 *   All columns iterate until the largest estimated relative residual is at
 *   most tol or max_iters Arnoldi steps were taken; *iters (may be NULL) =
 *   steps taken; relres (host, nrhs doubles) = true ||b - A x|| / ||b|| per
 *   column, recomputed at exit (0 for a zero column of b).
 * Synchronous: returns after the solve (it reads the Hessenberg entries on
 * the host every step).  Allocates its Krylov basis ((restart + 1) x 2N x
 * nrhs) for the call.  Errors as mlfma_matvec_LK; MLFMA_ERR_ARG for restart
 * outside 1..512, max_iters < 1 or tol <= 0.
 * ------------------------------------------------------------------------ */
int mlfma_gmres(mlfma_handle h, int op, int dtype, long long nrhs, const void *b, long long ldb, void *x,
                long long ldx, int restart, int max_iters, double tol, int *iters, double *relres, void *hip_stream);

/* ------------------------------------------------------------------------
 * Sparse approximate inverse (SAI) preconditioner.  The paper preconditions
 * GMRES with an SAI built from the BI block C alone (Sec. III, dielectric
 * plate, citing the Frobenius-norm SAI of Lee et al.).  M minimises
 * || I - C_near M ||_F column by column, where C_near holds the entries of
 * op's matrix for RWG pairs in adjacent leaf boxes (the near field the
 * library stores; for MLFMA_OP_C with its Gram terms): the columns (n, J)
 * and (n, M) live on the J and M unknowns of pattern(n) = the k_nearest
 * RWGs whose centres (edge midpoints) are nearest to n's among the RWGs of
 * the leaf boxes adjacent to n's (n itself included; every RWG tied with the
 * k-th distance to 1e-9 relative is included), and solve min || C_near m -
 * e ||_2 over all rows of C_near by its normal equations (double precision,
 * on the device).  Stored in complex128 and complex64.
 *
 * mlfma_sai_build: after mlfma_precompute_nearfield; k_nearest in 1..32.
 *   Synchronous.  Replaces an earlier SAI of the same op (after a failed
 *   build the op has none).  Allocates
 *   N x 2 x 64 entries in each precision plus index lists (counted against
 *   the handle's budget).  MLFMA_ERR_UNSUPPORTED if ties push a pattern past
 *   32 RWGs or a Gram matrix is not numerically positive definite.
 * mlfma_sai_apply: y = M x for device x, y (column-major 2N x nrhs in user
 *   RWG order, J rows then M rows; ldx, ldy >= 2N; must not overlap),
 *   enqueued on hip_stream.  MLFMA_ERR_STATE before mlfma_sai_build.
 * mlfma_sai_info: RWG-pair entries of M (each a 2 x 2 block), the largest
 *   pattern, build time in ms (host + device) and device bytes held.
 * mlfma_gmres_precond: mlfma_gmres with precond = MLFMA_PRECOND_SAI (right
 *   preconditioning: GMRES on A M u = b, x = x0 + M u; the residuals and tol
 *   are those of A x = b) or MLFMA_PRECOND_NONE (= mlfma_gmres).
 *   MLFMA_ERR_STATE if the SAI of op was not built.
 * ------------------------------------------------------------------------ */
enum { MLFMA_PRECOND_NONE = 0, MLFMA_PRECOND_SAI = 1 };
int mlfma_sai_build(mlfma_handle h, int op, int k_nearest);
int mlfma_sai_apply(mlfma_handle h, int op, int dtype, long long nrhs, const void *x, long long ldx, void *y,
                    long long ldy, void *hip_stream);
int mlfma_sai_info(mlfma_handle h, int op, long long *nnz, int *max_pattern, double *build_ms,
                   unsigned long long *bytes);
int mlfma_gmres_precond(mlfma_handle h, int op, int dtype, long long nrhs, const void *b, long long ldb, void *x,
                        long long ldx, int restart, int max_iters, double tol, int precond, int *iters,
                        double *relres, void *hip_stream);

/* ------------------------------------------------------------------------
 * Hybrid product of the reduced system (Sec. II-E "Hybrid Solver", eq. 52):
 *   y = (C - D^{X Lambda} Q^{-1} D^{Lambda X}) x,
 * steps 2(a)-(e) of the hybrid solver's matrix-vector subroutine: (a) y_d =
 * C x by MLFMA (mlfma_matvec_LK, op C), (b) x1 = D^{Lambda X} x, (c) x2 =
 * Q^{-1} x1 by the caller's solve (the paper factorises the sparse HDG
 * block Q once with a sparse direct solver; here the caller supplies that
 * solve), (d) y_s = -D^{X Lambda} x2, (e) y = y_d + y_s.  D^{Lambda X}
 * (n_hdg x 2N) and D^{X Lambda} (2N x n_hdg) are the sparse couplings of
 * eq. 51 between the HDG unknowns Lambda and the BI unknowns X = [J; M]
 * (rows / columns in the RWG order of the vectors, J then M).
 *
 * mlfma_hybrid_create: host CSR arrays (copied to the device, values kept
 *   in complex128 and complex64): *_ptr (rows + 1 int64, ptr[0] = 0,
 *   non-decreasing), *_col (int32 column indices), *_val (complex128
 *   values, interleaved re/im).  solve(user, dtype, n, nrhs, b, ldb, xq,
 *   ldxq, hip_stream) must write xq = Q^{-1} b for the n x nrhs
 *   column-major DEVICE blocks it is given (complex128 or complex64 by
 *   dtype), ordered after the work enqueued on hip_stream, and return 0 (a
 *   non-zero return fails the product with MLFMA_ERR_ARG).  b and xq are
 *   always the caller's buffers buf1 and buf2 (device, ldbuf >= n_hdg,
 *   room for max_rhs columns of complex128; owned by the caller, alive as
 *   long as the operator).  The handle must outlive the operator.
 * mlfma_hybrid_matvec: arguments and asynchrony of mlfma_matvec_LK (op C
 *   implied), nrhs <= max_rhs.
 * mlfma_hybrid_gmres: mlfma_gmres_precond on the reduced operator (the SAI
 *   preconditioner, when asked for, is the one built from C alone).
 * Errors: MLFMA_ERR_ARG (bad CSR, sizes or pointers), MLFMA_ERR_OOM,
 *   MLFMA_ERR_HIP, and those of the product.
 * ------------------------------------------------------------------------ */
typedef int (*mlfma_qsolve_fn)(void *user, int dtype, long long n, long long nrhs, const void *b, long long ldb,
                               void *xq, long long ldxq, void *hip_stream);
typedef struct mlfma_hybrid_s *mlfma_hybrid;
int mlfma_hybrid_create(mlfma_handle h, long long n_hdg, const long long *dlx_ptr, const int *dlx_col,
                        const double *dlx_val, const long long *dxl_ptr, const int *dxl_col, const double *dxl_val,
                        mlfma_qsolve_fn solve, void *user, void *buf1, void *buf2, long long ldbuf,
                        long long max_rhs, mlfma_hybrid *out);
int mlfma_hybrid_matvec(mlfma_hybrid hy, int dtype, long long nrhs, const void *x, long long ldx, void *y,
                        long long ldy, void *hip_stream);
int mlfma_hybrid_gmres(mlfma_hybrid hy, int dtype, long long nrhs, const void *b, long long ldb, void *x,
                       long long ldx, int restart, int max_iters, double tol, int precond, int *iters,
                       double *relres, void *hip_stream);
/* NULL accepted; waits for the device. */
int mlfma_hybrid_destroy(mlfma_hybrid hy);

/* ------------------------------------------------------------------------
 * Serving (the request loop around step 2(a) of Sec. II-E for many outer
 * solvers at once): concurrent Krylov clients submit products for resident
 * geometries; the server batches continuously.  A scheduler thread merges
 * queued requests of the same (geometry, op, dtype) into one multi-RHS
 * product of at most max_batch_rhs columns and admits it to a free launch
 * slot (one stream and one workspace arena each; the arenas together stay
 * within hbm_budget_bytes, 0 = no limit); requests arriving while others run
 * are admitted as soon as a slot frees, so products for different geometries
 * overlap on the device.  x and y of a request are DEVICE buffers owned by
 * the caller and must stay valid until mlfma_server_wait returns; results are
 * the same as mlfma_matvec_LK's up to rounding.  Handles must outlive the
 * server's use of them.  All calls are thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct mlfma_server_s *mlfma_server;
typedef struct {
    int streams;                          /* launch slots (1..16, default 4)      */
    int max_batch_rhs;                    /* columns merged per product (16)      */
    int device;                           /* -1: the current device               */
    unsigned long long hbm_budget_bytes;  /* bound on the slots' arenas, 0 = none */
    int use_graphs;                       /* 1 (default): each slot replays its products as captured HIP
                                             graphs, one per (geometry, op, dtype, width), captured on
                                             first use; 0: every kernel launched from the host */
} mlfma_server_opts;
int mlfma_server_opts_default(mlfma_server_opts *opt);
int mlfma_server_create(const mlfma_server_opts *opt, mlfma_server *out);
/* Enqueue y = A x (arguments as mlfma_matvec_LK); *ticket identifies it.
 * The server reads x and writes y only after the work enqueued on hip_stream
 * (the caller's stream, NULL = default stream) before this call: an x that
 * the caller has just computed on its stream is used as computed.
 * MLFMA_ERR_STATE while the server is being destroyed. */
int mlfma_server_submit(mlfma_server s, mlfma_handle h, int op, int dtype, long long nrhs, const void *x,
                        long long ldx, void *y, long long ldy, void *hip_stream, long long *ticket);
/* Wait for a ticket (timeout_s < 0: forever).  On return y is complete;
 * *latency_s = completion - submission (seconds), *batch_rhs = columns of the
 * product it ran in (either pointer may be NULL).  MLFMA_ERR_STATE on timeout
 * (the ticket stays valid), MLFMA_ERR_OOM if it can never be admitted. */
int mlfma_server_wait(mlfma_server s, long long ticket, double timeout_s, double *latency_s, int *batch_rhs);
/* out[0..4] = {products launched, requests served, arena bytes, queued
 * requests, products captured as graphs} */
int mlfma_server_stats(mlfma_server s, long long out[5]);
/* Stop the threads and free the slots.  Requests still queued or running
 * fail with MLFMA_ERR_STATE (their buffers are no longer touched once this
 * returns); threads blocked in mlfma_server_wait return before the server is
 * freed.  No call on s may start once destroy has begun.  NULL accepted. */
int mlfma_server_destroy(mlfma_server s);

/* Free every device and host resource of the handle (library housekeeping:
 * no passage of the paper defines it).  NULL is accepted. */
int mlfma_release(mlfma_handle h);

/* Sizes: RWG count N (the paper's BI unknowns are 2N: J and M per RWG),
 * octree levels (root = level 0), bytes of device memory held by the
 * handle.  Any output pointer may be NULL. */
int mlfma_query(mlfma_handle h, long long *n_rwg, int *levels, unsigned long long *hbm_bytes);

/* RWG table in the order of the vectors: edge_ab (N x 2, a < b) and tri_pm
 * (N x 2, T+ then T-); host buffers supplied by the caller, either may be NULL. */
int mlfma_rwg_table(mlfma_handle h, int *edge_ab, int *tri_pm);

/* Per-level description: for level l (2 <= l < levels) writes
 * info[0..5] = {boxes, L, K samples, translations, box edge * 1e6 (rounded),
 * 0}.  Returns MLFMA_ERR_ARG for a level without translations. */
int mlfma_level_info(mlfma_handle h, int level, long long info[6]);

/* Near-field sizes: info[0..3] = {stored RWG pairs (slots), identity-term
 * entries, touching triangle pairs, leaf boxes}.  MLFMA_ERR_STATE before
 * mlfma_precompute_nearfield. */
int mlfma_near_info(mlfma_handle h, long long info[4]);

/* Translation kernel and shape chosen by the autotuner that mlfma_build_tree
 * runs (Sec. II-E diagonal translations).  Every shape of the kernels that
 * the trans_kernel option admits, within their LDS and register limits, is
 * timed on the device with the handle's right-hand-side count, capped at 16.
 * LDS-tiled kernel: shape[0] = target boxes per tile (= waves per
 * workgroup), shape[1] = source boxes per LDS batch, shape[2] = right-hand
 * sides per lane, shape[3] = 0.  Sibling-group kernel (sums of all targets
 * of a group of siblings kept in registers, sources streamed once per
 * group): shape[0] = targets per group, shape[1] = 0 (a group is one sibling
 * set or part of one), -1 (whole sibling sets merged up to shape[0]
 * targets) or -2 (merged, and a workgroup of four groups stages the
 * translation operators of its sample chunk in LDS), shape[2] = right-hand
 * sides per lane, shape[3] = lanes of a wavefront over the right-hand sides.  Matrix-core kernel: shape[0] = 16,
 * shape[1] = -1, shape[2] = samples per wavefront, shape[3] = tiles of 16
 * (component, right-hand side) columns per wavefront.  *ms (may be NULL) =
 * the timed translation of all levels, milliseconds.  dtype MLFMA_C128 or
 * MLFMA_C64; MLFMA_ERR_ARG otherwise. */
int mlfma_tuning(mlfma_handle h, int dtype, int shape[4], double *ms);

/* Level steps of complex64 products (aggregation with Lagrange
 * interpolation, disaggregation with anterpolation; Sec. II-E): on the
 * vector units or as real-split 16 x 16 x 4 FP32 MFMA products of the
 * separable stencil matrices, as the autotuner of mlfma_build_tree picked
 * (timing both for every level with the handle's right-hand-side count,
 * capped at 16) or mlfma_options.level_kernel fixed.  *matrix_cores = 1 for
 * the matrix-core kernels; ms[0], ms[1] (may be NULL) = the timed steps of
 * all levels, vector and matrix cores (0 when not timed).  MLFMA_ERR_ARG for
 * a NULL handle. */
int mlfma_tuning_steps(mlfma_handle h, int *matrix_cores, double ms[2]);

/* Shape of the vector level-step kernels of the step between octree level
 * `level` (2 <= level < levels - 1) and level + 1 for products of four or
 * more right-hand sides in precision dtype: shape[0], shape[1] = the
 * aggregation's right-hand sides per workgroup (0: the launcher's default)
 * and pipelined right-hand sides per pass (0: not pipelined; 4 counts as
 * 2); shape[2], shape[3] the same for the disaggregation, whose pipelined
 * passes count vectors (one component of one right-hand side: 1, 2 or 4); shape[4] = the aggregation's
 * children staged together (0: the launcher's default).  MLFMA_ERR_ARG for a
 * NULL handle or shape, an unknown dtype or a level out of range. */
int mlfma_tuning_level(mlfma_handle h, int dtype, int level, int shape[5]);

/*
 * Stage timing with HIP events recorded on the matvec's stream.  Stages:
 * 0 permute in, 1 near field, 2 radiation, 3 aggregation, 4 translation,
 * 5 disaggregation, 6 receive, 7 permute out.  mlfma_profile(h, 1) resets
 * the totals and records events around every stage of every later matvec;
 * mlfma_profile(h, 0) stops.  mlfma_profile_read waits for the recorded
 * events and returns per-stage totals in milliseconds (ms[8]) and the number
 * of profiled matvecs.
 */
enum { MLFMA_STAGES = 8 };
int mlfma_profile(mlfma_handle h, int enable);
int mlfma_profile_read(mlfma_handle h, double ms[8], long long *calls);

/*
 * Machine ceilings measured on the device (diagnostic; allocates and frees
 * its own buffers, synchronous): kind 0 = HBM bandwidth of a plain 1 GiB
 * copy in GB/s (read + write bytes), kind 1 = FP32 matrix-core rate of
 * v_mfma_f32_16x16x4f32 in TFLOP/s, kind 2 = FP32 vector fused
 * multiply-add rate (non-packed instructions, as the library's kernels are
 * built) in TFLOP/s.  device < 0: the current device.  These are the
 * measured ceilings beside the published ones that the stages' roofline
 * fractions are stated against.  Errors: MLFMA_ERR_ARG, MLFMA_ERR_OOM,
 * MLFMA_ERR_HIP (mlfma_last_error is not set).
 */
int mlfma_peak_probe(int kind, int device, double *value);

/* Text of the last error of the calling thread ("" if none; library
 * housekeeping). */
const char *mlfma_last_error(void);

/*
 * Host utility (no device use): the diagonal translation operator
 * T_L(khat, X) = sum_{l=0..L} (-j)^l (2l+1) h_l^(2)(k|X|) P_l(khat . X/|X|)
 * for nk unit directions khat (nk x 3), written as nk complex (re, im) pairs.
 * With it exp(-jk|X+d|)/(4 pi |X+d|) = -jk/(16 pi^2) Int exp(-jk khat.d) T_L dOmega
 * for |d| < |X| (the plane-wave expansion MLFMA is built on).
 */
int mlfma_translation_operator(double k, int L, const double X[3], long long nk, const double *khat,
                               double *out);

#ifdef __cplusplus
}
#endif
#endif
