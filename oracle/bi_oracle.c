/*
 * bi_oracle.c -- plain, slow, dense CPU reference for the boundary-integral
 * (BI) block of the coupled HDG-BI method (arXiv 2210.04892).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file; only tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU path.
 *
 * What it computes (all in complex double, time convention e^{+j w t},
 * Green's function G = exp(-jkR)/(4 pi R), lambda-normalised fields so that
 * the EFIE operator carries -jk and the MFIE operator carries 1):
 *
 *   L{X}(r) = -jk Int [I + grad div / k^2] X(r') G(r,r') ds'      (Sec. II-C, BI)
 *   K{X}(r) =      Int grad G(r,r') x X(r') ds'                   (Sec. II-C, BI)
 *
 * Galerkin-tested with RWG functions f_m on the closed surface (Sec. II-C,
 * weak forms eqs. 32-33; expansions eqs. exp4-exp5).  Primitive matrices
 * (D = surface divergence, g_m = n x f_m with n the outward normal of the
 * TEST triangle):
 *
 *   T_mn  = <f_m, L f_n>      = -jk IntInt [f_m.f_n - D_m D_n / k^2] G
 *   K_mn  = <f_m, Kbar f_n>   =     IntInt f_m . (grad G x f_n)
 *   Tx_mn = <f_m, n x L f_n>  = -   IntInt g_m . [-jk f_n G - (j/k) D_n grad G]
 *   Kx_mn = <f_m, n x Kbar f_n> = - IntInt g_m . (grad G x f_n)
 *   Gram_mn = Int f_m . f_n,   Gx_mn = Int f_m . (n x f_n)
 *
 * (the divergence term of L is moved onto the test function by parts; Kbar is
 * the principal value, whose coincident-triangle contribution vanishes for
 * flat triangles).  Two outputs:
 *
 *   op EM (Stratton-Chu pair, eqs. 22a/b and EFIE/MFIE eqs. 24a/b):
 *       y_E = T xJ - K xM,   y_H = T xM + K xJ
 *   op C  (the BI block C of eq. 42, entries eqs. 43-46, alpha = 1/2):
 *       C^JJ = Gram - T/2 - Kx/2      C^JM = Gx/2 - Tx/2 + K/2
 *       C^MJ = Tx/2 - K/2             C^MM = Gram/2 - T/2 - Kx/2
 *
 * Quadrature: triangle pairs that share no vertex use the 7-point degree-5
 * rule on both triangles (this defines the discrete matrix for them); pairs
 * that share a vertex, an edge or the whole triangle use Duffy-type
 * relative-coordinate transformations that remove the 1/R and 1/R^2
 * singularities, followed by tensor Gauss-Legendre rules of order q per
 * dimension, converged far below 1e-12.
 *
 * RWG convention (the paper only says "pairs of triangles"): edge (a,b) with
 * a < b; RWG index = rank of (a,b) in lexicographic order; T+ is the triangle
 * in which the directed edge a->b appears in counter-clockwise order, T- the
 * other; f = (l/2A+)(r - p+) on T+ and (l/2A-)(p- - r) on T-.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef double complex cplx;

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_MESH (-2)
#define ORC_ERR_QUAD (-3)

/* relative agreement of two successive orders that ends the order search */
#define AUTO_TOL 3e-11

/* ---------------------------------------------------------------- vectors */
static void vsub(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static double vdot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void vcross(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double vnorm(const double *a) { return sqrt(vdot(a, a)); }

/* ------------------------------------------------------------------- mesh */
typedef struct {
    int nv, nt, n;          /* vertices, triangles, RWG functions           */
    const double *v;        /* nv x 3                                       */
    const int *t;           /* nt x 3                                       */
    int *ea, *eb;           /* RWG n: edge endpoints, ea < eb               */
    int *tp, *tm;           /* RWG n: T+ and T- triangle                    */
    int *tri_rwg;           /* nt x 3: RWG on the edge opposite local vertex */
    double *tri_sgn;        /* nt x 3: +1 on T+, -1 on T-                   */
    double *area;           /* nt                                           */
    double *nrm;            /* nt x 3 unit outward normal                   */
    double *len;            /* n: edge length                               */
} mesh_t;

static void mesh_free(mesh_t *m)
{
    free(m->ea); free(m->eb); free(m->tp); free(m->tm);
    free(m->tri_rwg); free(m->tri_sgn); free(m->area); free(m->nrm); free(m->len);
}

typedef struct { int a, b, tri, loc, dir; } half_edge;

static int cmp_half(const void *x, const void *y)
{
    const half_edge *p = x, *q = y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    return p->dir > q->dir ? -1 : (p->dir < q->dir ? 1 : 0);
}

/* Build the RWG table; reject open, non-manifold, inconsistently oriented,
 * inward-oriented or degenerate meshes. */
static int mesh_build(mesh_t *m, int nv, const double *v, int nt, const int *t)
{
    memset(m, 0, sizeof(*m));
    m->nv = nv; m->nt = nt; m->v = v; m->t = t;
    if (nv < 4 || nt < 4) return ORC_ERR_MESH;
    m->area = malloc(sizeof(double) * nt);
    m->nrm = malloc(sizeof(double) * 3 * nt);
    double maxa = 0.0;
    for (int i = 0; i < nt; i++) {
        for (int c = 0; c < 3; c++)
            if (t[3 * i + c] < 0 || t[3 * i + c] >= nv) return ORC_ERR_MESH;
        const double *p0 = v + 3 * t[3 * i], *p1 = v + 3 * t[3 * i + 1], *p2 = v + 3 * t[3 * i + 2];
        double e1[3], e2[3], c[3];
        vsub(p1, p0, e1); vsub(p2, p0, e2); vcross(e1, e2, c);
        double a2 = vnorm(c);
        m->area[i] = 0.5 * a2;
        if (m->area[i] > maxa) maxa = m->area[i];
        for (int k = 0; k < 3; k++) m->nrm[3 * i + k] = a2 > 0 ? c[k] / a2 : 0.0;
    }
    for (int i = 0; i < nt; i++)
        if (!(m->area[i] > 1e-12 * maxa)) return ORC_ERR_MESH;

    half_edge *h = malloc(sizeof(half_edge) * 3 * nt);
    for (int i = 0; i < nt; i++)
        for (int j = 0; j < 3; j++) {
            int p = t[3 * i + (j + 1) % 3], q = t[3 * i + (j + 2) % 3];   /* edge opposite vertex j, CCW */
            half_edge *e = &h[3 * i + j];
            e->tri = i; e->loc = j;
            if (p < q) { e->a = p; e->b = q; e->dir = 1; } else { e->a = q; e->b = p; e->dir = -1; }
        }
    qsort(h, 3 * (size_t)nt, sizeof(half_edge), cmp_half);
    if ((3 * nt) % 2) { free(h); return ORC_ERR_MESH; }
    int n = 3 * nt / 2;
    m->n = n;
    m->ea = malloc(sizeof(int) * n); m->eb = malloc(sizeof(int) * n);
    m->tp = malloc(sizeof(int) * n); m->tm = malloc(sizeof(int) * n);
    m->len = malloc(sizeof(double) * n);
    m->tri_rwg = malloc(sizeof(int) * 3 * nt);
    m->tri_sgn = malloc(sizeof(double) * 3 * nt);
    for (int r = 0; r < n; r++) {
        half_edge *p = &h[2 * r], *q = &h[2 * r + 1];
        if (p->a != q->a || p->b != q->b) { free(h); return ORC_ERR_MESH; }
        if (r > 0 && h[2 * r - 1].a == p->a && h[2 * r - 1].b == p->b) { free(h); return ORC_ERR_MESH; }
        if (!(p->dir == 1 && q->dir == -1)) { free(h); return ORC_ERR_MESH; }
        m->ea[r] = p->a; m->eb[r] = p->b;
        m->tp[r] = p->tri; m->tm[r] = q->tri;
        double d[3];
        vsub(v + 3 * p->b, v + 3 * p->a, d);
        m->len[r] = vnorm(d);
        m->tri_rwg[3 * p->tri + p->loc] = r; m->tri_sgn[3 * p->tri + p->loc] = 1.0;
        m->tri_rwg[3 * q->tri + q->loc] = r; m->tri_sgn[3 * q->tri + q->loc] = -1.0;
    }
    free(h);
    /* Several disconnected scatterers may share one surface mesh (the BI
     * equations then hold on each closed surface, Sec. II-E remarks): every
     * connected surface must enclose a positive volume (outward normals).
     * Connected pieces are found by joining the two triangles of each RWG. */
    int *root = malloc(sizeof(int) * nt);
    double *vol6 = calloc(nt, sizeof(double));
    for (int i = 0; i < nt; i++) root[i] = i;
    for (int r = 0; r < n; r++) {
        int a = m->tp[r], b = m->tm[r];
        while (root[a] != a) { root[a] = root[root[a]]; a = root[a]; }
        while (root[b] != b) { root[b] = root[root[b]]; b = root[b]; }
        if (a != b) root[a < b ? b : a] = a < b ? a : b;
    }
    for (int i = 0; i < nt; i++) {
        int a = i;
        while (root[a] != a) { root[a] = root[root[a]]; a = root[a]; }
        const double *p0 = v + 3 * t[3 * i], *p1 = v + 3 * t[3 * i + 1], *p2 = v + 3 * t[3 * i + 2];
        double pc[3];
        vcross(p1, p2, pc);
        vol6[a] += vdot(p0, pc);
    }
    int inward = 0;
    for (int i = 0; i < nt; i++)
        if (root[i] == i && !(vol6[i] > 0)) inward = 1;
    free(root);
    free(vol6);
    return inward ? ORC_ERR_MESH : ORC_OK;
}

/* coefficient of (r - p_j) for the RWG on local edge j of triangle i */
static double rwg_coef(const mesh_t *m, int i, int j)
{
    return m->tri_sgn[3 * i + j] * m->len[m->tri_rwg[3 * i + j]] / (2.0 * m->area[i]);
}

/* ------------------------------------------------------------ quadrature */
/* 7-point degree-5 rule on the triangle (Radon; tabulated by Dunavant). */
static void tri7(double bary[7][3], double w[7])
{
    const double s15 = sqrt(15.0);
    const double a = (6.0 - s15) / 21.0, b = (6.0 + s15) / 21.0;
    const double wa = (155.0 - s15) / 1200.0, wb = (155.0 + s15) / 1200.0;
    double pts[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3},
                        {a, a, 1 - 2 * a}, {a, 1 - 2 * a, a}, {1 - 2 * a, a, a},
                        {b, b, 1 - 2 * b}, {b, 1 - 2 * b, b}, {1 - 2 * b, b, b}};
    double ww[7] = {9.0 / 40, wa, wa, wa, wb, wb, wb};
    memcpy(bary, pts, sizeof(pts));
    memcpy(w, ww, sizeof(ww));
}

/* Gauss-Legendre nodes/weights on [0,1] by Newton iteration on P_n. */
static void gauss01(int n, double *x, double *w)
{
    for (int i = 0; i < n; i++) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);   /* = 2/((1-z^2)P'^2) / 2 */
    }
}

/* --------------------------------------------------------------- kernels */
/* kernel families: 0 = full Helmholtz G, 1 = static 1/(4 pi R),
 * 2 = radiating part sin(kR)/(4 pi R) (entire; used only by checks). */
enum { KER_FULL = 0, KER_STATIC = 1, KER_SIN = 2 };

/* G(R) and the scalar g1 with grad_r G = g1 * (r - r'). */
static void kernel_eval(int kind, double k, double R, cplx *G, cplx *g1)
{
    const double f = 1.0 / (4.0 * M_PI);
    if (kind == KER_FULL) {
        cplx e = cexp(-I * k * R);
        *G = f * e / R;
        *g1 = -f * (1.0 + I * k * R) * e / (R * R * R);
    } else if (kind == KER_STATIC) {
        *G = f / R;
        *g1 = -f / (R * R * R);
    } else {
        double kr = k * R;
        if (kr < 1e-3) {   /* series: sin(x)/x and (x cos x - sin x)/x^3 */
            double x2 = kr * kr;
            *G = f * k * (1.0 - x2 / 6.0 + x2 * x2 / 120.0);
            *g1 = f * k * k * k * (-1.0 / 3.0 + x2 / 30.0 - x2 * x2 / 840.0);
        } else {
            *G = f * sin(kr) / R;
            *g1 = f * (kr * cos(kr) - sin(kr)) / (R * R * R);
        }
    }
}

/*
 * Integrand of the four operators for local test edge i (free vertex p_i)
 * and local source edge j (free vertex q_j), without the RWG coefficients:
 *   a = x - p_i, b = y - q_j, divergences 2 and 2, g = n_t x a
 *   T : -jk [a.b - 4/k^2] G
 *   K : a . (gradG x b)
 *   Tx: -g . [-jk b G - (2j/k) gradG]
 *   Kx: -g . (gradG x b)
 * accumulated with weight wt into out[op][i][j].
 */
static void accumulate(const double *x, const double *y, const double P[3][3], const double Q[3][3],
                       const double *nt, int kind, double k, double wt, cplx out[4][3][3])
{
    double d[3];
    vsub(x, y, d);
    double R = vnorm(d);
    cplx G, g1;
    kernel_eval(kind, k, R, &G, &g1);
    cplx gG[3] = {g1 * d[0], g1 * d[1], g1 * d[2]};
    for (int i = 0; i < 3; i++) {
        double a[3], g[3];
        vsub(x, P[i], a);
        vcross(nt, a, g);
        for (int j = 0; j < 3; j++) {
            double b[3];
            vsub(y, Q[j], b);
            /* gradG x b */
            cplx c0 = gG[1] * b[2] - gG[2] * b[1];
            cplx c1 = gG[2] * b[0] - gG[0] * b[2];
            cplx c2 = gG[0] * b[1] - gG[1] * b[0];
            cplx tT = -I * k * (vdot(a, b) - 4.0 / (k * k)) * G;
            cplx tK = a[0] * c0 + a[1] * c1 + a[2] * c2;
            cplx gb = g[0] * b[0] + g[1] * b[1] + g[2] * b[2];
            cplx ggG = g[0] * gG[0] + g[1] * gG[1] + g[2] * gG[2];
            cplx tTx = -(-I * k * gb * G - (2.0 * I / k) * ggG);
            cplx tKx = -(g[0] * c0 + g[1] * c1 + g[2] * c2);
            out[0][i][j] += wt * tT;
            out[1][i][j] += wt * tK;
            out[2][i][j] += wt * tTx;
            out[3][i][j] += wt * tKx;
        }
    }
}

/* 7x7 product rule: the matrix definition for pairs that share no vertex. */
static void pair_regular(const double P[3][3], const double Q[3][3], double At, double As,
                         const double *nt, int kind, double k, cplx out[4][3][3])
{
    double bary[7][3], w[7];
    tri7(bary, w);
    for (int p = 0; p < 7; p++) {
        double x[3];
        for (int c = 0; c < 3; c++) x[c] = bary[p][0] * P[0][c] + bary[p][1] * P[1][c] + bary[p][2] * P[2][c];
        for (int q = 0; q < 7; q++) {
            double y[3];
            for (int c = 0; c < 3; c++) y[c] = bary[q][0] * Q[0][c] + bary[q][1] * Q[1][c] + bary[q][2] * Q[2][c];
            accumulate(x, y, P, Q, nt, kind, k, w[p] * At * w[q] * As, out);
        }
    }
}

/*
 * Pairs that share one vertex.  Reordered so that P[0] = Q[0] = v.  Each
 * triangle is written in collapsed coordinates around v:
 *   x = v + r1 [(1-a1)(P1-v) + a1 (P2-v)],   dx = 2At r1 dr1 da1
 *   y = v + r2 [(1-a2)(Q1-v) + a2 (Q2-v)],   dy = 2As r2 dr2 da2
 * and the square (r1, r2) is split on its diagonal: {r2 <= r1}: r1 = s,
 * r2 = s e and {r1 <= r2}: r2 = s, r1 = s e (Jacobian s).  In both pieces
 * |x - y| = s |V(e, a1, a2)| with |V| bounded away from zero, and the total
 * weight s^3 e cancels both the 1/R and 1/R^2 kernels.
 */
static void pair_vertex(const double P[3][3], const double Q[3][3], double At, double As,
                        const double *nt, int kind, double k, int nq, cplx out[4][3][3])
{
    double gx[64], gw[64];
    gauss01(nq, gx, gw);
    const double *v = P[0];
    double A1[3], A2[3], B1[3], B2[3];
    vsub(P[1], v, A1); vsub(P[2], v, A2); vsub(Q[1], v, B1); vsub(Q[2], v, B2);
    for (int piece = 0; piece < 2; piece++)
        for (int is = 0; is < nq; is++)
            for (int ie = 0; ie < nq; ie++) {
                double s = gx[is], e = gx[ie];
                double r1 = piece == 0 ? s : s * e;
                double r2 = piece == 0 ? s * e : s;
                double wse = gw[is] * gw[ie] * s * s * s * e;
                for (int i1 = 0; i1 < nq; i1++)
                    for (int i2 = 0; i2 < nq; i2++) {
                        double a1 = gx[i1], a2 = gx[i2], x[3], y[3];
                        for (int c = 0; c < 3; c++) {
                            x[c] = v[c] + r1 * ((1 - a1) * A1[c] + a1 * A2[c]);
                            y[c] = v[c] + r2 * ((1 - a2) * B1[c] + a2 * B2[c]);
                        }
                        accumulate(x, y, P, Q, nt, kind, k, wse * gw[i1] * gw[i2] * 4.0 * At * As, out);
                    }
            }
}

/*
 * Pairs that share an edge.  Reordered so that P = (v0, v1, a) and
 * Q = (v0, v1, b).  Each triangle is swept by segments from a point of the
 * shared edge to its apex:
 *   x = (1-ht)(v0 + st e) + ht a,   dx = 2At (1-ht) dst dht,  e = v1 - v0
 *   y = (1-hs)(v0 + ss e) + hs b,   dy = 2As (1-hs) dss dhs
 * The singular set is {ht = hs = 0, st = ss}.  Split on the sign of st - ss
 * (offset d >= 0 from the larger abscissa sg in [d, 1], written
 * sg = d + (1-d) tau), then split the cube of (d, ht, hs) into the three
 * pyramids on which one coordinate is the largest (that coordinate = u, the
 * others = u*e1, u*e2; Jacobian u^2).  |x - y| = u |V| with |V| bounded away
 * from zero, so u^2 cancels both kernels' singularities.
 */
static void pair_edge(const double P[3][3], const double Q[3][3], double At, double As,
                      const double *nt, int kind, double k, int nq, cplx out[4][3][3])
{
    double gx[64], gw[64];
    gauss01(nq, gx, gw);
    const double *v0 = P[0];
    double e[3];
    vsub(P[1], P[0], e);
    for (int order = 0; order < 2; order++)          /* 0: st >= ss, 1: ss >= st */
        for (int pyr = 0; pyr < 3; pyr++)            /* which of (d, ht, hs) is largest */
            for (int iu = 0; iu < nq; iu++)
                for (int i1 = 0; i1 < nq; i1++)
                    for (int i2 = 0; i2 < nq; i2++) {
                        double u = gx[iu], e1 = gx[i1], e2 = gx[i2];
                        double d, ht, hs;
                        if (pyr == 0) { d = u; ht = u * e1; hs = u * e2; }
                        else if (pyr == 1) { ht = u; d = u * e1; hs = u * e2; }
                        else { hs = u; d = u * e1; ht = u * e2; }
                        double w3 = gw[iu] * gw[i1] * gw[i2] * u * u;
                        for (int it = 0; it < nq; it++) {
                            double tau = gx[it];
                            double sg = d + (1.0 - d) * tau;
                            double st = order == 0 ? sg : sg - d;
                            double ss = order == 0 ? sg - d : sg;
                            double x[3], y[3];
                            for (int c = 0; c < 3; c++) {
                                x[c] = (1 - ht) * (v0[c] + st * e[c]) + ht * P[2][c];
                                y[c] = (1 - hs) * (v0[c] + ss * e[c]) + hs * Q[2][c];
                            }
                            double wt = w3 * gw[it] * (1.0 - d) * (1.0 - ht) * (1.0 - hs) * 4.0 * At * As;
                            accumulate(x, y, P, Q, nt, kind, k, wt, out);
                        }
                    }
}

/*
 * Coincident pair.  Parameter coordinates x = P0 + x1 (P1-P0) + x2 (P2-P1)
 * on S = {0 <= x2 <= x1 <= 1} (Jacobian 2A).  The difference z = y - x ranges
 * over the hexagon S - S; for z = u w with w on hexagon edge i,
 * w = a_i(e) - b_i(e) with a_i, b_i on the boundary of S, the admissible x form
 * the shrunk copy (1-u) S + u b_i, i.e. x = (1-u) s + u b_i, y = (1-u) s + u a_i
 * with s in S.  Jacobian: u (hexagon polar) * (1-u)^2 * t1 (s = (t1, t1 t2)).
 * Hexagon edges i and i+3 are the same points with x and y exchanged; they are
 * evaluated together so that the odd 1/R^2 part of grad G cancels pointwise.
 */
static void pair_coincident(const double P[3][3], double At, const double *nt, int kind, double k, int nq,
                            cplx out[4][3][3])
{
    double gx[64], gw[64];
    gauss01(nq, gx, gw);
    double E1[3], E2[3];
    vsub(P[1], P[0], E1);
    vsub(P[2], P[1], E2);
    for (int edge = 0; edge < 3; edge++)
        for (int iu = 0; iu < nq; iu++)
            for (int ie = 0; ie < nq; ie++) {
                double u = gx[iu], e = gx[ie];
                double a[2], b[2];     /* the pair (a, b) of hexagon edge 0, 1 or 2 */
                if (edge == 0) { a[0] = 1; a[1] = e; b[0] = 0; b[1] = 0; }
                else if (edge == 1) { a[0] = 1; a[1] = 1; b[0] = e; b[1] = 0; }
                else { a[0] = 1 - e; a[1] = 1 - e; b[0] = 1; b[1] = 0; }
                double w2 = gw[iu] * gw[ie] * u * (1 - u) * (1 - u);
                for (int i1 = 0; i1 < nq; i1++)
                    for (int i2 = 0; i2 < nq; i2++) {
                        double t1 = gx[i1], t2 = gx[i2];
                        double s0 = t1, s1 = t1 * t2;
                        double xp0 = (1 - u) * s0 + u * b[0], xp1 = (1 - u) * s1 + u * b[1];
                        double yp0 = (1 - u) * s0 + u * a[0], yp1 = (1 - u) * s1 + u * a[1];
                        double x[3], y[3];
                        for (int c = 0; c < 3; c++) {
                            x[c] = P[0][c] + xp0 * E1[c] + xp1 * E2[c];
                            y[c] = P[0][c] + yp0 * E1[c] + yp1 * E2[c];
                        }
                        double wt = w2 * gw[i1] * gw[i2] * t1 * 4.0 * At * At;
                        accumulate(x, y, P, P, nt, kind, k, wt, out);   /* hexagon edge i   */
                        accumulate(y, x, P, P, nt, kind, k, wt, out);   /* hexagon edge i+3 */
                    }
            }
    /* K and Kx vanish identically on a flat triangle: (x-y) x f_n is normal
     * to the triangle while f_m and n x f_m are tangential. */
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) { out[1][i][j] = 0; out[3][i][j] = 0; }
}

/*
 * Local 4x3x3 integrals for test triangle (vertex ids ti, coords P) and
 * source triangle (ids si, coords Q).  out[op][i][j]: op 0..3 = T, K, Tx, Kx;
 * i / j = local edge opposite vertex i of the test / j of the source triangle
 * in the CALLER's vertex order.
 */
static void pair_integrals(const int ti[3], const double Praw[3][3], const int si[3], const double Qraw[3][3],
                           const double *nt, int kind, double k, int nq, cplx out[4][3][3])
{
    double At, As;
    {
        double e1[3], e2[3], c[3];
        vsub(Praw[1], Praw[0], e1); vsub(Praw[2], Praw[0], e2); vcross(e1, e2, c); At = 0.5 * vnorm(c);
        vsub(Qraw[1], Qraw[0], e1); vsub(Qraw[2], Qraw[0], e2); vcross(e1, e2, c); As = 0.5 * vnorm(c);
    }
    for (int o = 0; o < 4; o++)
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) out[o][i][j] = 0;
    int shared = 0, sp[3], sq[3];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            if (ti[i] == si[j]) { sp[shared] = i; sq[shared] = j; shared++; }
    if (shared == 0) {
        pair_regular(Praw, Qraw, At, As, nt, kind, k, out);
        return;
    }
    /* permutations pp / qq: new local index -> caller's local index */
    int pp[3], qq[3];
    if (shared == 3) {
        for (int i = 0; i < 3; i++) { pp[i] = i; }
        /* source order must match the test order vertex by vertex */
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++)
                if (si[j] == ti[i]) qq[i] = j;
    } else if (shared == 2) {
        pp[0] = sp[0]; pp[1] = sp[1]; pp[2] = 3 - sp[0] - sp[1];
        qq[0] = sq[0]; qq[1] = sq[1]; qq[2] = 3 - sq[0] - sq[1];
    } else {
        pp[0] = sp[0]; pp[1] = (sp[0] + 1) % 3; pp[2] = (sp[0] + 2) % 3;
        qq[0] = sq[0]; qq[1] = (sq[0] + 1) % 3; qq[2] = (sq[0] + 2) % 3;
    }
    double P[3][3], Q[3][3];
    for (int i = 0; i < 3; i++)
        for (int c = 0; c < 3; c++) { P[i][c] = Praw[pp[i]][c]; Q[i][c] = Qraw[qq[i]][c]; }
    cplx loc[4][3][3];
    memset(loc, 0, sizeof(loc));
    if (shared == 3) pair_coincident(P, At, nt, kind, k, nq, loc);
    else if (shared == 2) pair_edge(P, Q, At, As, nt, kind, k, nq, loc);
    else pair_vertex(P, Q, At, As, nt, kind, k, nq, loc);
    for (int o = 0; o < 4; o++)
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) out[o][pp[i]][qq[j]] = loc[o][i][j];
}

/*
 * Touching pairs with an a-posteriori order check: orders 10, 13, 16, ... are
 * tried until two successive results agree to tol relative to the largest
 * entry of the pair (the last, higher-order result is returned).  With
 * the exponential convergence of the transformed integrands the returned
 * value is then accurate to a small fraction of tol.
 */
static int pair_integrals_auto(const int ti[3], const double P[3][3], const int si[3], const double Q[3][3],
                               const double *nt, int kind, double k, double tol, cplx out[4][3][3])
{
    cplx prev[4][3][3];
    pair_integrals(ti, P, si, Q, nt, kind, k, 10, prev);
    int touching = 0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) touching |= ti[i] == si[j];
    if (!touching) { memcpy(out, prev, sizeof(prev)); return 0; }
    for (int nq = 13; nq <= 49; nq += 3) {
        pair_integrals(ti, P, si, Q, nt, kind, k, nq, out);
        /* one scale for the four operators: they enter the products of
         * eqs. 22-24 and 43-46 side by side, so an error is judged against
         * the pair's largest entry (an operator that nearly vanishes, such as
         * K on almost coplanar triangles, only has a rounding floor) */
        double scale = 0, diff = 0;
        for (int o = 0; o < 4; o++)
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    if (cabs(out[o][i][j]) > scale) scale = cabs(out[o][i][j]);
                    if (cabs(out[o][i][j] - prev[o][i][j]) > diff) diff = cabs(out[o][i][j] - prev[o][i][j]);
                }
        if (diff <= tol * scale) return nq;
        memcpy(prev, out, sizeof(prev));
    }
    return -1;   /* not converged at order 48: result kept, caller is told */
}

/* ---------------------------------- touching pairs: singularity subtraction */
/*
 * Second, independent route for pairs that share a vertex, an edge or the
 * whole triangle.  The kernels are split into closed-form static parts and
 * smooth remainders (Taylor series of exp(-jkR) about R = 0):
 *
 *   G  = (1/4pi) [ R^-1 - (k^2/2) R + (k^4/24) R^3 ] + G_r
 *   g1 = -(1/4pi) [ R^-3 + (k^2/2) R^-1 - (k^4/8) R + (k^6/144) R^3 ] + g1_r
 *
 * (grad_x G = g1 (x - y); the parts removed are every odd power of R up to
 * R^3, so G_r and g1_r (x - y) are C^4 and C^5 at R = 0).  For a test point
 * x the source-triangle integrals of the static parts are closed forms of
 * the flat triangle (line integrals K_n = Int_edge R^n by their recursion,
 * surface integrals I_n = Int R^n and the vectors W_n = Int (y - x) R^n by
 * the divergence theorem in the plane of the triangle; Wilton et al. 1984,
 * Graglia 1993), the remainders are integrated by a Gauss product rule over
 * the source triangle.  Every operator of a triangle pair then needs only
 *   S0 = Int G,  S1 = Int (y - x) G,  V = Int g1 (x - y)  (= grad_x S0)
 * at the test point, because with b = y - q_j:
 *   Int b G = S1 + (x - q_j) S0,   Int grad G x b = V x (x - q_j).
 * The test-triangle integral uses Gauss rules on geometrically graded
 * intervals of sweep coordinates x = (1-h)(B0 + s (B1 - B0)) + h C, graded
 * towards the set the pair shares (the whole boundary for the coincident
 * pair, split into three sweeps from its edges to the centroid; the shared
 * edge; the shared vertex), where the static parts are not smooth.
 */

/* Closed-form integrals over the flat triangle Q for the point x:
 *   I[0..2] = Int R^-1, Int R, Int R^3
 *   W[0..3] = Int (y - x) R^n, n = -3 (principal value), -1, 1, 3. */
static void static_integrals(const double Q[3][3], const double *x, double In[3], double W[4][3])
{
    double e1[3], e2[3], nn[3];
    vsub(Q[1], Q[0], e1);
    vsub(Q[2], Q[0], e2);
    vcross(e1, e2, nn);
    double nl = vnorm(nn);
    for (int c = 0; c < 3; c++) nn[c] /= nl;
    double d[3];
    vsub(x, Q[0], d);
    const double h = vdot(d, nn), ah = fabs(h);
    double rho[3];
    for (int c = 0; c < 3; c++) rho[c] = x[c] - h * nn[c];
    double omega = 0, st_m1 = 0, st_1 = 0, st_3 = 0;
    double Mm1[3] = {0, 0, 0}, M1[3] = {0, 0, 0}, M3[3] = {0, 0, 0}, M5[3] = {0, 0, 0};
    for (int i = 0; i < 3; i++) {
        const double *A = Q[i], *B = Q[(i + 1) % 3];
        double l[3], m[3], ar[3], br[3];
        vsub(B, A, l);
        double len = vnorm(l);
        for (int c = 0; c < 3; c++) l[c] /= len;
        vcross(l, nn, m);                       /* outward in-plane normal of the edge */
        vsub(A, rho, ar);
        vsub(B, rho, br);
        const double t0 = vdot(ar, m), lm = vdot(ar, l), lp = vdot(br, l);
        const double R0sq = t0 * t0 + h * h;
        const double Rm = sqrt(lm * lm + R0sq), Rp = sqrt(lp * lp + R0sq);
        double Km1;
        if (lm >= 0) Km1 = log((Rp + lp) / (Rm + lm));
        else if (lp <= 0) Km1 = log((Rm - lm) / (Rp - lp));
        else Km1 = log((Rp + lp) * (Rm - lm) / R0sq);     /* projection inside the edge */
        const double R0K = R0sq > 0 ? R0sq * Km1 : 0.0;
        const double K1 = 0.5 * (R0K + lp * Rp - lm * Rm);
        const double K3 = 0.25 * (3.0 * R0sq * K1 + lp * Rp * Rp * Rp - lm * Rm * Rm * Rm);
        const double K5 = (5.0 * R0sq * K3 + lp * pow(Rp, 5) - lm * pow(Rm, 5)) / 6.0;
        if (t0 != 0) {
            omega += atan(t0 * lp / (R0sq + ah * Rp)) - atan(t0 * lm / (R0sq + ah * Rm));
            st_m1 += t0 * Km1;
        }
        st_1 += t0 * K1;
        st_3 += t0 * K3;
        for (int c = 0; c < 3; c++) {
            if (R0sq > 0 || !(lm < 0 && lp > 0)) Mm1[c] += m[c] * Km1;
            M1[c] += m[c] * K1;
            M3[c] += m[c] * K3;
            M5[c] += m[c] * K5;
        }
    }
    const double Im1 = st_m1 - ah * omega;
    const double I1 = (h * h * Im1 + st_1) / 3.0;
    const double I3 = (3.0 * h * h * I1 + st_3) / 5.0;
    const double sg = h > 0 ? 1.0 : (h < 0 ? -1.0 : 0.0);
    In[0] = Im1;
    In[1] = I1;
    In[2] = I3;
    for (int c = 0; c < 3; c++) {
        W[0][c] = -Mm1[c] - sg * omega * nn[c];
        W[1][c] = M1[c] - h * nn[c] * Im1;
        W[2][c] = M3[c] / 3.0 - h * nn[c] * I1;
        W[3][c] = M5[c] / 5.0 - h * nn[c] * I3;
    }
}

/* Remainders G_r(R) and g1_r(R) of the split above. */
static void kernel_remainder(double k, double R, cplx *Gr, cplx *g1r)
{
    const double f = 1.0 / (4.0 * M_PI);
    if (k * R < 2.0) {
        /* G = f sum (-jk)^n R^(n-1) / n!,  g1 = -f sum (-jk)^n (1-n)/n! R^(n-3),
         * without the terms n = 0, 2, 4 (G) and n = 0, 2, 4, 6 (g1) */
        cplx term = 1.0;     /* (-jk)^n / n! */
        cplx sG = 0, sg = 0;
        double Rp = 1.0 / (R * R * R);   /* R^(n-3) */
        for (int n = 0; n <= 60; n++) {
            if (n != 0 && n != 2 && n != 4) sG += term * Rp * R * R;
            if (n != 0 && n != 2 && n != 4 && n != 6) sg += term * (1.0 - n) * Rp;
            term *= -I * k / (n + 1);
            Rp *= R;
            if (n > 10 && cabs(term) * Rp * R * R < 1e-30) break;
        }
        *Gr = f * sG;
        *g1r = -f * sg;
    } else {
        const double k2 = k * k, k4 = k2 * k2, k6 = k4 * k2, R3 = R * R * R;
        cplx e = cexp(-I * k * R);
        *Gr = f * e / R - f * (1.0 / R - 0.5 * k2 * R + k4 / 24.0 * R3);
        *g1r = -f * (1.0 + I * k * R) * e / R3 + f * (1.0 / R3 + 0.5 * k2 / R - k4 / 8.0 * R + k6 / 144.0 * R3);
    }
}

/* Collapsed Gauss-Legendre product rule with n x n points on Q (exact for
 * polynomials of degree 2n - 2); returns the point count. */
static int tri_gauss_rule(const double Q[3][3], int n, double (*pts)[3], double *wts)
{
    double gx[64], gw[64];
    gauss01(n, gx, gw);
    double e1[3], e2[3], c[3];
    vsub(Q[1], Q[0], e1);
    vsub(Q[2], Q[0], e2);
    vcross(e1, e2, c);
    const double A2 = vnorm(c);
    int np = 0;
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++) {
            const double u = gx[a], v = gx[b];
            const double l1 = u * (1 - v), l2 = u * v;
            for (int cc = 0; cc < 3; cc++) pts[np][cc] = Q[0][cc] + l1 * e1[cc] + l2 * e2[cc];
            wts[np] = gw[a] * gw[b] * u * A2;
            np++;
        }
    return np;
}

/* Gauss rule on [0,1] over geometrically graded intervals: side 0 grades
 * towards 0, side 1 towards 1, side 2 towards both ends (halves), side 3 is
 * no grading (levels equal intervals).  Ratio sigma between neighbouring
 * interval lengths, n points each.  Returns the point count. */
static int graded_rule(int side, double sigma, int levels, int n, double *x, double *w)
{
    double gx[64], gw[64];
    gauss01(n, gx, gw);
    int np = 0;
    double br[130];
    int nb = 0;
    if (side == 3) {
        for (int i = 0; i <= levels; i++) br[nb++] = (double)i / levels;
    } else {
        const double span = side == 2 ? 0.5 : 1.0;
        double tmp[66];
        int nt = 0;
        tmp[nt++] = 0.0;
        for (int i = levels; i >= 1; i--) tmp[nt++] = span * pow(sigma, i);
        tmp[nt++] = span;
        if (side == 0 || side == 2) for (int i = 0; i < nt; i++) br[nb++] = tmp[i];
        if (side == 1) for (int i = nt - 1; i >= 0; i--) br[nb++] = 1.0 - tmp[i];
        if (side == 2) for (int i = nt - 2; i >= 0; i--) br[nb++] = 1.0 - tmp[i];
    }
    for (int b = 0; b + 1 < nb; b++) {
        const double a0 = br[b], len = br[b + 1] - br[b];
        if (len <= 0) continue;
        for (int i = 0; i < n; i++) {
            x[np] = a0 + len * gx[i];
            w[np] = len * gw[i];
            np++;
        }
    }
    return np;
}

/* Test-triangle rule: grading ratio sigma; towards the singular edge or
 * vertex (sweep coordinate h) `levels` intervals of n points; along the
 * sweep base (s) s_levels intervals towards each graded end of n_s points;
 * n_inner x n_inner points for the remainders on the source triangle. */
typedef struct { double sigma; int levels, n, n_inner, n_s, s_levels; } subtract_opts;

/* Accumulate the four operators' integrands at the test point x with weight
 * wt (local edges as in accumulate(): a = x - P_i, b = y - Q_j). */
static void accumulate_sub(const double *x, const double P[3][3], const double Q[3][3], const double *nt, double k,
                           double wt, int n_inner, cplx out[4][3][3])
{
    double Is[3], Ws[4][3];
    static_integrals(Q, x, Is, Ws);
    const double f = 1.0 / (4.0 * M_PI), k2 = k * k, k4 = k2 * k2, k6 = k4 * k2;
    cplx S0 = f * (Is[0] - 0.5 * k2 * Is[1] + k4 / 24.0 * Is[2]);
    cplx S1[3], V[3];
    for (int c = 0; c < 3; c++) {
        S1[c] = f * (Ws[1][c] - 0.5 * k2 * Ws[2][c] + k4 / 24.0 * Ws[3][c]);
        V[c] = f * (Ws[0][c] + 0.5 * k2 * Ws[1][c] - k4 / 8.0 * Ws[2][c] + k6 / 144.0 * Ws[3][c]);
    }
    /* smooth remainders by the Gauss rule on Q */
    double pts[64 * 64][3], wts[64 * 64];
    const int np = tri_gauss_rule(Q, n_inner, pts, wts);
    for (int q = 0; q < np; q++) {
        double d[3];
        vsub(pts[q], x, d);                   /* y - x */
        const double R = vnorm(d);
        cplx Gr, g1r;
        kernel_remainder(k, R, &Gr, &g1r);
        S0 += wts[q] * Gr;
        for (int c = 0; c < 3; c++) {
            S1[c] += wts[q] * d[c] * Gr;
            V[c] -= wts[q] * d[c] * g1r;       /* g1 (x - y) */
        }
    }
    for (int i = 0; i < 3; i++) {
        double a[3], g[3];
        vsub(x, P[i], a);
        vcross(nt, a, g);
        for (int j = 0; j < 3; j++) {
            double xq[3];
            vsub(x, Q[j], xq);
            cplx Bv[3], VxC[3];
            for (int c = 0; c < 3; c++) Bv[c] = S1[c] + xq[c] * S0;           /* Int b G */
            VxC[0] = V[1] * xq[2] - V[2] * xq[1];                              /* Int grad G x b */
            VxC[1] = V[2] * xq[0] - V[0] * xq[2];
            VxC[2] = V[0] * xq[1] - V[1] * xq[0];
            const cplx aB = a[0] * Bv[0] + a[1] * Bv[1] + a[2] * Bv[2];
            const cplx gB = g[0] * Bv[0] + g[1] * Bv[1] + g[2] * Bv[2];
            const cplx gV = g[0] * V[0] + g[1] * V[1] + g[2] * V[2];
            const cplx aX = a[0] * VxC[0] + a[1] * VxC[1] + a[2] * VxC[2];
            const cplx gX = g[0] * VxC[0] + g[1] * VxC[1] + g[2] * VxC[2];
            out[0][i][j] += wt * (-I * k) * (aB - 4.0 / k2 * S0);
            out[1][i][j] += wt * aX;
            out[2][i][j] += wt * -(-I * k * gB - (2.0 * I / k) * gV);
            out[3][i][j] += wt * -gX;
        }
    }
}

/* Test-triangle integral over the sweep of base B0 -> B1 to apex C with the
 * given grading of s (along the base) and h (towards the apex). */
static void sweep_sub(const double B0[3], const double B1[3], const double C[3], int sside, int hside,
                      const subtract_opts *o, const double P[3][3], const double Q[3][3], const double *nt, double k,
                      cplx out[4][3][3])
{
    double sx[2048], sw[2048], hx[2048], hw[2048];
    /* the vertex sweep is smooth along its base: two plain intervals */
    const int ns = sside == 3 ? graded_rule(3, 0, 2, o->n_s, sx, sw)
                              : graded_rule(sside, o->sigma, o->s_levels, o->n_s, sx, sw);
    const int nh = graded_rule(hside, o->sigma, o->levels, o->n, hx, hw);
    double e1[3], e2[3], c[3];
    vsub(B1, B0, e1);
    vsub(C, B0, e2);
    vcross(e1, e2, c);
    const double A2 = vnorm(c);               /* twice the sweep's area */
    for (int a = 0; a < ns; a++)
        for (int b = 0; b < nh; b++) {
            const double s = sx[a], h = hx[b];
            double x[3];
            for (int cc = 0; cc < 3; cc++) x[cc] = (1 - h) * (B0[cc] + s * e1[cc]) + h * C[cc];
            accumulate_sub(x, P, Q, nt, k, sw[a] * hw[b] * (1 - h) * A2, o->n_inner, out);
        }
}

/* Defaults of the second route: agreement with the first route to about
 * 1e-13 of the pair's largest entry on the pins' meshes. */
static const subtract_opts SUB_DEFAULT = {0.35, 24, 10, 6, 8, 12};

/* T, K, Tx, Kx of a touching pair (caller's vertex order, as pair_integrals). */
static void pair_integrals_sub(const int ti[3], const double P[3][3], const int si[3], const double Q[3][3],
                               const double *nt, double k, const subtract_opts *o, cplx out[4][3][3])
{
    memset(out, 0, sizeof(cplx) * 36);
    int shared = 0, sp[3], sq[3];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            if (ti[i] == si[j]) { sp[shared] = i; sq[shared] = j; shared++; }
    (void)sq;
    if (shared == 3) {
        double cen[3];
        for (int c = 0; c < 3; c++) cen[c] = (P[0][c] + P[1][c] + P[2][c]) / 3.0;
        for (int e = 0; e < 3; e++) sweep_sub(P[e], P[(e + 1) % 3], cen, 2, 0, o, P, Q, nt, k, out);
        /* K and Kx vanish on a flat triangle (see pair_coincident) */
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) { out[1][i][j] = 0; out[3][i][j] = 0; }
    } else if (shared == 2) {
        const int third = 3 - sp[0] - sp[1];
        sweep_sub(P[sp[0]], P[sp[1]], P[third], 2, 0, o, P, Q, nt, k, out);
    } else if (shared == 1) {
        const int v = sp[0];
        sweep_sub(P[(v + 1) % 3], P[(v + 2) % 3], P[v], 3, 1, o, P, Q, nt, k, out);
    }
}

/* ------------------------------------------------------------- box rule */
/* Leaf box of every RWG (centre = edge midpoint): root cube centred on the
 * vertex bounding box, edge leaf * 2^(levels-1), levels = ceil(log2(extent /
 * leaf)) + 1; integer coordinates floor((c - origin) / leaf), clamped. */
static int leaf_boxes(const mesh_t *m, double leaf, int *levels_out, int *coords)
{
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int i = 0; i < m->nv; i++)
        for (int c = 0; c < 3; c++) {
            double x = m->v[3 * i + c];
            if (x < lo[c]) lo[c] = x;
            if (x > hi[c]) hi[c] = x;
        }
    double extent = 0;
    for (int c = 0; c < 3; c++) if (hi[c] - lo[c] > extent) extent = hi[c] - lo[c];
    int levels = (int)ceil(log2(extent / leaf)) + 1;
    if (levels < 1) levels = 1;
    double side = leaf * ldexp(1.0, levels - 1);
    int nb = 1 << (levels - 1);
    for (int r = 0; r < m->n; r++)
        for (int c = 0; c < 3; c++) {
            double centre = 0.5 * (lo[c] + hi[c]);
            double origin = centre - 0.5 * side;
            double mid = 0.5 * (m->v[3 * m->ea[r] + c] + m->v[3 * m->eb[r] + c]);
            int b = (int)floor((mid - origin) / leaf);
            if (b < 0) b = 0;
            if (b > nb - 1) b = nb - 1;
            coords[3 * r + c] = b;
        }
    *levels_out = levels;
    return ORC_OK;
}

/* class of the RWG pair (m, n): 0 = near (leaf boxes at Chebyshev distance
 * <= 1), otherwise the level l >= 2 at which their boxes first become
 * well separated (Chebyshev distance >= 2 while the parents are adjacent). */
static int pair_class(const int *coords, int levels, int a, int b)
{
    if (!coords || levels < 3) return 0;
    int leafl = levels - 1;
    for (int l = 2; l <= leafl; l++) {
        int sh = leafl - l, far = 0;
        for (int c = 0; c < 3; c++) {
            int d = (coords[3 * a + c] >> sh) - (coords[3 * b + c] >> sh);
            if (d > 1 || d < -1) far = 1;
        }
        if (far) return l;
    }
    return 0;
}

/* ------------------------------------------------------------ public API */
int oracle_rwg(int nv, const double *v, int nt, const int *t, int *edges, int *tri_pm)
{
    mesh_t m;
    int rc = mesh_build(&m, nv, v, nt, t);
    if (rc == ORC_OK) {
        for (int r = 0; r < m.n; r++) {
            if (edges) { edges[2 * r] = m.ea[r]; edges[2 * r + 1] = m.eb[r]; }
            if (tri_pm) { tri_pm[2 * r] = m.tp[r]; tri_pm[2 * r + 1] = m.tm[r]; }
        }
        rc = m.n;
    }
    mesh_free(&m);
    return rc;
}

/* Raw local integrals of one triangle pair (tests of the quadrature). */
int oracle_pair(const int *ti, const double *P, const int *si, const double *Q, int kind, double k, int nq,
                double *out /* 4 x 3 x 3 complex, interleaved re/im */)
{
    if (nq > 64) return ORC_ERR_ARG;
    double Pm[3][3], Qm[3][3], nt[3];
    memcpy(Pm, P, sizeof(Pm));
    memcpy(Qm, Q, sizeof(Qm));
    double e1[3], e2[3], c[3];
    vsub(Pm[1], Pm[0], e1); vsub(Pm[2], Pm[0], e2); vcross(e1, e2, c);
    double a2 = vnorm(c);
    for (int i = 0; i < 3; i++) nt[i] = c[i] / a2;
    cplx o[4][3][3];
    int used = nq;
    if (nq > 0) pair_integrals(ti, Pm, si, Qm, nt, kind, k, nq, o);
    else used = pair_integrals_auto(ti, Pm, si, Qm, nt, kind, k, AUTO_TOL, o);
    for (int q = 0; q < 36; q++) {
        out[2 * q] = creal(((cplx *)o)[q]);
        out[2 * q + 1] = cimag(((cplx *)o)[q]);
    }
    return used;
}

/* Raw local integrals of one touching pair by singularity subtraction
 * (the second route); params = {sigma, levels, n, n_inner, n_s}. */
int oracle_pair_sub(const int *ti, const double *P, const int *si, const double *Q, double k, const double *params,
                    double *out)
{
    subtract_opts o = {params[0], (int)params[1], (int)params[2], (int)params[3], (int)params[4], (int)params[5]};
    if (o.n < 1 || o.n > 64 || o.n_inner < 1 || o.n_inner > 64 || o.levels < 1 || o.levels > 60 || o.n_s < 1 ||
        o.n_s > 64 || o.s_levels < 1 || o.s_levels > 60 || (o.levels + 2) * 2 * o.n > 2048 ||
        (o.s_levels + 2) * 2 * o.n_s > 2048 || !(o.sigma > 0 && o.sigma < 1))
        return ORC_ERR_ARG;
    double Pm[3][3], Qm[3][3], nt[3];
    memcpy(Pm, P, sizeof(Pm));
    memcpy(Qm, Q, sizeof(Qm));
    double e1[3], e2[3], c[3];
    vsub(Pm[1], Pm[0], e1); vsub(Pm[2], Pm[0], e2); vcross(e1, e2, c);
    double a2 = vnorm(c);
    for (int i = 0; i < 3; i++) nt[i] = c[i] / a2;
    cplx o4[4][3][3];
    pair_integrals_sub(ti, Pm, si, Qm, nt, k, &o, o4);
    for (int q = 0; q < 36; q++) {
        out[2 * q] = creal(((cplx *)o4)[q]);
        out[2 * q + 1] = cimag(((cplx *)o4)[q]);
    }
    return ORC_OK;
}

/*
 * Dense Galerkin products, by classes.
 *   x    : 2N x nrhs column-major complex (interleaved), rows [0,N) = J
 *          (or E-side) coefficients, [N,2N) = M.
 *   rows : test RWG indices (0..N-1) to evaluate, or NULL for all N;
 *          nrows entries.
 *   y    : ncls blocks, each (2*nrows) x nrhs column-major complex; block c
 *          holds class c; block rows [0,nrows) = J/E-tested, [nrows,2nrows)
 *          = M/H-tested, in the order of `rows`.
 *   op   : 0 = C block (eqs. 43-46), 1 = EM pair (eqs. 22, 24),
 *          2..7 = single primitive matrix applied to the J half of x only
 *          (T, K, Tx, Kx, Gram, Gx), written to the J half of y,
 *          8 = both 0 and 1 (y then holds 2*ncls blocks: op C, then op EM).
 *   leaf : leaf box edge (> 0 enables classes: class 0 = near, class l =
 *          interaction level l; ncls must be >= levels), or <= 0 (ncls = 1).
 *   nq   : Gauss order per dimension for touching pairs, 0 for the order
 *          search of pair_integrals_auto (the default), or -1 for the
 *          second route (singularity subtraction, pair_integrals_sub).
 *   Source triangles on which every RWG coefficient of x is zero add
 *   nothing and are skipped.
 *   Returns ORC_ERR_QUAD if some touching pair did not converge.
 */
int oracle_matvec(int nv, const double *v, int nt, const int *t, double k, int op, int nrhs,
                  const double *x_in, const int *rows, int nrows, double *y_out, double leaf, int ncls, int nq)
{
    if (nrhs < 1 || k <= 0 || nq < -1 || nq > 64 || op < 0 || op > 8) return ORC_ERR_ARG;
    int quad_fail = 0;
    mesh_t m;
    int rc = mesh_build(&m, nv, v, nt, t);
    if (rc != ORC_OK) { mesh_free(&m); return rc; }
    const int N = m.n;
    int *coords = NULL, levels = 0;
    if (leaf > 0) {
        coords = malloc(sizeof(int) * 3 * N);
        leaf_boxes(&m, leaf, &levels, coords);
        if (ncls < levels) { free(coords); mesh_free(&m); return ORC_ERR_ARG; }
    } else if (ncls < 1) { mesh_free(&m); return ORC_ERR_ARG; }
    const cplx *x = (const cplx *)x_in;
    cplx *y = (cplx *)y_out;
    int nr = rows ? nrows : N;
    /* position of each requested RWG in the output */
    int *outpos = malloc(sizeof(int) * N);
    for (int r = 0; r < N; r++) outpos[r] = -1;
    for (int r = 0; r < nr; r++) {
        int g = rows ? rows[r] : r;
        if (g < 0 || g >= N) { free(outpos); free(coords); mesh_free(&m); return ORC_ERR_ARG; }
        outpos[g] = r;
    }
    memset(y, 0, sizeof(cplx) * (size_t)(op == 8 ? 2 : 1) * ncls * 2 * nr * nrhs);
    /* test triangles touching a requested row */
    char *need = calloc(nt, 1);
    for (int r = 0; r < N; r++)
        if (outpos[r] >= 0) { need[m.tp[r]] = 1; need[m.tm[r]] = 1; }
    /* source triangles that carry a non-zero coefficient */
    char *active = calloc(nt, 1);
    for (int r = 0; r < N; r++) {
        int nz = 0;
        for (int h = 0; h < 2 && !nz; h++)
            for (int q = 0; q < nrhs && !nz; q++) nz = x[(size_t)q * 2 * N + (size_t)h * N + r] != 0;
        if (nz) { active[m.tp[r]] = 1; active[m.tm[r]] = 1; }
    }

    /* per output row: acc[cls][opnd(4)][xhalf(2)][rhs] -- gathered per test
     * triangle, then combined into y.  Work per test triangle is private. */
    const size_t accsz = (size_t)ncls * 4 * 2 * nrhs;
    cplx *acc_all = calloc((size_t)nr * accsz, sizeof(cplx));   /* indexed by output row */
    omp_lock_t *locks = malloc(sizeof(omp_lock_t) * nr);
    for (int r = 0; r < nr; r++) omp_init_lock(&locks[r]);

#pragma omp parallel
    {
        cplx *part = malloc(sizeof(cplx) * 3 * accsz);
#pragma omp for schedule(dynamic, 1)
        for (int ti = 0; ti < nt; ti++) {
            if (!need[ti] || op == 6 || op == 7) continue;
            memset(part, 0, sizeof(cplx) * 3 * accsz);
            double P[3][3];
            int tv[3];
            for (int a = 0; a < 3; a++) {
                tv[a] = t[3 * ti + a];
                for (int c = 0; c < 3; c++) P[a][c] = v[3 * tv[a] + c];
            }
            for (int si = 0; si < nt; si++) {
                if (!active[si]) continue;
                double Q[3][3];
                int sv[3];
                for (int a = 0; a < 3; a++) {
                    sv[a] = t[3 * si + a];
                    for (int c = 0; c < 3; c++) Q[a][c] = v[3 * sv[a] + c];
                }
                cplx loc[4][3][3];
                int touch = 0;
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++) touch |= tv[a] == sv[b];
                if (nq < 0 && touch) pair_integrals_sub(tv, P, sv, Q, &m.nrm[3 * ti], k, &SUB_DEFAULT, loc);
                else if (nq > 0) pair_integrals(tv, P, sv, Q, &m.nrm[3 * ti], KER_FULL, k, nq, loc);
                else if (pair_integrals_auto(tv, P, sv, Q, &m.nrm[3 * ti], KER_FULL, k, AUTO_TOL, loc) < 0) {
#pragma omp atomic write
                    quad_fail = 1;
                }
                for (int i = 0; i < 3; i++) {
                    int mr = m.tri_rwg[3 * ti + i];
                    if (outpos[mr] < 0) continue;
                    double cm = rwg_coef(&m, ti, i);
                    for (int j = 0; j < 3; j++) {
                        int nr_ = m.tri_rwg[3 * si + j];
                        double cn = rwg_coef(&m, si, j);
                        int cls = pair_class(coords, levels, mr, nr_);
                        for (int o = 0; o < 4; o++) {
                            cplx val = cm * cn * loc[o][i][j];
                            cplx *dst = part + i * accsz + ((size_t)cls * 4 + o) * 2 * nrhs;
                            for (int h = 0; h < 2; h++)
                                for (int q = 0; q < nrhs; q++)
                                    dst[h * nrhs + q] += val * x[(size_t)q * 2 * N + (size_t)h * N + nr_];
                        }
                    }
                }
            }
            for (int i = 0; i < 3; i++) {
                int mr = m.tri_rwg[3 * ti + i];
                if (outpos[mr] < 0) continue;
                int orow = outpos[mr];
                omp_set_lock(&locks[orow]);
                cplx *dst = acc_all + (size_t)orow * accsz;
                for (size_t z = 0; z < accsz; z++) dst[z] += part[i * accsz + z];
                omp_unset_lock(&locks[orow]);
            }
        }
        free(part);
    }

    /* Gram and Gx: common triangles only; 7-point rule is exact (quadratic). */
    cplx *gram = calloc((size_t)nr * 2 * 2 * nrhs, sizeof(cplx));   /* [out row][Gram|Gx][xhalf][rhs] */
    {
        double bary[7][3], w[7];
        tri7(bary, w);
        for (int ti = 0; ti < nt; ti++) {
            if (!need[ti]) continue;
            const double *nn = &m.nrm[3 * ti];
            double P[3][3];
            for (int a = 0; a < 3; a++)
                for (int c = 0; c < 3; c++) P[a][c] = v[3 * t[3 * ti + a] + c];
            for (int i = 0; i < 3; i++) {
                int mr = m.tri_rwg[3 * ti + i];
                if (outpos[mr] < 0) continue;
                double cm = rwg_coef(&m, ti, i);
                for (int j = 0; j < 3; j++) {
                    int nr_ = m.tri_rwg[3 * ti + j];
                    double cn = rwg_coef(&m, ti, j);
                    double g = 0, gx = 0;
                    for (int p = 0; p < 7; p++) {
                        double r[3], a[3], b[3], nb[3];
                        for (int c = 0; c < 3; c++) r[c] = bary[p][0] * P[0][c] + bary[p][1] * P[1][c] + bary[p][2] * P[2][c];
                        vsub(r, P[i], a); vsub(r, P[j], b); vcross(nn, b, nb);
                        g += w[p] * m.area[ti] * vdot(a, b);
                        gx += w[p] * m.area[ti] * vdot(a, nb);
                    }
                    for (int h = 0; h < 2; h++)
                        for (int q = 0; q < nrhs; q++) {
                            cplx xv = x[(size_t)q * 2 * N + (size_t)h * N + nr_];
                            gram[(((size_t)outpos[mr] * 2 + 0) * 2 + h) * nrhs + q] += cm * cn * g * xv;
                            gram[(((size_t)outpos[mr] * 2 + 1) * 2 + h) * nrhs + q] += cm * cn * gx * xv;
                        }
                }
            }
        }
    }

    /* combine into the requested operator */
    for (int mr = 0; mr < N; mr++) {
        int r = outpos[mr];
        if (r < 0) continue;
        for (int pass = 0; pass < (op == 8 ? 2 : 1); pass++) {
            int o_ = op == 8 ? pass : op;
            for (int cls = 0; cls < ncls; cls++)
                for (int q = 0; q < nrhs; q++) {
#define A(o, h) acc_all[(size_t)r * accsz + (((size_t)cls * 4 + (o)) * 2 + (h)) * nrhs + q]
#define GR(g, h) (cls == 0 ? gram[(((size_t)r * 2 + (g)) * 2 + (h)) * nrhs + q] : 0)
                    cplx yJ, yM;
                    if (o_ == 0) {
                        yJ = GR(0, 0) - 0.5 * A(0, 0) - 0.5 * A(3, 0) + 0.5 * GR(1, 1) - 0.5 * A(2, 1) + 0.5 * A(1, 1);
                        yM = 0.5 * A(2, 0) - 0.5 * A(1, 0) + 0.5 * GR(0, 1) - 0.5 * A(0, 1) - 0.5 * A(3, 1);
                    } else if (o_ == 1) {
                        yJ = A(0, 0) - A(1, 1);
                        yM = A(0, 1) + A(1, 0);
                    } else if (o_ <= 5) {
                        yJ = A(o_ - 2, 0);
                        yM = 0;
                    } else {
                        yJ = GR(o_ - 6, 0);
                        yM = 0;
                    }
#undef A
#undef GR
                    size_t blk = (size_t)pass * ncls + cls;
                    y[(blk * nrhs + q) * 2 * nr + r] = yJ;
                    y[(blk * nrhs + q) * 2 * nr + nr + r] = yM;
                }
        }
    }
    for (int r = 0; r < nr; r++) omp_destroy_lock(&locks[r]);
    free(locks); free(acc_all); free(gram); free(need); free(active); free(outpos); free(coords);
    mesh_free(&m);
    return quad_fail ? ORC_ERR_QUAD : ORC_OK;
}

/*
 * Primitive matrix entries of explicit RWG pairs (test m, source n):
 * out[6 e + o] (complex, interleaved) = T, K, Tx, Kx, Gram, Gx of pair e, by
 * the same rules as oracle_matvec (7 x 7 points for triangle pairs sharing
 * no vertex, converged singular rules otherwise, 7-point Gram terms).  The
 * sum over the four triangle pairs of the two RWGs is written out here; the
 * product oracle sums the same local integrals in another order.
 */
int oracle_entries(int nv, const double *v, int nt, const int *t, double k, int npairs, const int *pairs,
                   double *out_)
{
    if (npairs < 0 || k <= 0) return ORC_ERR_ARG;
    mesh_t m;
    int rc = mesh_build(&m, nv, v, nt, t);
    if (rc != ORC_OK) { mesh_free(&m); return rc; }
    for (int e = 0; e < npairs; e++)
        if (pairs[2 * e] < 0 || pairs[2 * e] >= m.n || pairs[2 * e + 1] < 0 || pairs[2 * e + 1] >= m.n) {
            mesh_free(&m);
            return ORC_ERR_ARG;
        }
    cplx *out = (cplx *)out_;
    int quad_fail = 0;
    double bary[7][3], w[7];
    tri7(bary, w);
#pragma omp parallel for schedule(dynamic, 4)
    for (int e = 0; e < npairs; e++) {
        const int mr = pairs[2 * e], nr_ = pairs[2 * e + 1];
        const int ttri[2] = {m.tp[mr], m.tm[mr]}, stri[2] = {m.tp[nr_], m.tm[nr_]};
        cplx acc[6] = {0, 0, 0, 0, 0, 0};
        for (int a = 0; a < 2; a++) {
            const int ti = ttri[a];
            int i = 0;
            while (m.tri_rwg[3 * ti + i] != mr) i++;
            double P[3][3];
            int tv[3];
            for (int q = 0; q < 3; q++) {
                tv[q] = t[3 * ti + q];
                for (int c = 0; c < 3; c++) P[q][c] = v[3 * tv[q] + c];
            }
            const double cm = rwg_coef(&m, ti, i);
            for (int b = 0; b < 2; b++) {
                const int si = stri[b];
                int j = 0;
                while (m.tri_rwg[3 * si + j] != nr_) j++;
                double Q[3][3];
                int sv[3];
                for (int q = 0; q < 3; q++) {
                    sv[q] = t[3 * si + q];
                    for (int c = 0; c < 3; c++) Q[q][c] = v[3 * sv[q] + c];
                }
                const double cn = rwg_coef(&m, si, j);
                cplx loc[4][3][3];
                if (pair_integrals_auto(tv, P, sv, Q, &m.nrm[3 * ti], KER_FULL, k, AUTO_TOL, loc) < 0) {
#pragma omp atomic write
                    quad_fail = 1;
                }
                for (int o = 0; o < 4; o++) acc[o] += cm * cn * loc[o][i][j];
                if (ti == si) {          /* Gram and Gx: common triangle, exact 7-point rule */
                    const double *nn = &m.nrm[3 * ti];
                    double g = 0, gx = 0;
                    for (int p = 0; p < 7; p++) {
                        double r[3], x1[3], x2[3], nb[3];
                        for (int c = 0; c < 3; c++)
                            r[c] = bary[p][0] * P[0][c] + bary[p][1] * P[1][c] + bary[p][2] * P[2][c];
                        vsub(r, P[i], x1); vsub(r, P[j], x2); vcross(nn, x2, nb);
                        g += w[p] * m.area[ti] * vdot(x1, x2);
                        gx += w[p] * m.area[ti] * vdot(x1, nb);
                    }
                    acc[4] += cm * cn * g;
                    acc[5] += cm * cn * gx;
                }
            }
        }
        for (int o = 0; o < 6; o++) out[6 * (size_t)e + o] = acc[o];
    }
    mesh_free(&m);
    return quad_fail ? ORC_ERR_QUAD : ORC_OK;
}

/*
 * Right-hand sides of the coupled system for incident plane waves (eqs. 49,
 * 50): b^J_m = <f_m, E/2 + n x H/2>, b^M_m = <f_m, H/2 - n x E/2> with
 * E = p exp(-jk khat.r), H = khat x p exp(-jk khat.r) (the plane wave of
 * Sec. III with E0 = 1 in the normalised units), 7-point rule per triangle.
 * khat, pol: nrhs x 3 (unit vectors); out: 2N x nrhs column-major complex.
 */
int oracle_plane_wave_rhs(int nv, const double *v, int nt, const int *t, double k, int nrhs, const double *khat,
                          const double *pol, double *out)
{
    mesh_t m;
    int rc = mesh_build(&m, nv, v, nt, t);
    if (rc != ORC_OK) { mesh_free(&m); return rc; }
    const int N = m.n;
    cplx *b = (cplx *)out;
    memset(b, 0, sizeof(cplx) * 2 * (size_t)N * nrhs);
    double bary[7][3], w[7];
    tri7(bary, w);
    for (int q = 0; q < nrhs; q++) {
        const double *kh = khat + 3 * q, *p = pol + 3 * q;
        double h[3];
        vcross(kh, p, h);
        for (int ti = 0; ti < nt; ti++) {
            double P[3][3];
            for (int a = 0; a < 3; a++)
                for (int c = 0; c < 3; c++) P[a][c] = v[3 * t[3 * ti + a] + c];
            const double *nn = &m.nrm[3 * ti];
            double nxe[3], nxh[3];
            vcross(nn, p, nxe);
            vcross(nn, h, nxh);
            for (int i = 0; i < 3; i++) {
                int r = m.tri_rwg[3 * ti + i];
                double cm = rwg_coef(&m, ti, i);
                cplx bj = 0, bm = 0;
                for (int pt = 0; pt < 7; pt++) {
                    double x[3], a[3];
                    for (int c = 0; c < 3; c++) x[c] = bary[pt][0] * P[0][c] + bary[pt][1] * P[1][c] + bary[pt][2] * P[2][c];
                    vsub(x, P[i], a);
                    cplx ph = cexp(-I * k * vdot(kh, x)) * w[pt] * m.area[ti] * cm;
                    bj += ph * 0.5 * (vdot(a, p) + vdot(a, nxh));
                    bm += ph * 0.5 * (vdot(a, h) - vdot(a, nxe));
                }
                b[(size_t)q * 2 * N + r] += bj;
                b[(size_t)q * 2 * N + N + r] += bm;
            }
        }
    }
    mesh_free(&m);
    return ORC_OK;
}

/*
 * Far field of the surface currents J = sum_n xJ_n f_n, M = sum_n xM_n f_n
 * (the radar cross section of Sec. III is computed from it).  In the
 * normalised units of the operators above the field E = L{J} - K{M} behaves
 * far away as exp(-jkr)/r F(khat), with the plane-wave limits
 * L -> -jk (I - khat khat) and K -> -jk khat x:
 *
 *   F(khat) = (-jk / 4 pi) [ P_J - khat (khat . P_J) - khat x P_M ],
 *   P_X(khat) = Int X(r') exp(+jk khat . r') ds'   (7-point rule per triangle).
 *
 * Output: F . theta_hat and F . phi_hat of each direction khat (theta_hat =
 * (cos t cos p, cos t sin p, -sin t), phi_hat = (-sin p, cos p, 0) with
 * t = acos(khat_z), p = atan2(khat_y, khat_x)); x: 2N x nrhs column-major
 * (J rows then M rows); dirs: ndir x 3 unit vectors; out: ndir x 2 x nrhs
 * complex, row-major.  sigma = 4 pi |F|^2 for a unit incident field.
 */
int oracle_far_field(int nv, const double *v, int nt, const int *t, double k, int nrhs, const double *xin,
                     int ndir, const double *dirs, double *out)
{
    mesh_t m;
    int rc = mesh_build(&m, nv, v, nt, t);
    if (rc != ORC_OK) { mesh_free(&m); return rc; }
    const int N = m.n;
    const cplx *x = (const cplx *)xin;
    cplx *F = (cplx *)out;
    double bary[7][3], w[7];
    tri7(bary, w);
    for (int d = 0; d < ndir; d++)
        for (int q = 0; q < nrhs; q++) {
            const double *kh = dirs + 3 * d;
            cplx PJ[3] = {0, 0, 0}, PM[3] = {0, 0, 0};
            for (int ti = 0; ti < nt; ti++) {
                double P[3][3];
                for (int a = 0; a < 3; a++)
                    for (int c = 0; c < 3; c++) P[a][c] = v[3 * t[3 * ti + a] + c];
                for (int pt = 0; pt < 7; pt++) {
                    double r[3];
                    for (int c = 0; c < 3; c++) r[c] = bary[pt][0] * P[0][c] + bary[pt][1] * P[1][c] + bary[pt][2] * P[2][c];
                    const cplx ph = cexp(I * k * vdot(kh, r)) * w[pt] * m.area[ti];
                    for (int i = 0; i < 3; i++) {
                        const int n = m.tri_rwg[3 * ti + i];
                        const double cm = rwg_coef(&m, ti, i);
                        double a[3];
                        vsub(r, P[i], a);
                        const cplx xj = x[(size_t)q * 2 * N + n], xm = x[(size_t)q * 2 * N + N + n];
                        for (int c = 0; c < 3; c++) {
                            PJ[c] += ph * cm * a[c] * xj;
                            PM[c] += ph * cm * a[c] * xm;
                        }
                    }
                }
            }
            const cplx kpj = kh[0] * PJ[0] + kh[1] * PJ[1] + kh[2] * PJ[2];
            cplx Fv[3];
            Fv[0] = PJ[0] - kh[0] * kpj - (kh[1] * PM[2] - kh[2] * PM[1]);
            Fv[1] = PJ[1] - kh[1] * kpj - (kh[2] * PM[0] - kh[0] * PM[2]);
            Fv[2] = PJ[2] - kh[2] * kpj - (kh[0] * PM[1] - kh[1] * PM[0]);
            const double th = acos(fmax(-1.0, fmin(1.0, kh[2]))), phi = atan2(kh[1], kh[0]);
            const double tv[3] = {cos(th) * cos(phi), cos(th) * sin(phi), -sin(th)}, pv[3] = {-sin(phi), cos(phi), 0};
            const cplx pre = -I * k / (4 * M_PI);
            F[((size_t)d * 2 + 0) * nrhs + q] = pre * (Fv[0] * tv[0] + Fv[1] * tv[1] + Fv[2] * tv[2]);
            F[((size_t)d * 2 + 1) * nrhs + q] = pre * (Fv[0] * pv[0] + Fv[1] * pv[1] + Fv[2] * pv[2]);
        }
    mesh_free(&m);
    return ORC_OK;
}

/* Leaf-box coordinates and level count of the box rule (tests of the tree). */
int oracle_boxes(int nv, const double *v, int nt, const int *t, double leaf, int *coords, int *levels)
{
    mesh_t m;
    int rc = mesh_build(&m, nv, v, nt, t);
    if (rc == ORC_OK) rc = leaf_boxes(&m, leaf, levels, coords);
    mesh_free(&m);
    return rc;
}

int oracle_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------- interaction classes by box */
/* Open-addressing set of 64-bit keys (key + 1 stored, 0 = empty). */
typedef struct { unsigned long long *slot; size_t cap, n; } keyset;

static int keyset_add(keyset *s, unsigned long long key)
{
    if (2 * (s->n + 1) > s->cap) {
        size_t ncap = s->cap ? 2 * s->cap : 1024;
        unsigned long long *ns = calloc(ncap, sizeof(*ns));
        if (!ns) return ORC_ERR_ARG;
        for (size_t i = 0; i < s->cap; i++)
            if (s->slot[i]) {
                size_t h = (size_t)((s->slot[i] * 0x9E3779B97F4A7C15ULL) >> 7) & (ncap - 1);
                while (ns[h]) h = (h + 1) & (ncap - 1);
                ns[h] = s->slot[i];
            }
        free(s->slot);
        s->slot = ns;
        s->cap = ncap;
    }
    unsigned long long v = key + 1;
    size_t h = (size_t)((v * 0x9E3779B97F4A7C15ULL) >> 7) & (s->cap - 1);
    while (s->slot[h]) {
        if (s->slot[h] == v) return 0;
        h = (h + 1) & (s->cap - 1);
    }
    s->slot[h] = v;
    s->n++;
    return 1;
}

/* For every level l >= 2, the number of distinct ordered pairs of octree
 * boxes (A, B) at level l for which some RWG in A and some RWG in B have
 * interaction class l (pair_class above): the translations the MLFMA has to
 * make at that level.  counts[l] for l < levels (counts[0], counts[1] = 0).
 * Every RWG of one leaf box has the same class against any other RWG, so one
 * representative RWG per occupied leaf box is enough. */
int oracle_class_box_pairs(int nv, const double *v, int nt, const int *t, double leaf, long long *counts,
                           int max_levels)
{
    mesh_t m;
    int rc = mesh_build(&m, nv, v, nt, t);
    if (rc != ORC_OK) { mesh_free(&m); return rc; }
    int *coords = malloc(sizeof(int) * 3 * (size_t)m.n);
    int levels = 0;
    leaf_boxes(&m, leaf, &levels, coords);
    if (levels > max_levels) { free(coords); mesh_free(&m); return ORC_ERR_ARG; }
    for (int l = 0; l < max_levels; l++) counts[l] = 0;
    const int leafl = levels - 1;
    const long long nb = 1LL << leafl;
    /* one representative RWG per occupied leaf box */
    keyset seen = {0};
    int *rep = malloc(sizeof(int) * (size_t)m.n);
    int nrep = 0;
    for (int r = 0; r < m.n; r++) {
        unsigned long long key = ((unsigned long long)coords[3 * r] * nb + coords[3 * r + 1]) * nb + coords[3 * r + 2];
        if (keyset_add(&seen, key) == 1) rep[nrep++] = r;
    }
    free(seen.slot);
    keyset pairs[32];
    memset(pairs, 0, sizeof(pairs));
    for (int i = 0; i < nrep; i++)
        for (int j = 0; j < nrep; j++) {
            int cls = pair_class(coords, levels, rep[i], rep[j]);
            if (cls < 2) continue;
            int sh = leafl - cls;
            long long nl = 1LL << cls;
            const int *a = coords + 3 * rep[i], *b = coords + 3 * rep[j];
            unsigned long long ka = ((unsigned long long)(a[0] >> sh) * nl + (a[1] >> sh)) * nl + (a[2] >> sh);
            unsigned long long kb = ((unsigned long long)(b[0] >> sh) * nl + (b[1] >> sh)) * nl + (b[2] >> sh);
            keyset_add(&pairs[cls], ka * (unsigned long long)(nl * nl * nl) + kb);
        }
    for (int l = 2; l < levels && l < 32; l++) {
        counts[l] = (long long)pairs[l].n;
        free(pairs[l].slot);
    }
    free(rep);
    free(coords);
    mesh_free(&m);
    return levels;
}
