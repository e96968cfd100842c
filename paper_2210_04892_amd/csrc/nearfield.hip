// Double-precision set-up kernels: leaf radiation/receive patterns and the
// near-field blocks (regular triangle pairs by the 7-point rule on both
// triangles, touching pairs by singularity-cancelling transformations of the
// 4-D integral followed by tensor Gauss-Legendre rules).
#include "nearfield.hpp"

namespace mlfma {

// Radon's 7-point degree-5 rule: barycentric points and weights (sum 1)
__host__ __device__ inline void radon7(int p, double &l0, double &l1, double &l2, double &w)
{
    const double s15 = 3.872983346207417;   // sqrt(15)
    const double a = (6.0 - s15) / 21.0, b = (6.0 + s15) / 21.0;
    const double wa = (155.0 - s15) / 1200.0, wb = (155.0 + s15) / 1200.0;
    switch (p) {
        case 0: l0 = l1 = l2 = 1.0 / 3.0; w = 9.0 / 40.0; break;
        case 1: l0 = a; l1 = a; l2 = 1 - 2 * a; w = wa; break;
        case 2: l0 = a; l1 = 1 - 2 * a; l2 = a; w = wa; break;
        case 3: l0 = 1 - 2 * a; l1 = a; l2 = a; w = wa; break;
        case 4: l0 = b; l1 = b; l2 = 1 - 2 * b; w = wb; break;
        case 5: l0 = b; l1 = 1 - 2 * b; l2 = b; w = wb; break;
        default: l0 = 1 - 2 * b; l1 = b; l2 = b; w = wb; break;
    }
}

struct V3 { double x, y, z; };
__host__ __device__ inline V3 v3(const double *p) { return {p[0], p[1], p[2]}; }
__host__ __device__ inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__host__ __device__ inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__host__ __device__ inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__host__ __device__ inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__host__ __device__ inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

// Helmholtz kernel at separation d = x - y: G = e^{-jkR}/(4 pi R) and the
// factor g with grad_x G = g d.
__host__ __device__ inline void helmholtz(V3 d, double k, cpx<double> &G, cpx<double> &g)
{
    const double R = sqrt(dot(d, d));
    double sn, cs;
    sincos(k * R, &sn, &cs);
    const double inv = 1.0 / (4.0 * M_PI * R);
    G = {cs * inv, -sn * inv};                       // e^{-jkR}/(4 pi R)
    const double ir2 = 1.0 / (R * R);
    // -(1 + jkR) e^{-jkR} / (4 pi R^3)
    const double kr = k * R;
    g = {-(cs + kr * sn) * inv * ir2, -(kr * cs - sn) * inv * ir2};
}

// Adds the integrand of T, K, n x L, n x Kbar at the point pair (x, y) for
// test edge i (free vertex P[i]) and source edge j (free vertex Q[j]).
struct Integrand {
    const V3 *P, *Q;
    V3 nt;
    double k;
    __host__ __device__ inline void term(V3 x, V3 y, int i, int j, double w, cpx<double> G, cpx<double> g, cpx<double> out[4]) const
    {
        const V3 d = x - y;
        const V3 a = x - P[i], b = y - Q[j];
        const V3 tw = cross(nt, a);                       // n_t x (x - p_i)
        const double ab = dot(a, b), twb = dot(tw, b), twd = dot(tw, d);
        const V3 dxb = cross(d, b);
        const double a_dxb = dot(a, dxb), tw_dxb = dot(tw, dxb);
        // T = -jk (a.b - 4/k^2) G
        const double f = ab - 4.0 / (k * k);
        out[0].re += w * (k * f * G.im);
        out[0].im += w * (-k * f * G.re);
        // K = a . (g d x b)
        out[1].re += w * g.re * a_dxb;
        out[1].im += w * g.im * a_dxb;
        // Tx = jk (tw.b) G + (2j/k) g (tw.d)
        out[2].re += w * (-k * twb * G.im - (2.0 / k) * twd * g.im);
        out[2].im += w * (k * twb * G.re + (2.0 / k) * twd * g.re);
        // Kx = -tw . (g d x b)
        out[3].re -= w * g.re * tw_dxb;
        out[3].im -= w * g.im * tw_dxb;
    }
};

// ---------------------------------------------------------------- patterns
// R_n(k) = Int f_n e^{+jk khat.(r - r_b)} (theta, phi components) and the
// receive pattern of the C block Q_n = conj(Rg_n) - khat x conj(R_n) with
// Rg_n = Int (n x f_n) e^{+jk khat.(r - r_b)}; both by the 7-point rule.
__global__ void k_patterns(int N, int K, int nph, const double *__restrict__ ct, double k,
                           const int *__restrict__ rtri, const double *__restrict__ rcoef, const int *__restrict__ rloc,
                           const double *__restrict__ tri_v, const double *__restrict__ tri_n,
                           const double *__restrict__ tri_a, const double *__restrict__ centre,
                           cpx<double> *__restrict__ R, cpx<double> *__restrict__ Q)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)N * K) return;
    const int n = (int)(g / K), q = (int)(g % K);
    const int it = q / nph, ip = q % nph;
    const double c = ct[it], s = sqrt(fmax(0.0, 1 - c * c));
    double sp, cp;
    sincos(2.0 * M_PI * ip / nph, &sp, &cp);
    const V3 kh = {s * cp, s * sp, c}, th = {c * cp, c * sp, -s}, ph = {-sp, cp, 0.0};
    const V3 rb = v3(centre + 3 * (long long)n);
    cpx<double> Rt{0, 0}, Rp{0, 0}, Gt{0, 0}, Gp{0, 0};
    for (int h = 0; h < 2; h++) {
        const int t = rtri[2 * n + h];
        const double cf = rcoef[2 * n + h] * tri_a[t];
        const V3 P0 = v3(tri_v + 9 * (long long)t), P1 = v3(tri_v + 9 * (long long)t + 3),
                 P2 = v3(tri_v + 9 * (long long)t + 6);
        const V3 pf = v3(tri_v + 9 * (long long)t + 3 * rloc[2 * n + h]);
        const V3 nt = v3(tri_n + 3 * (long long)t);
        for (int p = 0; p < 7; p++) {
            double l0, l1, l2, w;
            radon7(p, l0, l1, l2, w);
            const V3 r = l0 * P0 + l1 * P1 + l2 * P2;
            const V3 f = (w * cf) * (r - pf);
            const V3 tw = cross(nt, f);
            double sn, cs;
            sincos(k * dot(kh, r - rb), &sn, &cs);
            const double ft = dot(f, th), fp = dot(f, ph), gt = dot(tw, th), gp = dot(tw, ph);
            Rt.re += ft * cs; Rt.im += ft * sn;
            Rp.re += fp * cs; Rp.im += fp * sn;
            Gt.re += gt * cs; Gt.im += gt * sn;
            Gp.re += gp * cs; Gp.im += gp * sn;
        }
    }
    R[2 * g] = Rt;
    R[2 * g + 1] = Rp;
    // Q = conj(Rg) - khat x conj(R),  khat x (v_t, v_p) = (-v_p, v_t)
    Q[2 * g] = conjg(Gt) + conjg(Rp);
    Q[2 * g + 1] = conjg(Gp) - conjg(Rt);
}

// ----------------------------------------------------------- touching pairs
// Reference coordinates: x = P0 + s1 (P1-P0) + s2 (P2-P0),
//                        y = Q0 + t1 (Q1-Q0) + t2 (Q2-Q0).
// rel 1 (shared vertex P0 = Q0): polar coordinates about the vertex on both
//   triangles, radial square split on its diagonal; weight xi^3 eta.
// rel 2 (shared edge P0P1 = Q0P1): each triangle swept from the edge to its
//   apex, x = (1-h)(P0 + sigma (P1-P0)) + h P2; split on the order of the two
//   edge abscissae, then the cube (offset, h_t, h_s) into three pyramids;
//   weight xi^2 (1 - offset) (1 - h_t) (1 - h_s).
// rel 3 (same triangle): difference vector over the hexagon S - S in polar
//   form; weight xi (1 - xi)^2 t1; each point also evaluated with x and y
//   exchanged (the opposite hexagon edge), so odd 1/R^2 parts cancel in pairs.
__host__ __device__ inline void rule_point(int rel, int n, long long idx, const double *gx, const double *gw, double &s1,
                                  double &s2, double &t1, double &t2, double &w)
{
    const int i3 = (int)(idx % n); idx /= n;
    const int i2 = (int)(idx % n); idx /= n;
    const int i1 = (int)(idx % n); idx /= n;
    const int i0 = (int)(idx % n); idx /= n;
    const int region = (int)idx;
    const double u0 = gx[i0], u1 = gx[i1], u2 = gx[i2], u3 = gx[i3];
    const double wg = gw[i0] * gw[i1] * gw[i2] * gw[i3];
    if (rel == 1) {
        const double xi = u0, eta = u1;
        const double r1 = region == 0 ? xi : xi * eta, r2 = region == 0 ? xi * eta : xi;
        s1 = r1 * (1 - u2); s2 = r1 * u2;
        t1 = r2 * (1 - u3); t2 = r2 * u3;
        w = wg * xi * xi * xi * eta;
    } else if (rel == 2) {
        const int ord = region / 3, pyr = region % 3;
        const double xi = u0, e1 = u1, e2 = u2, tau = u3;
        double off, ht, hs;
        if (pyr == 0) { off = xi; ht = xi * e1; hs = xi * e2; }
        else if (pyr == 1) { ht = xi; off = xi * e1; hs = xi * e2; }
        else { hs = xi; off = xi * e1; ht = xi * e2; }
        const double big = off + (1 - off) * tau, small = big - off;
        const double st = ord == 0 ? big : small, ss = ord == 0 ? small : big;
        s1 = (1 - ht) * st; s2 = ht;
        t1 = (1 - hs) * ss; t2 = hs;
        w = wg * xi * xi * (1 - off) * (1 - ht) * (1 - hs);
    } else {
        const double xi = u0, eta = u1;
        // hexagon edge `region` as a - b with a, b on the boundary of
        // S = {0 <= v <= u <= 1} (coordinates (u, v))
        double au, av, bu, bv;
        if (region == 0) { au = 1; av = eta; bu = 0; bv = 0; }
        else if (region == 1) { au = 1; av = 1; bu = eta; bv = 0; }
        else { au = 1 - eta; av = 1 - eta; bu = 1; bv = 0; }
        const double pu = u2, pv = u2 * u3;           // point of S
        const double xu = (1 - xi) * pu + xi * bu, xv = (1 - xi) * pv + xi * bv;
        const double yu = (1 - xi) * pu + xi * au, yv = (1 - xi) * pv + xi * av;
        s1 = xu - xv; s2 = xv;                          // (u, v) -> reference
        t1 = yu - yv; t2 = yv;
        w = wg * xi * (1 - xi) * (1 - xi) * u2;
    }
}

__global__ __launch_bounds__(256) void k_touch(int npairs, const TouchPair *__restrict__ pairs, double k,
                                               const double *__restrict__ gnodes, const int *__restrict__ goff,
                                               cpx<double> *__restrict__ out)
{
    const int p = blockIdx.x;
    if (p >= npairs) return;
    const TouchPair tp = pairs[p];
    V3 P[3], Q[3];
    for (int a = 0; a < 3; a++) {
        P[a] = {tp.P[3 * a], tp.P[3 * a + 1], tp.P[3 * a + 2]};
        Q[a] = {tp.Q[3 * a], tp.Q[3 * a + 1], tp.Q[3 * a + 2]};
    }
    Integrand ig{P, Q, {tp.nt[0], tp.nt[1], tp.nt[2]}, k};
    const int n = tp.order;
    const double *gx = gnodes + goff[n], *gw = gx + n;
    const double scale = 4.0 * tp.At * tp.As;   // (2 A_t)(2 A_s): reference -> physical
    const long long n4 = (long long)n * n * n * n;
    const long long count = tp.rel == 1 ? 2 * n4 : (tp.rel == 2 ? 6 * n4 : 3 * n4);
    cpx<double> acc[9][4];
    for (int e = 0; e < 9; e++)
        for (int o = 0; o < 4; o++) acc[e][o] = {0, 0};
    const V3 e1 = P[1] - P[0], e2 = P[2] - P[0], f1 = Q[1] - Q[0], f2 = Q[2] - Q[0];
    for (long long idx = threadIdx.x; idx < count; idx += blockDim.x) {
        double s1, s2, t1, t2, w;
        rule_point(tp.rel, n, idx, gx, gw, s1, s2, t1, t2, w);
        w *= scale;
        for (int sw = 0; sw < (tp.rel == 3 ? 2 : 1); sw++) {
            const V3 x = sw == 0 ? P[0] + s1 * e1 + s2 * e2 : P[0] + t1 * e1 + t2 * e2;
            const V3 y = sw == 0 ? Q[0] + t1 * f1 + t2 * f2 : Q[0] + s1 * f1 + s2 * f2;
            cpx<double> G, g;
            helmholtz(x - y, k, G, g);
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) ig.term(x, y, i, j, w, G, g, acc[3 * i + j]);
        }
    }
    // block reduction: waves by shuffles, then across waves through LDS
    __shared__ double red[4][72];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    for (int e = 0; e < 9; e++)
        for (int o = 0; o < 4; o++) {
            double re = acc[e][o].re, im = acc[e][o].im;
            for (int m = 32; m >= 1; m >>= 1) {
                re += __shfl_xor(re, m, 64);
                im += __shfl_xor(im, m, 64);
            }
            if (lane == 0) {
                red[wave][2 * (4 * e + o)] = re;
                red[wave][2 * (4 * e + o) + 1] = im;
            }
        }
    __syncthreads();
    if (threadIdx.x < 72) {
        double v = 0;
        for (int wv = 0; wv < (int)(blockDim.x / 64); wv++) v += red[wv][threadIdx.x];
        const int e = threadIdx.x / 8, o = (threadIdx.x / 2) % 4, part = threadIdx.x % 2;
        const int i = e / 3, j = e % 3;
        // result stored as [op][original test edge][original source edge]
        double *dst = reinterpret_cast<double *>(out + 36LL * p + 9 * o + 3 * tp.pi[i] + tp.qi[j]);
        dst[part] = (tp.rel == 3 && (o == 1 || o == 3)) ? 0.0 : v;   // K, n x Kbar vanish on one flat triangle
    }
}

// --------------------------------------------------------------- near slots
// One workgroup per leaf box; threads over the (row, near column) slots of the
// box.  Each slot sums the four triangle pairs of its two RWGs.
__host__ __device__ inline void regular_pair(const double *Pv, const double *Qv, const double *nt, double At, double As, int i,
                                    int j, double k, cpx<double> out[4])
{
    V3 P[3] = {v3(Pv), v3(Pv + 3), v3(Pv + 6)}, Q[3] = {v3(Qv), v3(Qv + 3), v3(Qv + 6)};
    Integrand ig{P, Q, v3(nt), k};
    for (int p = 0; p < 7; p++) {
        double a0, a1, a2, wp;
        radon7(p, a0, a1, a2, wp);
        const V3 x = a0 * P[0] + a1 * P[1] + a2 * P[2];
        for (int q = 0; q < 7; q++) {
            double b0, b1, b2, wq;
            radon7(q, b0, b1, b2, wq);
            const V3 y = b0 * Q[0] + b1 * Q[1] + b2 * Q[2];
            cpx<double> G, g;
            helmholtz(x - y, k, G, g);
            ig.term(x, y, i, j, wp * At * wq * As, G, g, out);
        }
    }
}

__global__ __launch_bounds__(256) void k_slots(const int *__restrict__ box_start, const int *__restrict__ near_start,
                                               const int *__restrict__ near_box, const long long *__restrict__ val_off,
                                               const int *__restrict__ rtri, const int *__restrict__ rloc,
                                               const double *__restrict__ rcoef, const double *__restrict__ tri_v,
                                               const double *__restrict__ tri_n, const double *__restrict__ tri_a,
                                               const int *__restrict__ tp_start, const int *__restrict__ tp_s,
                                               const cpx<double> *__restrict__ touch, double k,
                                               cpx<double> *__restrict__ em64, cpx<double> *__restrict__ c64,
                                               cpx<float> *__restrict__ em32, cpx<float> *__restrict__ c32)
{
    __shared__ int cstart[32];
    __shared__ int pre[33];
    const int b = blockIdx.x;
    const int nn = near_start[b + 1] - near_start[b];
    if (threadIdx.x == 0) {
        pre[0] = 0;
        for (int q = 0; q < nn; q++) {
            int nb = near_box[near_start[b] + q];
            cstart[q] = box_start[nb];
            pre[q + 1] = pre[q] + box_start[nb + 1] - box_start[nb];
        }
    }
    __syncthreads();
    const int ncols = pre[nn];
    const int m0 = box_start[b];
    const long long nslot = (long long)(box_start[b + 1] - m0) * ncols;
    for (long long sl = threadIdx.x; sl < nslot; sl += blockDim.x) {
        const int m = m0 + (int)(sl / ncols), jc = (int)(sl % ncols);
        int q = 0;
        while (jc >= pre[q + 1]) q++;
        const int n = cstart[q] + (jc - pre[q]);
        cpx<double> acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
        for (int h1 = 0; h1 < 2; h1++)
            for (int h2 = 0; h2 < 2; h2++) {
                const int t = rtri[2 * m + h1], s = rtri[2 * n + h2];
                const int i = rloc[2 * m + h1], j = rloc[2 * n + h2];
                const double cc = rcoef[2 * m + h1] * rcoef[2 * n + h2];
                int hit = -1;
                for (int e = tp_start[t]; e < tp_start[t + 1]; e++)
                    if (tp_s[e] == s) { hit = e; break; }
                cpx<double> part[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
                if (hit >= 0) {
                    for (int o = 0; o < 4; o++) part[o] = touch[36LL * hit + 9 * o + 3 * i + j];
                } else {
                    regular_pair(tri_v + 9LL * t, tri_v + 9LL * s, tri_n + 3LL * t, tri_a[t], tri_a[s], i, j, k, part);
                }
                for (int o = 0; o < 4; o++) acc[o] = acc[o] + cc * part[o];
            }
        const cpx<double> T = acc[0], Kk = acc[1], Tx = acc[2], Kx = acc[3];
        const cpx<double> A = -0.5 * (T + Kx), B = 0.5 * (Tx - Kk);
        const long long slot = val_off[b] + sl;
        em64[2 * slot] = T;
        em64[2 * slot + 1] = Kk;
        c64[2 * slot] = A;
        c64[2 * slot + 1] = B;
        em32[2 * slot] = {(float)T.re, (float)T.im};
        em32[2 * slot + 1] = {(float)Kk.re, (float)Kk.im};
        c32[2 * slot] = {(float)A.re, (float)A.im};
        c32[2 * slot + 1] = {(float)B.re, (float)B.im};
    }
}

// ------------------------------------------------------------- conversions
__global__ void k_to_float(const cpx<double> *__restrict__ a, cpx<float> *__restrict__ b, long long n)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) b[g] = {(float)a[g].re, (float)a[g].im};
}

// ------------------------------------------------------------- plane waves
// b^J = <f, E/2 + n x H/2>, b^M = <f, H/2 - n x E/2>, E = p e^{-jk khat.r},
// H = khat x p e^{-jk khat.r}; 7-point rule on both triangles of the RWG.
template <class T>
__global__ void k_plane_wave(int N, int nrhs, double k, const int *__restrict__ perm, const int *__restrict__ rtri,
                             const int *__restrict__ rloc, const double *__restrict__ rcoef,
                             const double *__restrict__ tri_v, const double *__restrict__ tri_n,
                             const double *__restrict__ tri_a, const double *__restrict__ dirs,
                             cpx<T> *__restrict__ b, long long ldb)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)N * nrhs) return;
    const int i = (int)(g % N), r = (int)(g / N);
    const V3 kh = v3(dirs + 6 * r), p = v3(dirs + 6 * r + 3);
    const V3 h = cross(kh, p);
    cpx<double> bj{0, 0}, bm{0, 0};
    for (int s = 0; s < 2; s++) {
        const int t = rtri[2 * i + s];
        const double cf = rcoef[2 * i + s] * tri_a[t];
        const V3 P0 = v3(tri_v + 9LL * t), P1 = v3(tri_v + 9LL * t + 3), P2 = v3(tri_v + 9LL * t + 6);
        const V3 pf = v3(tri_v + 9LL * t + 3 * rloc[2 * i + s]);
        const V3 n = v3(tri_n + 3LL * t);
        const V3 nxe = cross(n, p), nxh = cross(n, h);
        for (int q = 0; q < 7; q++) {
            double l0, l1, l2, w;
            radon7(q, l0, l1, l2, w);
            const V3 x = l0 * P0 + l1 * P1 + l2 * P2;
            const V3 a = x - pf;
            double sn, cs;
            sincos(k * dot(kh, x), &sn, &cs);
            const double fj = 0.5 * w * cf * (dot(a, p) + dot(a, nxh));
            const double fm = 0.5 * w * cf * (dot(a, h) - dot(a, nxe));
            bj.re += fj * cs; bj.im -= fj * sn;
            bm.re += fm * cs; bm.im -= fm * sn;
        }
    }
    const int u = perm[i];
    b[(long long)r * ldb + u] = {(T)bj.re, (T)bj.im};
    b[(long long)r * ldb + N + u] = {(T)bm.re, (T)bm.im};
}

// -------------------------------------------------------------- far field
// F(khat) = (-jk/4pi)[P_J - khat (khat . P_J) - khat x P_M], the far-zone
// limit of E = L{J} - K{M} (plane-wave limits L -> -jk(I - khat khat),
// K -> -jk khat x); P_X = Int X exp(+jk khat . r) ds with the 7-point rule on
// both triangles of every RWG; the radar cross section of Sec. III is
// 4 pi |F|^2.  Workgroup = (direction, right-hand side), threads over RWGs,
// double-precision sums reduced in LDS; output F . theta_hat, F . phi_hat.
template <class T>
__global__ __launch_bounds__(256) void k_far_field(int N, double k, const int *__restrict__ perm,
                                                   const int *__restrict__ rtri, const int *__restrict__ rloc,
                                                   const double *__restrict__ rcoef, const double *__restrict__ tri_v,
                                                   const double *__restrict__ tri_a, const double *__restrict__ dirs,
                                                   const cpx<T> *__restrict__ x, long long ldx, cpx<T> *__restrict__ F,
                                                   int nrhs)
{
    __shared__ double red[12][256];
    const int d = blockIdx.x, r = blockIdx.y;
    const V3 kh = v3(dirs + 3 * d);
    double acc[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};   // P_J (re, im) xyz, then P_M
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int u = perm[i];
        const cpx<T> xj = x[(long long)r * ldx + u], xm = x[(long long)r * ldx + N + u];
        for (int s2 = 0; s2 < 2; s2++) {
            const int t = rtri[2 * i + s2];
            const double cf = rcoef[2 * i + s2] * tri_a[t];
            const V3 P0 = v3(tri_v + 9LL * t), P1 = v3(tri_v + 9LL * t + 3), P2 = v3(tri_v + 9LL * t + 6);
            const V3 pf = v3(tri_v + 9LL * t + 3 * rloc[2 * i + s2]);
            for (int q = 0; q < 7; q++) {
                double l0, l1, l2, w;
                radon7(q, l0, l1, l2, w);
                const V3 xq = l0 * P0 + l1 * P1 + l2 * P2;
                const V3 a = (w * cf) * (xq - pf);
                double sn, cs;
                sincos(k * dot(kh, xq), &sn, &cs);
                // a e^{+j phase} times the coefficients
                const double pjr = cs * xj.re - sn * xj.im, pji = cs * xj.im + sn * xj.re;
                const double pmr = cs * xm.re - sn * xm.im, pmi = cs * xm.im + sn * xm.re;
                const double av[3] = {a.x, a.y, a.z};
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    acc[2 * c] += av[c] * pjr;
                    acc[2 * c + 1] += av[c] * pji;
                    acc[6 + 2 * c] += av[c] * pmr;
                    acc[6 + 2 * c + 1] += av[c] * pmi;
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 12; c++) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
#pragma unroll
            for (int c = 0; c < 12; c++) red[c][threadIdx.x] += red[c][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double kk[3] = {kh.x, kh.y, kh.z};
    double PJr[3], PJi[3], PMr[3], PMi[3];
    for (int c = 0; c < 3; c++) {
        PJr[c] = red[2 * c][0];
        PJi[c] = red[2 * c + 1][0];
        PMr[c] = red[6 + 2 * c][0];
        PMi[c] = red[6 + 2 * c + 1][0];
    }
    const double kpr = kk[0] * PJr[0] + kk[1] * PJr[1] + kk[2] * PJr[2];
    const double kpi = kk[0] * PJi[0] + kk[1] * PJi[1] + kk[2] * PJi[2];
    double Fr[3], Fi[3];
    for (int c = 0; c < 3; c++) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        Fr[c] = PJr[c] - kk[c] * kpr - (kk[c1] * PMr[c2] - kk[c2] * PMr[c1]);
        Fi[c] = PJi[c] - kk[c] * kpi - (kk[c1] * PMi[c2] - kk[c2] * PMi[c1]);
    }
    const double th = acos(fmax(-1.0, fmin(1.0, kk[2]))), ph = atan2(kk[1], kk[0]);
    const double tv[3] = {cos(th) * cos(ph), cos(th) * sin(ph), -sin(th)}, pv[3] = {-sin(ph), cos(ph), 0.0};
    const double pre = k / (4 * M_PI);   // F = -j pre (...)
    double ftr = 0, fti = 0, fpr = 0, fpi = 0;
    for (int c = 0; c < 3; c++) {
        ftr += Fr[c] * tv[c];
        fti += Fi[c] * tv[c];
        fpr += Fr[c] * pv[c];
        fpi += Fi[c] * pv[c];
    }
    // -j (a + jb) = b - ja
    F[((long long)d * 2) * nrhs + r] = {(T)(pre * fti), (T)(-pre * ftr)};
    F[((long long)d * 2 + 1) * nrhs + r] = {(T)(pre * fpi), (T)(-pre * fpr)};
}

// ---------------------------------------------------------------- launchers
void launch_far_field(bool single, int N, double k, const int *perm, const int *rtri, const int *rloc,
                      const double *rcoef, const double *tri_v, const double *tri_a, const double *dirs, int ndir,
                      const void *x, long long ldx, void *F, int nrhs, hipStream_t s)
{
    if (ndir <= 0 || nrhs <= 0) return;
    const dim3 grid(ndir, nrhs);
    if (single)
        hipLaunchKernelGGL(k_far_field<float>, grid, dim3(256), 0, s, N, k, perm, rtri, rloc, rcoef, tri_v, tri_a,
                           dirs, (const cpx<float> *)x, ldx, (cpx<float> *)F, nrhs);
    else
        hipLaunchKernelGGL(k_far_field<double>, grid, dim3(256), 0, s, N, k, perm, rtri, rloc, rcoef, tri_v, tri_a,
                           dirs, (const cpx<double> *)x, ldx, (cpx<double> *)F, nrhs);
}

void launch_plane_wave(bool single, int N, int nrhs, double k, const int *perm, const int *rtri, const int *rloc,
                       const double *rcoef, const double *tri_v, const double *tri_n, const double *tri_a,
                       const double *dirs, void *b, long long ldb, hipStream_t s)
{
    long long n = (long long)N * nrhs;
    dim3 grid((unsigned)((n + 255) / 256));
    if (single)
        hipLaunchKernelGGL(k_plane_wave<float>, grid, dim3(256), 0, s, N, nrhs, k, perm, rtri, rloc, rcoef, tri_v,
                           tri_n, tri_a, dirs, (cpx<float> *)b, ldb);
    else
        hipLaunchKernelGGL(k_plane_wave<double>, grid, dim3(256), 0, s, N, nrhs, k, perm, rtri, rloc, rcoef, tri_v,
                           tri_n, tri_a, dirs, (cpx<double> *)b, ldb);
}

void launch_patterns(int N, int K, int nph, const double *ct, double k, const int *rtri, const double *rcoef,
                     const int *rloc, const double *tri_v, const double *tri_n, const double *tri_a,
                     const double *centre, cpx<double> *R, cpx<double> *Q, hipStream_t s)
{
    long long n = (long long)N * K;
    hipLaunchKernelGGL(k_patterns, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, K, nph, ct, k, rtri, rcoef,
                       rloc, tri_v, tri_n, tri_a, centre, R, Q);
}

void launch_touch(int npairs, const TouchPair *pairs, double k, const double *gnodes, const int *goff,
                  cpx<double> *out, hipStream_t s)
{
    if (npairs > 0)
        hipLaunchKernelGGL(k_touch, dim3(npairs), dim3(256), 0, s, npairs, pairs, k, gnodes, goff, out);
}

void launch_slots(int nbox, const int *box_start, const int *near_start, const int *near_box, const long long *val_off,
                  const int *rtri, const int *rloc, const double *rcoef, const double *tri_v, const double *tri_n,
                  const double *tri_a, const int *tp_start, const int *tp_s, const cpx<double> *touch, double k,
                  cpx<double> *em64, cpx<double> *c64, cpx<float> *em32, cpx<float> *c32, hipStream_t s)
{
    hipLaunchKernelGGL(k_slots, dim3(nbox), dim3(256), 0, s, box_start, near_start, near_box, val_off, rtri, rloc,
                       rcoef, tri_v, tri_n, tri_a, tp_start, tp_s, touch, k, em64, c64, em32, c32);
}

void launch_to_float(const cpx<double> *a, cpx<float> *b, long long n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_to_float, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n);
}

}  // namespace mlfma
