// Aggregation and disaggregation steps on the matrix cores (complex64).
//
// The level steps of Sec. II-E's MLFMA are separable products of small real
// matrices with a box pattern P[theta row][phi column] (for one component
// and one right-hand side):
//   aggregation    U_P += shift_c (.) ( A_th CE_c  B_ph^T )
//   disaggregation V_c += D_th X_ext + D_th' X_ext'   with X = rowf (.) conj(shift_c) (.) V_P  D_ph^T
// A_th is the theta interpolation over the child rows extended across the
// poles (row e of CE is child theta row idx(e), its phi columns turned by
// half a circle for the reflected copies), B_ph the periodic phi
// interpolation, D_ph / D_th the weighted transposes (anterpolation), with
// D_th' the taps that reach across a pole (their columns turned by half a
// circle).  Each product is a 16 x 16 x 4 FP32 MFMA sequence, complex data
// times real weights as two real MFMAs (real and imaginary parts).
//
// Lane layout of v_mfma_f32_16x16x4f32 (wave64): lane l supplies A[l % 16][l
// / 16] and B[l / 16][l % 16] and holds D[(l / 16) * 4 + v][l % 16].  The
// first product of each step is computed transposed so that its result
// registers are directly the A (aggregation) or B (disaggregation) operand
// of the second one: the K index of the second product runs over (lane group
// g, register v) as 4 g + v, a permutation of K that both operands share.
//
// One wave owns one (box, component, right-hand side) pattern (aggregation:
// and one tile of 16 parent theta rows), so waves need no LDS and no
// barriers; every output element is written by one lane.
#include "device.hpp"

namespace mlfma {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
__device__ inline f4 mma(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

constexpr int NXCD_S = 8;
// every XCD takes a contiguous range of waves (four per workgroup); wave
// counts stay below 2^31 (checked by the launchers), so the index
// arithmetic is 32-bit
__device__ inline int xcd_wave(int nwave)
{
    const int nblk = (nwave + 3) / 4;
    const int per = (nblk + NXCD_S - 1) / NXCD_S;
    const int lb = (int)(blockIdx.x % NXCD_S) * per + (int)(blockIdx.x / NXCD_S);
    if (lb >= nblk) return -1;
    const int w = lb * 4 + (int)(threadIdx.x / 64);
    return w < nwave ? w : -1;
}

// aggregation: wave = (parent, component, right-hand side, tile of 16 parent
// theta rows).  The wave walks the (child, child phi tile) steps of its
// parent in order; the operands of the theta product of step s + 1 (at most
// KSM k-steps of 4 extended child rows) are loaded while step s is
// multiplied, so every step waits on one round of loads, not on one load per
// k-step.
constexpr int KSM = 8;
template <int NPT>
__global__ __launch_bounds__(256) void k_aggregate_mfma(const StepMfma a, const cpx<float> *__restrict__ in,
                                                        cpx<float> *__restrict__ out, int nrhs)
{
    const int w = xcd_wave(a.nbox * 2 * nrhs * a.nit);
    if (w < 0) return;
    const int it = w % a.nit;
    const int pr = w / a.nit;
    const int r = pr % nrhs, comp = (pr / nrhs) & 1;
    const int P = pr / nrhs / 2;
    const int lane = threadIdx.x & 63, m16 = lane & 15, g = lane >> 4;
    const int Kc = a.nth_c * a.nph_c, Kp = a.nth_p * a.nph_p;
    const int ks0 = a.ks_lo[it], nks = a.ks_hi[it] - ks0;   // nks <= KSM (checked by the host)
    const int c0 = a.child_start[P], nstep = (a.child_start[P + 1] - c0) * a.njt;
    // per k-step: this lane's extended row and its turned column offset
    int erow[KSM], esh[KSM];
    float bth[KSM];
    const float *ath = a.ath + (size_t)(it * 16 + m16) * a.e_pad;
#pragma unroll
    for (int k = 0; k < KSM; k++) {
        const int e = 4 * (ks0 + k) + g;
        const bool ok = k < nks && e < a.ne;
        erow[k] = ok ? a.ext_row[e] : -1;
        esh[k] = ok ? a.ext_sh[e] : 0;
        bth[k] = k < nks ? ath[e] : 0.f;
    }
    f4 accr[NPT], acci[NPT], d2r[NPT], d2i[NPT];
#pragma unroll
    for (int p = 0; p < NPT; p++) accr[p] = acci[p] = d2r[p] = d2i[p] = f4{0.f, 0.f, 0.f, 0.f};
    float nr[KSM], ni[KSM];   // operands of the next step
    auto load = [&](int s) {
        const int c = c0 + s / a.njt, jc = (s % a.njt) * 16 + m16;
        const cpx<float> *cb = in + ((long long)(c * 2 + comp) * nrhs + r) * Kc;
#pragma unroll
        for (int k = 0; k < KSM; k++) {
            nr[k] = ni[k] = 0.f;
            if (erow[k] >= 0 && jc < a.nph_c) {
                int col = jc + esh[k];
                col = col >= a.nph_c ? col - a.nph_c : col;
                const cpx<float> v = cb[erow[k] * a.nph_c + col];
                nr[k] = v.re;
                ni[k] = v.im;
            }
        }
    };
    if (nstep > 0) load(0);
    for (int s = 0; s < nstep; s++) {
        float cr[KSM], ci[KSM];
#pragma unroll
        for (int k = 0; k < KSM; k++) {
            cr[k] = nr[k];
            ci[k] = ni[k];
        }
        if (s + 1 < nstep) load(s + 1);
        const int jt = s % a.njt;
        // MID^T tile (child phi columns x parent theta rows) = CE^T A_th^T
        f4 d1r = {0.f, 0.f, 0.f, 0.f}, d1i = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < KSM; k++) {
            if (k >= nks) break;
            d1r = mma(cr[k], bth[k], d1r);
            d1i = mma(ci[k], bth[k], d1i);
        }
        // OUT tile (parent theta rows x parent phi columns) += MID B_ph^T
        const unsigned mask = a.bmask[jt];
#pragma unroll
        for (int p = 0; p < NPT; p++) {
            if (!((mask >> p) & 1)) continue;
            const f4 bv = *reinterpret_cast<const f4 *>(a.bph + (size_t)(p * 16 + m16) * a.jc_pad + jt * 16 + 4 * g);
#pragma unroll
            for (int v = 0; v < 4; v++) {
                d2r[p] = mma(d1r[v], bv[v], d2r[p]);
                d2i[p] = mma(d1i[v], bv[v], d2i[p]);
            }
        }
        if (jt + 1 < a.njt) continue;
        // child done: shift to the parent centre and add to the sums
        const int c = c0 + s / a.njt;
        const cpx<float> *sh = a.shift + (long long)a.oct[c] * Kp;
#pragma unroll
        for (int p = 0; p < NPT; p++) {
            const int jp = p * 16 + m16;
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int ip = it * 16 + 4 * g + v;
                if (ip < a.nth_p && jp < a.nph_p) {
                    const cpx<float> sv = sh[ip * a.nph_p + jp];
                    accr[p][v] += sv.re * d2r[p][v] - sv.im * d2i[p][v];
                    acci[p][v] += sv.re * d2i[p][v] + sv.im * d2r[p][v];
                }
            }
            d2r[p] = d2i[p] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    cpx<float> *ob = out + ((long long)(P * 2 + comp) * nrhs + r) * Kp;
#pragma unroll
    for (int p = 0; p < NPT; p++) {
        const int jp = p * 16 + m16;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int ip = it * 16 + 4 * g + v;
            if (ip < a.nth_p && jp < a.nph_p) ob[ip * a.nph_p + jp] = {accr[p][v], acci[p][v]};
        }
    }
}

// disaggregation: wave = (child, component, right-hand side).  The phi
// product's operands (shifted parent samples) are loaded a chunk of k-steps
// at a time, the next chunk while the current one is multiplied; the child's
// outputs of a tile are loaded before the theta product that adds to them.
template <int NIP>
__global__ __launch_bounds__(256) void k_disaggregate_mfma(const StepMfma a, const cpx<float> *__restrict__ in,
                                                           cpx<float> *__restrict__ out, int nrhs)
{
    const int w = xcd_wave(a.nbox * 2 * nrhs);
    if (w < 0) return;
    const int r = w % nrhs, comp = (w / nrhs) & 1;
    const int c = w / nrhs / 2;
    const int P = a.parent[c];
    const int lane = threadIdx.x & 63, m16 = lane & 15, g = lane >> 4;
    const int Kc = a.nth_c * a.nph_c, Kp = a.nth_p * a.nph_p;
    const cpx<float> *xb = in + ((long long)(P * 2 + comp) * nrhs + r) * Kp;
    const cpx<float> *sh = a.shift + (long long)a.oct[c] * Kp;
    cpx<float> *ob = out + ((long long)(c * 2 + comp) * nrhs + r) * Kc;
    const int half = a.nph_c / 2;
    float rf[NIP];
#pragma unroll
    for (int t = 0; t < NIP; t++) rf[t] = a.rowf[t * 16 + m16];
    for (int jt = 0; jt < a.njt; jt++) {
        const int jc = jt * 16 + m16;
        const bool jok = jc < a.nph_c;
        int jcs = jc + half;
        jcs = jcs >= a.nph_c ? jcs - a.nph_c : jcs;
        // MID tiles (parent theta rows x child phi columns) = X D_ph^T, and
        // for the tiles that reach across a pole the same at the columns
        // turned by half a circle
        f4 mr[NIP], mi[NIP], sr[NIP], si[NIP];
#pragma unroll
        for (int t = 0; t < NIP; t++) mr[t] = mi[t] = sr[t] = si[t] = f4{0.f, 0.f, 0.f, 0.f};
        const unsigned long long kmask = a.kmask[jt], kmask_s = a.kmask_s[jt];
        unsigned long long rest = kmask | kmask_s;
        const float *dph = a.dph + (size_t)(jok ? jc : 0) * a.jp_pad;
        const float *dphs = a.dph + (size_t)(jok ? jcs : 0) * a.jp_pad;
        // one chunk: up to CH k-steps (the next set bits of rest); two for
        // the wide parent levels, whose operand registers would otherwise
        // cost occupancy
        constexpr int CH = NIP >= 3 ? 2 : 4;
        int kk[CH], nk = 0;
        float xr[CH][NIP], xi[CH][NIP];
        auto take = [&]() {
            nk = 0;
#pragma unroll
            for (int u = 0; u < CH; u++) {
                kk[u] = -1;
                if (rest) {
                    kk[u] = __builtin_ctzll(rest);
                    rest &= rest - 1;
                    nk++;
                }
            }
#pragma unroll
            for (int u = 0; u < CH; u++) {
                const int jp = 4 * kk[u] + g;
#pragma unroll
                for (int t = 0; t < NIP; t++) {
                    const int ip = t * 16 + m16;
                    xr[u][t] = xi[u][t] = 0.f;
                    if (kk[u] >= 0 && ip < a.nth_p && jp < a.nph_p) {
                        const cpx<float> x = xb[ip * a.nph_p + jp], s_ = sh[ip * a.nph_p + jp];
                        xr[u][t] = rf[t] * (s_.re * x.re + s_.im * x.im);   // rowf conj(shift) x
                        xi[u][t] = rf[t] * (s_.re * x.im - s_.im * x.re);
                    }
                }
            }
        };
        take();
        while (nk > 0) {
            int ck[CH];
            float cr[CH][NIP], ci[CH][NIP];
            const int cn = nk;
#pragma unroll
            for (int u = 0; u < CH; u++) {
                ck[u] = kk[u];
#pragma unroll
                for (int t = 0; t < NIP; t++) {
                    cr[u][t] = xr[u][t];
                    ci[u][t] = xi[u][t];
                }
            }
            take();   // the next chunk's loads are in flight during these products
#pragma unroll
            for (int u = 0; u < CH; u++) {
                if (u >= cn) break;
                const int ks = ck[u], jp = 4 * ks + g;
                const bool in_d = (kmask >> ks) & 1, in_s = (kmask_s >> ks) & 1;
                const float b = in_d && jok ? dph[jp] : 0.f;
                const float bs = in_s && jok ? dphs[jp] : 0.f;
#pragma unroll
                for (int t = 0; t < NIP; t++) {
                    if (in_d) {
                        mr[t] = mma(cr[u][t], b, mr[t]);
                        mi[t] = mma(ci[u][t], b, mi[t]);
                    }
                    if (in_s && ((a.rmask >> t) & 1)) {
                        sr[t] = mma(cr[u][t], bs, sr[t]);
                        si[t] = mma(ci[u][t], bs, si[t]);
                    }
                }
            }
        }
        // child tiles (child theta rows x child phi columns) += D_th MID + D_th' MID_turned
        for (int ct = 0; ct < a.nict; ct++) {
            cpx<float> yo[4];
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int ic = ct * 16 + 4 * g + v;
                yo[v] = jok && ic < a.nth_c ? ob[ic * a.nph_c + jc] : cpx<float>{0.f, 0.f};
            }
            f4 yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
            const unsigned dm = a.dmask[ct], rm = a.rmask_c[ct];
            const float *dd = a.dthd + (size_t)(ct * 16 + m16) * a.ip_pad + 4 * g;
            const float *dr = a.dthr + (size_t)(ct * 16 + m16) * a.ip_pad + 4 * g;
#pragma unroll
            for (int t = 0; t < NIP; t++) {
                if ((dm >> t) & 1) {
                    const f4 wv = *reinterpret_cast<const f4 *>(dd + t * 16);
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        yr = mma(wv[v], mr[t][v], yr);
                        yi = mma(wv[v], mi[t][v], yi);
                    }
                }
                if ((rm >> t) & 1) {
                    const f4 wv = *reinterpret_cast<const f4 *>(dr + t * 16);
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        yr = mma(wv[v], sr[t][v], yr);
                        yi = mma(wv[v], si[t][v], yi);
                    }
                }
            }
            if (!jok) continue;
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int ic = ct * 16 + 4 * g + v;
                if (ic < a.nth_c) ob[ic * a.nph_c + jc] = {yo[v].re + yr[v], yo[v].im + yi[v]};
            }
        }
    }
}

}  // namespace

bool launch_aggregate_mfma(const StepMfma &a, const cpx<float> *in, cpx<float> *out, int nrhs, hipStream_t s)
{
    if (!a.ok || a.nbox <= 0 || nrhs <= 0) return a.ok;
    const long long nwave = (long long)a.nbox * 2 * nrhs * a.nit;
    if (nwave >= (1LL << 31)) return false;
    const long long nblk = (nwave + 3) / 4;
    const dim3 grid((unsigned)(((nblk + NXCD_S - 1) / NXCD_S) * NXCD_S)), block(256);
    const int npt = (a.nph_p + 15) / 16;
    if (npt <= 2) hipLaunchKernelGGL(k_aggregate_mfma<2>, grid, block, 0, s, a, in, out, nrhs);
    else if (npt <= 4) hipLaunchKernelGGL(k_aggregate_mfma<4>, grid, block, 0, s, a, in, out, nrhs);
    else if (npt <= 8) hipLaunchKernelGGL(k_aggregate_mfma<8>, grid, block, 0, s, a, in, out, nrhs);
    else return false;
    return true;
}

bool launch_disaggregate_mfma(const StepMfma &a, const cpx<float> *in, cpx<float> *out, int nrhs, hipStream_t s)
{
    if (!a.ok || a.nbox <= 0 || nrhs <= 0) return a.ok;
    const long long nwave = (long long)a.nbox * 2 * nrhs;
    if (nwave >= (1LL << 31)) return false;
    const long long nblk = (nwave + 3) / 4;
    const dim3 grid((unsigned)(((nblk + NXCD_S - 1) / NXCD_S) * NXCD_S)), block(256);
    const int nip = (a.nth_p + 15) / 16;
    if (nip <= 1) hipLaunchKernelGGL(k_disaggregate_mfma<1>, grid, block, 0, s, a, in, out, nrhs);
    else if (nip <= 2) hipLaunchKernelGGL(k_disaggregate_mfma<2>, grid, block, 0, s, a, in, out, nrhs);
    else if (nip <= 4) hipLaunchKernelGGL(k_disaggregate_mfma<4>, grid, block, 0, s, a, in, out, nrhs);
    else return false;
    return true;
}

}  // namespace mlfma
