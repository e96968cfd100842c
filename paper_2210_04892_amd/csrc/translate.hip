// Diagonal translation by sibling groups, register-blocked over targets.
//
// V_A(k) = sum_{(B, o) in IL(A)} T_o(k) U_B(k)  (Sec. II-E, MLFMA far field;
// diagonal in k).  Siblings share most of their interaction lists (the
// children of their parent's neighbours, less the boxes adjacent to each),
// so a group of up to TG siblings streams the union of its sources once:
// every lane loads a source's samples and applies them to every target of
// the group that has the source in its list, keeping all targets' sums in
// registers.  Nothing is staged in LDS and there are no barriers; a source's
// value is loaded once per group instead of once per (target, source) pair.
//
// Lanes: QW = 64 / RW consecutive samples x RW right-hand sides; each lane
// handles RB right-hand sides (rbase + j RW).  Fewer samples per wave (more
// lanes over the right-hand sides) load each operator value for fewer sums
// but keep fewer sums per lane (more waves resident): the autotuner picks.  A workgroup of four waves
// takes four consecutive sample chunks of one group.  Workgroups are ordered
// sample chunk first, group second, and every XCD takes a contiguous range
// of each level: consecutive groups (Morton order) share sources through the
// XCD's L2, and the operator rows of one sample chunk stay resident there.
#include "device.hpp"

namespace mlfma {

namespace {

constexpr int WAVE = 64;     // lanes of a wavefront
constexpr int NXCD = 8;      // dies (XCDs); hardware block b runs on XCD b mod 8
constexpr int GWAVES = 4;

typedef const __attribute__((address_space(4))) int cint_g;
__device__ inline int ldu(const int *p, int i) { return ((cint_g *)p)[i]; }

template <class T, int TG, int RW, int RB>
__global__ __launch_bounds__(GWAVES * WAVE) void k_translate_groups(const GroupArgs<T> a, int nrhs)
{
    constexpr int QW = WAVE / RW;
    const int xcd = blockIdx.x % NXCD, pos = blockIdx.x / NXCD;
    if (pos >= a.nblocks) return;
    int l = 0;
    while (l + 1 < a.nlev && pos >= a.lv[l + 1].first) l++;
    const GroupLevel<T> &L = a.lv[l];
    const int nblk = L.ngroup * L.nqc, per = (nblk + NXCD - 1) / NXCD;
    const int lb = xcd * per + (pos - L.first);
    if (lb >= nblk) return;
    const int g = lb % L.ngroup, qc = lb / L.ngroup;
    const int K = L.K;
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int qi = lane % QW, ri = lane / QW;
    const int q = (qc * GWAVES + wave) * QW + qi;
    const bool qok = q < K;
    const int qr = qok ? q : K - 1;   // lanes past the last sample read a valid element, store nothing
    const int rbase = blockIdx.y * RW * RB + ri;
    const long long S = 2LL * nrhs * K;   // one box's patterns
    long long ro[RB];
#pragma unroll
    for (int j = 0; j < RB; j++) ro[j] = (long long)min(rbase + j * RW, nrhs - 1) * K + qr;
    const long long half = (long long)nrhs * K;   // second component
    const int t0 = ldu(L.first_tgt, g), nt = ldu(L.count, g);
    const int r0 = ldu(L.rec_start, g), r1 = ldu(L.rec_start, g + 1);
    const cpx<T> *tq = L.trans + qr;
    cpx<T> acc[TG][2][RB];
#pragma unroll
    for (int t = 0; t < TG; t++)
#pragma unroll
        for (int j = 0; j < RB; j++) acc[t][0][j] = acc[t][1][j] = mk<T>(0, 0);
    // the next record (its source samples, operator values and offsets) is
    // loaded while the current one is summed, so that the wait for its data
    // does not also wait for loads issued in the same iteration
    cpx<T> u0[RB], u1[RB], opn[TG];
    int offn[TG];
    const int *srcp = L.src, *offp = L.off;
    const cpx<T> *Ub = L.U;
    auto load = [&](int r) {
        const cpx<T> *us = Ub + (long long)ldu(srcp, r) * S;
#pragma unroll
        for (int j = 0; j < RB; j++) {
            u0[j] = us[ro[j]];
            u1[j] = us[half + ro[j]];
        }
#pragma unroll
        for (int t = 0; t < TG; t++) {
            offn[t] = ldu(offp, r * TG + t);
            opn[t] = tq[(long long)max(offn[t], 0) * K];   // a valid row also where the source is absent
        }
    };
    if (r0 < r1) load(r0);
    for (int r = r0; r < r1; r++) {
        cpx<T> v0[RB], v1[RB], op[TG];
        int off[TG];
#pragma unroll
        for (int j = 0; j < RB; j++) {
            v0[j] = u0[j];
            v1[j] = u1[j];
        }
#pragma unroll
        for (int t = 0; t < TG; t++) {
            op[t] = opn[t];
            off[t] = offn[t];
        }
        if (r + 1 < r1) load(r + 1);
#pragma unroll
        for (int t = 0; t < TG; t++) {
            if (off[t] < 0) continue;   // uniform: the source is not in target t's list
#pragma unroll
            for (int j = 0; j < RB; j++) {
                fma_to(acc[t][0][j], op[t], v0[j]);
                fma_to(acc[t][1][j], op[t], v1[j]);
            }
        }
    }
    if (!qok) return;
#pragma unroll
    for (int t = 0; t < TG; t++) {
        if (t >= nt) break;
        cpx<T> *vt = L.V + (long long)(t0 + t) * S;
#pragma unroll
        for (int j = 0; j < RB; j++) {
            const int rr = rbase + j * RW;
            if (rr >= nrhs) continue;
            vt[(long long)rr * K + q] = acc[t][0][j];
            vt[half + (long long)rr * K + q] = acc[t][1][j];
        }
    }
}

}  // namespace

template <class T>
bool launch_translate_groups(const GroupArgs<T> &args, int nrhs, hipStream_t s)
{
    const int tg = args.tg;
    int rb = args.rb, rw = args.rw > 0 ? args.rw : trans_rw(nrhs);
    if (tg != 4 && tg != 8) return false;
    // (lanes over the RHS, RHS per lane) with a kernel
    auto valid = [&](int w, int b) {
        return (b == 1 && (w == 1 || w == 2 || w == 4 || w == 8 || w == 16)) || (w == 4 && (b == 2 || b == 4)) ||
               (w == 8 && b == 2) || (w == 2 && b == 8 && tg == 4 && sizeof(T) == 4);
    };
    if (!valid(rw, rb)) return false;
    // a shape tuned for more right-hand sides than this call has: fewer per
    // lane, else the default lane split (no lanes idle for lack of them)
    if (rw * rb > nrhs && nrhs > 0) {
        while (rb > 1 && (rw * rb > nrhs || !valid(rw, rb))) rb /= 2;
        if (rw * rb > nrhs) {
            rw = trans_rw(nrhs);
            rb = 1;
        }
    }
    if (args.nlev <= 0 || nrhs <= 0) return true;
    const int qw = WAVE / rw;
    GroupArgs<T> a = args;
    a.rb = rb;
    a.rw = rw;
    a.nblocks = 0;
    for (int l = 0; l < a.nlev; l++) {
        a.lv[l].nqc = (a.lv[l].K + GWAVES * qw - 1) / (GWAVES * qw);
        a.lv[l].first = a.nblocks;
        a.nblocks += (a.lv[l].ngroup * a.lv[l].nqc + NXCD - 1) / NXCD;
    }
    if (a.nblocks <= 0) return true;
    const dim3 grid((unsigned)a.nblocks * NXCD, (nrhs + rw * rb - 1) / (rw * rb)), block(GWAVES * WAVE);
#define GROUP_LAUNCH(TG_, RW_, RB_) hipLaunchKernelGGL((k_translate_groups<T, TG_, RW_, RB_>), grid, block, 0, s, a, nrhs)
#define GROUP_SHAPES(TG_)                          \
    if (rw == 4 && rb == 4) GROUP_LAUNCH(TG_, 4, 4);       \
    else if (rw == 4 && rb == 2) GROUP_LAUNCH(TG_, 4, 2);  \
    else if (rw == 8 && rb == 2) GROUP_LAUNCH(TG_, 8, 2);  \
    else if (rw == 16) GROUP_LAUNCH(TG_, 16, 1);           \
    else if (rw == 8) GROUP_LAUNCH(TG_, 8, 1);             \
    else if (rw == 4) GROUP_LAUNCH(TG_, 4, 1);             \
    else if (rw == 2) GROUP_LAUNCH(TG_, 2, 1);             \
    else GROUP_LAUNCH(TG_, 1, 1);
    if (tg == 4 && rw == 2 && rb == 8) {
        if constexpr (sizeof(T) == 4) GROUP_LAUNCH(4, 2, 8);   // single precision only (register budget)
    } else if (tg == 4) {
        GROUP_SHAPES(4)
    } else {
        GROUP_SHAPES(8)
    }
#undef GROUP_SHAPES
#undef GROUP_LAUNCH
    return true;
}

template bool launch_translate_groups<float>(const GroupArgs<float> &, int, hipStream_t);
template bool launch_translate_groups<double>(const GroupArgs<double> &, int, hipStream_t);

}  // namespace mlfma
