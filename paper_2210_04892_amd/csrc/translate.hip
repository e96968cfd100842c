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
// but keep fewer sums per lane (more waves resident): the autotuner picks.
// A workgroup of four waves takes four consecutive sample chunks of one
// group.  Workgroups are ordered sample chunk first, group second, and every
// XCD takes a contiguous range of each level: consecutive groups (Morton
// order) share sources through the XCD's L2, and the operator rows of one
// sample chunk stay resident there.
//
// Two variants share the group tables: k_translate_lds stages the operator
// rows of a sample chunk in LDS for a workgroup of four groups (only source
// samples then travel through the vector memory path), and k_translate_mfma
// forms the sums of a 16-target group as one complex product per sample on
// the matrix cores.
#include "device.hpp"
#include "mfma_ops.hpp"

namespace mlfma {

namespace {

constexpr int WAVE = 64;     // lanes of a wavefront
constexpr int NXCD = 8;      // dies (XCDs); hardware block b runs on XCD b mod 8
constexpr int GWAVES = 4;

typedef const __attribute__((address_space(4))) int cint_g;
__device__ inline int ldu(const int *p, int i) { return ((cint_g *)p)[i]; }

// Raw buffer loads: a resource descriptor for a uniform base address (no
// range check: every offset used lies inside the array) and a per-lane
// 32-bit byte offset, so that a loop's loads need no 64-bit vector address
// arithmetic.  Descriptor word 3 = 0x00020000 (the gfx9 family's 32-bit
// data format, no swizzle).
__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void *base)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, -1, 0x00020000);
}
template <class T>
__device__ inline cpx<T> bload(__amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ inline cpx<float> bload<float>(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(cpx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ inline cpx<double> bload<double>(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(cpx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

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
    const long long half = (long long)nrhs * K;   // second component
    // per-lane byte offsets within a box's patterns and within an operator
    // row: every load takes a uniform 64-bit base (scalar registers, from
    // the record's source and offset ids) and one of these 32-bit offsets
    unsigned rob[RB];
#pragma unroll
    for (int j = 0; j < RB; j++)
        rob[j] = (unsigned)(((long long)min(rbase + j * RW, nrhs - 1) * K + qr) * (long long)sizeof(cpx<T>));
    const unsigned qb = (unsigned)(qr * sizeof(cpx<T>));
    const int t0 = ldu(L.first_tgt, g), nt = ldu(L.count, g);
    const int r0 = ldu(L.rec_start, g), r1 = ldu(L.rec_start, g + 1);
    cpx<T> acc[TG][2][RB];
#pragma unroll
    for (int t = 0; t < TG; t++)
#pragma unroll
        for (int j = 0; j < RB; j++) acc[t][0][j] = acc[t][1][j] = mk<T>(0, 0);
    // a record: its source's samples, the group's operator values and offset
    // ids; the next record is loaded while the current one is summed (two
    // register sets used in turn)
    struct Rec {
        cpx<T> u0[RB], u1[RB], op[TG];
        int off[TG];
    };
    const int *srcp = L.src, *offp = L.off;
    const cpx<T> *Ub = L.U, *Tb = L.trans;
    auto load = [&](int r, Rec &o) {
        const cpx<T> *us = Ub + (long long)ldu(srcp, r) * S;
        const auto ru0 = rsrc(us), ru1 = rsrc(us + half);
#pragma unroll
        for (int j = 0; j < RB; j++) {
            o.u0[j] = bload<T>(ru0, rob[j]);
            o.u1[j] = bload<T>(ru1, rob[j]);
        }
#pragma unroll
        for (int t = 0; t < TG; t++) {
            o.off[t] = ldu(offp, r * TG + t);
            // a valid row also where the source is absent
            o.op[t] = bload<T>(rsrc(Tb + (long long)max(o.off[t], 0) * K), qb);
        }
    };
    auto sum = [&](const Rec &c) {
#pragma unroll
        for (int t = 0; t < TG; t++) {
            if (c.off[t] < 0) continue;   // uniform: the source is not in target t's list
#pragma unroll
            for (int j = 0; j < RB; j++) {
                fma_to(acc[t][0][j], c.op[t], c.u0[j]);
                fma_to(acc[t][1][j], c.op[t], c.u1[j]);
            }
        }
    };
    // the loads of the next record are issued on every path (past the last
    // record they repeat it), so that the wait before a sum counts the other
    // set's loads as in flight instead of merging with a path without them
    Rec ra, rb2;
    if (r0 < r1) load(r0, ra);
    for (int r = r0; r < r1; r += 2) {
        load(min(r + 1, r1 - 1), rb2);
        sum(ra);
        if (r + 1 >= r1) break;
        load(min(r + 2, r1 - 1), ra);
        sum(rb2);
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


// The sibling-group kernel with the operator values in LDS.  A workgroup
// takes four consecutive groups (one per wave) at one chunk of QW samples and
// first stages the operator rows of all 343 offsets for that chunk in LDS
// (343 QW complex values); the record loop then loads only source samples
// through the vector memory path and reads each present target's operator
// value from LDS.  Summing, record prefetch and stores are those of
// k_translate_groups.
template <class T, int TG, int RW, int RB>
__global__ __launch_bounds__(GWAVES * WAVE) void k_translate_lds(const GroupArgs<T> a, int nrhs)
{
    constexpr int QW = WAVE / RW;
    __shared__ cpx<T> tl[343 * QW];
    const int xcd = blockIdx.x % NXCD, pos = blockIdx.x / NXCD;
    if (pos >= a.nblocks) return;
    int l = 0;
    while (l + 1 < a.nlev && pos >= a.lv[l + 1].first) l++;
    const GroupLevel<T> &L = a.lv[l];
    const int ngb = (L.ngroup + GWAVES - 1) / GWAVES;
    const int nblk = ngb * L.nqc, per = (nblk + NXCD - 1) / NXCD;
    const int lb = xcd * per + (pos - L.first);
    if (lb >= nblk) return;
    const int gb = lb % ngb, qc = lb / ngb;
    const int K = L.K, q0 = qc * QW;
    // stage the chunk's operator rows (samples past K as zeros)
    for (int i = threadIdx.x; i < 343 * QW; i += GWAVES * WAVE) {
        const int o = i / QW, qq = q0 + i % QW;
        tl[i] = qq < K ? L.trans[(long long)o * K + qq] : mk<T>(0, 0);
    }
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int g = gb * GWAVES + wave;
    if (g >= L.ngroup) return;
    const int qi = lane % QW, ri = lane / QW;
    const int q = q0 + qi;
    const bool qok = q < K;
    const int qr = qok ? q : K - 1;   // lanes past the last sample read a valid element, store nothing
    const int rbase = blockIdx.y * RW * RB + ri;
    const long long S = 2LL * nrhs * K;   // one box's patterns
    const long long half = (long long)nrhs * K;   // second component
    unsigned rob[RB];
#pragma unroll
    for (int j = 0; j < RB; j++)
        rob[j] = (unsigned)(((long long)min(rbase + j * RW, nrhs - 1) * K + qr) * (long long)sizeof(cpx<T>));
    const int t0 = ldu(L.first_tgt, g), nt = ldu(L.count, g);
    const int r0 = ldu(L.rec_start, g), r1 = ldu(L.rec_start, g + 1);
    cpx<T> acc[TG][2][RB];
#pragma unroll
    for (int t = 0; t < TG; t++)
#pragma unroll
        for (int j = 0; j < RB; j++) acc[t][0][j] = acc[t][1][j] = mk<T>(0, 0);
    struct Rec {
        cpx<T> u0[RB], u1[RB];
        int off[TG];
    };
    const int *srcp = L.src, *offp = L.off;
    const cpx<T> *Ub = L.U;
    const cpx<T> *tq = tl + qi;
    auto load = [&](int r, Rec &o) {
        const cpx<T> *us = Ub + (long long)ldu(srcp, r) * S;
        const auto ru0 = rsrc(us), ru1 = rsrc(us + half);
#pragma unroll
        for (int j = 0; j < RB; j++) {
            o.u0[j] = bload<T>(ru0, rob[j]);
            o.u1[j] = bload<T>(ru1, rob[j]);
        }
#pragma unroll
        for (int t = 0; t < TG; t++) o.off[t] = ldu(offp, r * TG + t);
    };
    auto sum = [&](const Rec &c) {
#pragma unroll
        for (int t = 0; t < TG; t++) {
            if (c.off[t] >= 0) {   // uniform: the source is in target t's list
                const cpx<T> op = tq[c.off[t] * QW];
#pragma unroll
                for (int j = 0; j < RB; j++) {
                    fma_to(acc[t][0][j], op, c.u0[j]);
                    fma_to(acc[t][1][j], op, c.u1[j]);
                }
            }
        }
    };
    Rec ra, rb2;
    if (r0 < r1) load(r0, ra);
    for (int r = r0; r < r1; r += 2) {
        load(min(r + 1, r1 - 1), rb2);
        sum(ra);
        if (r + 1 >= r1) break;
        load(min(r + 2, r1 - 1), ra);
        sum(rb2);
    }
    if (!qok) return;
#pragma unroll
    for (int t = 0; t < TG; t++) {
        if (t < nt) {
            cpx<T> *vt = L.V + (long long)(t0 + t) * S;
#pragma unroll
            for (int j = 0; j < RB; j++) {
                const int rr = rbase + j * RW;
                if (rr < nrhs) {
                    vt[(long long)rr * K + q] = acc[t][0][j];
                    vt[half + (long long)rr * K + q] = acc[t][1][j];
                }
            }
        }
    }
}

// Translation on the matrix cores, for groups of up to 16 targets (whole
// sibling sets merged).  For one sample q a group's sums are a complex
// product
//   D[col][t] = sum_s U_s[col](q) T_{o(t, s)}(q),
// col = (component, right-hand side) and s running over the union of the
// targets' sources, four sources per MFMA step (T = 0 where s is not in
// t's list).  A wave takes QT consecutive samples (one accumulator pair per
// sample) and CT tiles of 16 columns; lane l feeds column and target l % 16
// and source slot l / 16 of a step, and loads its QT samples of one U row
// and one operator row as a run.  The next step's operands are loaded while
// the current step's MFMAs run.  Workgroups are ordered as in the
// sibling-group kernel (group innermost, every XCD a contiguous range).
template <class T, int QT, int CT>
__global__ __launch_bounds__(GWAVES * WAVE) void k_translate_mfma(const GroupArgs<T> a, int nrhs)
{
    typedef typename Mf<T>::v4 v4;
    const int xcd = blockIdx.x % NXCD, pos = blockIdx.x / NXCD;
    if (pos >= a.nblocks) return;
    int l = 0;
    while (l + 1 < a.nlev && pos >= a.lv[l + 1].first) l++;
    const GroupLevel<T> &L = a.lv[l];
    const int ncol = 2 * nrhs, nct = (ncol + 16 * CT - 1) / (16 * CT);
    const int nblk = L.ngroup * nct * L.nqc, per = (nblk + NXCD - 1) / NXCD;
    const int lb = xcd * per + (pos - L.first);
    if (lb >= nblk) return;
    const int g = lb % L.ngroup, rest = lb / L.ngroup;
    const int ct = rest % nct, qc = rest / nct;
    const int K = L.K;
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int q0 = (qc * GWAVES + wave) * QT;
    if (q0 >= K) return;
    const bool full = q0 + QT <= K;
    const int qlast = K - 1 - q0;   // last valid sample of the run
    const int lo = lane & 15, kk = lane >> 4;
    const long long S = (long long)ncol * K;   // one box's patterns
    long long co[CT];   // this lane's column rows (clamped to a valid one)
#pragma unroll
    for (int c = 0; c < CT; c++) co[c] = (long long)min((ct * CT + c) * 16 + lo, ncol - 1) * K + q0;
    const int t0 = ldu(L.first_tgt, g), nt = ldu(L.count, g);
    const int r0 = ldu(L.rec_start, g), r1 = ldu(L.rec_start, g + 1);
    v4 dre[CT][QT], dim[CT][QT];
#pragma unroll
    for (int c = 0; c < CT; c++)
#pragma unroll
        for (int u = 0; u < QT; u++) dre[c][u] = dim[c][u] = v4{0, 0, 0, 0};
    cpx<T> un[CT][QT], tn[QT];
    const int *srcp = L.src, *offp = L.off;
    const cpx<T> *Ub = L.U, *Tb = L.trans + q0;
    auto load = [&](int r) {
        const int rec = r + kk;
        const bool ok = rec < r1;
        const int sb = srcp[ok ? rec : r0];
        const int o = ok ? offp[(long long)rec * 16 + lo] : -1;
        const cpx<T> *us = Ub + (long long)sb * S;
        const cpx<T> *tp = Tb + (long long)max(o, 0) * K;
        if (full) {
#pragma unroll
            for (int c = 0; c < CT; c++)
#pragma unroll
                for (int u = 0; u < QT; u++) un[c][u] = us[co[c] + u];
#pragma unroll
            for (int u = 0; u < QT; u++) tn[u] = tp[u];
        } else {
#pragma unroll
            for (int c = 0; c < CT; c++)
#pragma unroll
                for (int u = 0; u < QT; u++) un[c][u] = us[co[c] + min(u, qlast)];
#pragma unroll
            for (int u = 0; u < QT; u++) tn[u] = tp[min(u, qlast)];
        }
        if (o < 0)
#pragma unroll
            for (int u = 0; u < QT; u++) tn[u] = mk<T>(0, 0);
    };
    if (r0 < r1) load(r0);
    for (int r = r0; r < r1; r += 4) {
        cpx<T> uc[CT][QT], tc[QT];
#pragma unroll
        for (int u = 0; u < QT; u++) {
            tc[u] = tn[u];
#pragma unroll
            for (int c = 0; c < CT; c++) uc[c][u] = un[c][u];
        }
        if (r + 4 < r1) load(r + 4);
#pragma unroll
        for (int u = 0; u < QT; u++)
#pragma unroll
            for (int c = 0; c < CT; c++) dre[c][u] = Mf<T>::mma(uc[c][u].re, tc[u].re, dre[c][u]);
#pragma unroll
        for (int u = 0; u < QT; u++)
#pragma unroll
            for (int c = 0; c < CT; c++) dim[c][u] = Mf<T>::mma(uc[c][u].re, tc[u].im, dim[c][u]);
#pragma unroll
        for (int u = 0; u < QT; u++)
#pragma unroll
            for (int c = 0; c < CT; c++) dre[c][u] = Mf<T>::mma(-uc[c][u].im, tc[u].im, dre[c][u]);
#pragma unroll
        for (int u = 0; u < QT; u++)
#pragma unroll
            for (int c = 0; c < CT; c++) dim[c][u] = Mf<T>::mma(uc[c][u].im, tc[u].re, dim[c][u]);
    }
    if (lo >= nt) return;
    cpx<T> *vt = L.V + (long long)(t0 + lo) * S + q0;
#pragma unroll
    for (int c = 0; c < CT; c++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int col = (ct * CT + c) * 16 + Mf<T>::row(kk, v);
            if (col >= ncol) continue;
#pragma unroll
            for (int u = 0; u < QT; u++)
                if (full || u <= qlast) vt[(long long)col * K + u] = mk<T>(dre[c][u][v], dim[c][u][v]);
        }
}

}  // namespace


// the LDS-operator kernel: (targets per group, lanes over the RHS, RHS per
// lane) in {8, 16} x {(4, 4), (8, 2), (16, 1), (8, 1)}, double precision only
// with at most 8 samples per wave (the LDS table) and TG * RB <= 16
template <class T>
bool launch_translate_lds(const GroupArgs<T> &args, int nrhs, hipStream_t s)
{
    const int tg = args.tg;
    int rw = args.rw, rb = args.rb;
    const bool shape = (rw == 4 && rb == 4) || (rw == 8 && rb == 2) || (rw == 16 && rb == 1) || (rw == 8 && rb == 1);
    if ((tg != 8 && tg != 16) || !shape || tg * rb > 32) return false;
    if (sizeof(T) == 8 && (rw < 8 || tg * rb > 16)) return false;
    if (args.nlev <= 0 || nrhs <= 0) return true;
    // a shape tuned for more right-hand sides than this call has: eight
    // lanes over them, or (groups of 8, fewer than 8 RHS) the register
    // kernel's default split
    if (rw * rb > nrhs) {
        if (tg == 8 && nrhs < 8) {
            GroupArgs<T> b = args;
            b.lds = 0;
            b.rw = 0;
            b.rb = 1;
            return launch_translate_groups<T>(b, nrhs, s);
        }
        rw = 8;
        rb = 1;
    }
    for (int l = 0; l < args.nlev; l++)   // 32-bit byte offsets within one box's patterns
        if (2.0 * nrhs * args.lv[l].K * sizeof(cpx<T>) >= 4294967296.0) return false;
    const int qw = WAVE / rw;
    GroupArgs<T> a = args;
    a.nblocks = 0;
    for (int l = 0; l < a.nlev; l++) {
        const int ngb = (a.lv[l].ngroup + GWAVES - 1) / GWAVES;
        a.lv[l].nqc = (a.lv[l].K + qw - 1) / qw;
        a.lv[l].first = a.nblocks;
        a.nblocks += (ngb * a.lv[l].nqc + NXCD - 1) / NXCD;
    }
    if (a.nblocks <= 0) return true;
    const dim3 grid((unsigned)a.nblocks * NXCD, (nrhs + rw * rb - 1) / (rw * rb)), block(GWAVES * WAVE);
#define LDS_LAUNCH(TG_, RW_, RB_) hipLaunchKernelGGL((k_translate_lds<T, TG_, RW_, RB_>), grid, block, 0, s, a, nrhs)
    if constexpr (sizeof(T) == 4) {
        if (tg == 8) {
            if (rw == 4) LDS_LAUNCH(8, 4, 4);
            else if (rw == 16) LDS_LAUNCH(8, 16, 1);
            else if (rb == 2) LDS_LAUNCH(8, 8, 2);
            else LDS_LAUNCH(8, 8, 1);
        } else {
            if (rw == 16) LDS_LAUNCH(16, 16, 1);
            else if (rb == 2) LDS_LAUNCH(16, 8, 2);
            else if (rw == 8) LDS_LAUNCH(16, 8, 1);
            else return false;
        }
    } else {
        if (tg == 8) {
            if (rw == 16) LDS_LAUNCH(8, 16, 1);
            else if (rb == 2) LDS_LAUNCH(8, 8, 2);
            else LDS_LAUNCH(8, 8, 1);
        } else {
            if (rw == 16) LDS_LAUNCH(16, 16, 1);
            else if (rb == 1) LDS_LAUNCH(16, 8, 1);
            else return false;
        }
    }
#undef LDS_LAUNCH
    return true;
}

// the matrix-core kernel: args.rb = samples per wave (QT), args.rw = tiles of
// 16 columns per wave (CT)
template <class T>
bool launch_translate_mfma(const GroupArgs<T> &args, int nrhs, hipStream_t s)
{
    const int qt = args.rb, ct = args.rw;
    const bool ok = sizeof(T) == 4 ? ((qt == 4 || qt == 8) && (ct == 1 || ct == 2))
                                   : ((qt == 4 && (ct == 1 || ct == 2)) || (qt == 2 && ct == 2));
    if (!ok) return false;
    if (args.nlev <= 0 || nrhs <= 0) return true;
    const int nct = (2 * nrhs + 16 * ct - 1) / (16 * ct);
    GroupArgs<T> a = args;
    a.nblocks = 0;
    for (int l = 0; l < a.nlev; l++) {
        a.lv[l].nqc = (a.lv[l].K + GWAVES * qt - 1) / (GWAVES * qt);
        a.lv[l].first = a.nblocks;
        a.nblocks += (a.lv[l].ngroup * nct * a.lv[l].nqc + NXCD - 1) / NXCD;
    }
    if (a.nblocks <= 0) return true;
    const dim3 grid((unsigned)a.nblocks * NXCD), block(GWAVES * WAVE);
#define MFMA_LAUNCH(QT_, CT_) hipLaunchKernelGGL((k_translate_mfma<T, QT_, CT_>), grid, block, 0, s, a, nrhs)
    if constexpr (sizeof(T) == 4) {
        if (qt == 8 && ct == 2) MFMA_LAUNCH(8, 2);
        else if (qt == 8) MFMA_LAUNCH(8, 1);
        else if (ct == 2) MFMA_LAUNCH(4, 2);
        else MFMA_LAUNCH(4, 1);
    } else {
        if (qt == 2) MFMA_LAUNCH(2, 2);
        else if (ct == 2) MFMA_LAUNCH(4, 2);
        else MFMA_LAUNCH(4, 1);
    }
#undef MFMA_LAUNCH
    return true;
}

template <class T>
bool launch_translate_groups(const GroupArgs<T> &args, int nrhs, hipStream_t s)
{
    const int tg = args.tg;
    if (args.lds) return launch_translate_lds<T>(args, nrhs, s);
    if (tg == 16) return launch_translate_mfma<T>(args, nrhs, s);
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
    for (int l = 0; l < args.nlev; l++)   // 32-bit byte offsets within one box's patterns
        if (2.0 * nrhs * args.lv[l].K * sizeof(cpx<T>) >= 4294967296.0) return false;
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
