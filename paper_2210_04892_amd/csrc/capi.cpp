// C boundary of the library: handle life cycle, device tables, and the
// launch sequence of one MLFMA matrix-vector product.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <tuple>
#include <memory>
#include <string>
#include <type_traits>
#include <thread>
#include <vector>

#include "../../include/mlfma.h"
#include "device.hpp"
#include "nearfield.hpp"
#include "sai.hpp"
#include "scratch.hpp"
#include "setup.hpp"

using namespace mlfma;

namespace {

thread_local std::string g_last_error;

#define HIPCHK(call)                                                                                     \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess)                                                                            \
            throw Error(e_ == hipErrorOutOfMemory ? MLFMA_ERR_OOM : MLFMA_ERR_HIP,                       \
                        std::string(#call) + ": " + hipGetErrorString(e_));                             \
    } while (0)

// Scoped switch to the handle's device (restores the caller's device).
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (dev >= 0 && dev != prev) HIPCHK(hipSetDevice(dev));
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Per-level device tables in one precision.
// theta-row chunks of one aggregation or disaggregation step (see LevelStep)
struct StepPlan {
    int rows = 0, nchunk = 0, wrows = 0;
    int *win = nullptr;
};

template <class T>
struct PrecLevel {
    cpx<T> *trans = nullptr, *shift = nullptr;
    T *ath_w = nullptr, *aph_w = nullptr, *dph_w = nullptr, *dth_w = nullptr;
    StepPlan agg, dis;      // step from level l + 1 up to l, and from l down to l + 1
    StepPlan agg1, dis1;    // the same with smaller chunks (more workgroups) for fewer than four RHS
    int agg_rb = 0, dis_rb = 0;   // right-hand sides per workgroup with four or more (autotuned; 0 = default)
    int agg_group = 0;            // aggregation: children staged together (autotuned; 0 = default)
    int agg_two = 0, dis_two = 0; // 1: the step as two kernels through the global intermediate (autotuned)
    int dis_pipe = 0;             // > 0: pipelined disaggregation with this many vectors per pass (autotuned)
    int agg_pipe = 0;             // the same for the aggregation
    // separable aggregation stencils (SepStencil; tth = 0: not separable)
    int ag_tth = 0, ag_tphi = 0;
    int *ag_th_row = nullptr, *ag_th_sh = nullptr, *ag_phi_col = nullptr;
    T *ag_th_w = nullptr, *ag_phi_w = nullptr;
    int tphi = 0, tth = 0;  // separable disaggregation stencils (0 = not separable)
    int *phi_col = nullptr, *th_row = nullptr, *th_sh = nullptr;
    T *phi_w = nullptr, *rowf = nullptr, *th_w = nullptr;
    // the step to level l + 1 on the matrix cores (complex64 only)
    StepMfma agg_m, dis_m;
    // translation tiles (a batch of sources fills 32 KB of LDS)
    int ntile = 0;
    int *tile_tgt = nullptr, *tile_bat = nullptr, *bat_src = nullptr, *src = nullptr;
    int *bat_row = nullptr, *row = nullptr, *ent = nullptr;
};


template <class T>
struct Prec {
    cpx<T> *R = nullptr, *Q = nullptr;           // leaf patterns, [rwg][sample][2]
    T *wq = nullptr;                              // receive weights (c0 folded)
    cpx<T> *near_em = nullptr, *near_c = nullptr; // near blocks, (A, B) per slot
    T *id_w = nullptr;                            // identity terms (gram, gx)
    std::vector<PrecLevel<T>> lv;
    int trans_tmax = 0, trans_smax = 0, trans_rb = 1;   // translation tile shape (autotuned)
    int trans_group = 0;                          // > 0: sibling-group kernel with this many targets per group
    int trans_rw = 0;                             // its lanes over the right-hand sides (0: default)
    int trans_gi = 0;                             // its group table (group_args)
    int trans_lds = 0;                            // 1: its operator values staged in LDS
    int level_mfma = 0;                           // level steps on the matrix cores (complex64, autotuned)
    int mfma_ends = 1;                            // near field, radiation and receive on the matrix cores
    double step_ms[2] = {0, 0};                   // timed level steps: vector, matrix cores
    double trans_ms = 0;                          // its timed translation, ms
};

constexpr int NGROUP_TABLES = 4;
// targets per group of group table gi
inline int group_tg(int gi) { return gi == 0 ? 4 : (gi == 3 ? 16 : 8); }

struct IntLevel {
    // sibling groups of the translation: 4 targets, 8 targets, 8 targets of
    // merged whole sibling sets (register-blocked kernel), 16 targets of
    // merged whole sibling sets (matrix-core kernel)
    int g_ngroup[NGROUP_TABLES] = {};
    int *g_first[NGROUP_TABLES] = {}, *g_count[NGROUP_TABLES] = {}, *g_rec[NGROUP_TABLES] = {};
    int *g_src[NGROUP_TABLES] = {}, *g_off[NGROUP_TABLES] = {};
    int *il_start = nullptr, *il_box = nullptr, *il_off = nullptr;
    int *child_start = nullptr, *parent = nullptr, *oct = nullptr;
    int *ath_s = nullptr, *ath_c = nullptr, *aph_s = nullptr, *aph_c = nullptr;
    int *dph_s = nullptr, *dph_c = nullptr, *dth_s = nullptr, *dth_c = nullptr;
};

// Per-product scratch: internal vectors, box patterns of every level and the
// stencil intermediate, sized for `rhs` right-hand sides in complex double
// units (the complex float path uses the first half of every buffer).
struct Workspace {
    int rhs = 0;
    unsigned long long bytes = 0;
    std::vector<void *> allocs;
    void *X = nullptr, *Y = nullptr, *mid = nullptr;
    void *X2 = nullptr, *Y2 = nullptr;   // complex64 copies in the caller's layout (products with FP32 parts)
    std::vector<void *> U, V;
    // optional second stream (not owned): the near field then runs beside
    // the far-field chain, forked after the radiation and joined before the
    // receive step
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    void release()
    {
        for (void *p : allocs) (void)hipFree(p);
        allocs.clear();
        rhs = 0;
        bytes = 0;
    }
};

// Sparse approximate inverse of one operator's near field (sai.hpp): the
// columns in both precisions and the row-wise entry lists of the apply.
struct SaiData {
    bool ready = false;
    int k = 0, maxp = 0;
    long long nnz = 0;          // RWG-pair entries (each a 2 x 2 block)
    double build_ms = 0;
    cpx<double> *M64 = nullptr;
    cpx<float> *M32 = nullptr;
    int *row_start = nullptr, *ent_col = nullptr, *ent_val = nullptr;
    std::vector<void *> allocs;
    unsigned long long bytes = 0;
};

}  // namespace

struct mlfma_ctx {
    mlfma_options opt{};
    int device = 0;
    Surface s;
    RwgTable r;
    Tree tr;
    std::vector<void *> allocs;
    unsigned long long bytes = 0;
    // integer tables
    int *perm = nullptr, *iperm = nullptr, *leaf_of = nullptr, *box_start = nullptr;
    int *near_start = nullptr, *near_box = nullptr, *id_start = nullptr, *id_col = nullptr;
    long long *val_off = nullptr;
    // matrix-core near field and receive: (leaf box, row tile) work items and
    // the column lists of the near-field block rows
    int n_items = 0;
    int2 *items = nullptr;
    int *col_off = nullptr, *cols = nullptr;
    // geometry on the device (internal RWG order): triangles and RWG pieces
    int *g_rtri = nullptr, *g_rloc = nullptr;
    double *g_rcoef = nullptr, *g_tv = nullptr, *g_tn = nullptr, *g_ta = nullptr;
    std::vector<IntLevel> lv;
    Prec<double> p64;
    Prec<float> p32;
    bool near_ready = false;
    bool mixed = false;       // complex128 products with an FP32 part (options)
    SaiData sai[2];           // per op (MLFMA_OP_C, MLFMA_OP_EM)
    hipStream_t side = nullptr;                    // near-field stream of ws
    hipEvent_t fork = nullptr, join = nullptr;
    hipStream_t bstream = nullptr;                 // this handle's products in mlfma_matvec_batch
    hipEvent_t bfork = nullptr, bjoin = nullptr;
    Workspace ws;             // workspace of mlfma_matvec_LK / mlfma_matvec_part
    long long ws_gen = 0;     // bumped whenever ws is reallocated (captured graphs refer to it)
    long long uid = 0;        // unique over the process (keys of the server's captured products)
    // stage profiling
    bool prof = false;
    std::vector<hipEvent_t> ev_free;
    std::vector<std::vector<hipEvent_t>> ev_pending;
    // host tables of the tiled translation per (targets per tile, sources
    // per batch), kept only while the autotuner runs
    std::map<std::pair<int, int>, std::vector<TransTiles>> tile_cache;
    double stage_ms[MLFMA_STAGES] = {0};
    long long prof_calls = 0;
    long long n_touch = 0, n_slots = 0, n_id = 0;

    template <class T>
    T *dalloc(size_t count, std::vector<void *> *list = nullptr)
    {
        size_t nbytes = std::max<size_t>(count, 1) * sizeof(T);
        if (opt.hbm_budget_bytes && bytes + nbytes > opt.hbm_budget_bytes)
            throw Error(MLFMA_ERR_OOM, "device memory budget exceeded");
        void *p = nullptr;
        HIPCHK(hipMalloc(&p, nbytes));
        (list ? list : &allocs)->push_back(p);
        bytes += nbytes;
        return static_cast<T *>(p);
    }
    template <class T>
    T *upload(const std::vector<T> &h)
    {
        T *d = dalloc<T>(h.size());
        if (!h.empty()) HIPCHK(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
        return d;
    }
    void free_ws()
    {
        ws_gen++;             // graphs captured over the old buffers may no longer replay
        bytes -= ws.bytes;
        ws.release();
    }
    void free_sai(int op)
    {
        SaiData &d = sai[op];
        for (void *p : d.allocs) (void)hipFree(p);
        bytes -= d.bytes;
        d = SaiData();
    }
    std::vector<hipEvent_t> take_events()
    {
        std::vector<hipEvent_t> ev(MLFMA_STAGES + 1);
        for (auto &e : ev) {
            if (!ev_free.empty()) {
                e = ev_free.back();
                ev_free.pop_back();
            } else {
                HIPCHK(hipEventCreate(&e));
            }
        }
        return ev;
    }
    void drain_events()
    {
        for (auto &ev : ev_pending) {
            (void)hipEventSynchronize(ev.back());
            for (int s = 0; s < MLFMA_STAGES; s++) {
                float ms = 0;
                if (hipEventElapsedTime(&ms, ev[s], ev[s + 1]) == hipSuccess) stage_ms[s] += ms;
            }
            prof_calls++;
            for (auto e : ev) ev_free.push_back(e);
        }
        ev_pending.clear();
    }
    ~mlfma_ctx()
    {
        drain_events();
        for (auto e : ev_free) (void)hipEventDestroy(e);
        free_ws();
        free_sai(0);
        free_sai(1);
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        if (side) (void)hipStreamDestroy(side);
        if (bfork) (void)hipEventDestroy(bfork);
        if (bjoin) (void)hipEventDestroy(bjoin);
        if (bstream) (void)hipStreamDestroy(bstream);
        for (void *p : allocs) (void)hipFree(p);
    }
};

namespace {

template <class T>
std::vector<T> cast_vec(const std::vector<double> &v)
{
    return std::vector<T>(v.begin(), v.end());
}

template <class T>
std::vector<cpx<T>> cast_cvec(const std::vector<cdouble> &v)
{
    std::vector<cpx<T>> o(v.size());
    for (size_t i = 0; i < v.size(); i++) o[i] = {(T)v[i].real(), (T)v[i].imag()};
    return o;
}

template <class T>
void plan_level_steps(mlfma_ctx *c, int l, PrecLevel<T> &PL)
{
    const Tree &tr = c->tr;
    const Level &L = tr.lv[l], &C = tr.lv[l + 1];
    // chunks of about 512 outputs; for few right-hand sides about 256, which
    // doubles the workgroups of the small coarse levels
    ChunkPlan cp;
    for (int small = 0; small < 2; small++) {
        const int per = small ? 256 : 512;
        plan_theta_chunks(tr.agg_theta[l], L.nth, C.nph, std::max(1, per / L.nph),
                          [&](int wrows, int rows) { return agg_lds_bytes<T>(wrows, rows, C.nph); }, STEP_LDS_MAX,
                          cp);
        (small ? PL.agg1 : PL.agg) = {cp.rows, cp.nchunk, cp.wrows, cp.rows ? c->upload(cp.win) : nullptr};
    }
    SepStencil sa;
    if (separable_aggregation(L, C, tr.agg_phi[l], tr.agg_theta[l], sa)) {
        PL.ag_tth = sa.tth;
        PL.ag_tphi = sa.tphi;
        PL.ag_th_row = c->upload(sa.th_row);
        PL.ag_th_sh = c->upload(sa.th_sh);
        PL.ag_th_w = c->upload(cast_vec<T>(sa.th_w));
        PL.ag_phi_col = c->upload(sa.phi_col);
        PL.ag_phi_w = c->upload(cast_vec<T>(sa.phi_w));
    }
    SepStencil sep;
    if (!separable_disaggregation(L, C, tr.dis_phi[l], tr.dis_theta[l], sep)) return;
    for (int small = 0; small < 2; small++) {
        const int per = small ? 256 : 512;
        plan_theta_chunks(tr.dis_theta[l], C.nth, C.nph, std::max(1, per / C.nph),
                          [&](int wrows, int) { return dis_lds_bytes<T>(wrows, L.nph, C.nph); }, STEP_LDS_MAX, cp);
        (small ? PL.dis1 : PL.dis) = {cp.rows, cp.nchunk, cp.wrows, cp.rows ? c->upload(cp.win) : nullptr};
    }
    PL.tphi = sep.tphi;
    PL.tth = sep.tth;
    PL.phi_col = c->upload(sep.phi_col);
    PL.th_row = c->upload(sep.th_row);
    PL.th_sh = c->upload(sep.th_sh);
    PL.phi_w = c->upload(cast_vec<T>(sep.phi_w));
    PL.rowf = c->upload(cast_vec<T>(sep.rowf));
    PL.th_w = c->upload(cast_vec<T>(sep.th_w));
}

// The step between parent level l and child level l + 1 as dense real
// matrices for the matrix-core kernels, checked to be separable: the theta
// interpolation the same for every child phi column (up to the half turn of
// the pole extension), the phi interpolation the same for every parent theta
// row; the anterpolation from the separable form (SepStencil).
void build_step_mfma(mlfma_ctx *c, int l, StepMfma &agg, StepMfma &dis)
{
    const Tree &tr = c->tr;
    const Level &L = tr.lv[l], &C = tr.lv[l + 1];
    agg = StepMfma();
    dis = StepMfma();
    const int nthp = L.nth, nphp = L.nph, nthc = C.nth, nphc = C.nph, half = nphc / 2;
    if (nphc % 2 || nphp > 128 || nthp > 64 || nphc > 256) return;
    const int npt = (nphp + 15) / 16, njt = (nphc + 15) / 16, nit = (nthp + 15) / 16, nict = (nthc + 15) / 16;
    // ---- aggregation
    const Csr &th = tr.agg_theta[l], &ph = tr.agg_phi[l];
    const int ne = 3 * nthc, e_pad = (ne + 3) / 4 * 4;
    std::vector<int> ext_row(ne), ext_sh(ne);
    for (int e = 0; e < ne; e++) {
        ext_row[e] = e < nthc ? nthc - 1 - e : (e < 2 * nthc ? e - nthc : 3 * nthc - 1 - e);
        ext_sh[e] = (e < nthc || e >= 2 * nthc) ? half : 0;
    }
    std::vector<float> ath((size_t)nit * 16 * e_pad, 0.f);
    std::vector<int> ks_lo(nit, 1 << 30), ks_hi(nit, 0);
    for (int ip = 0; ip < nthp; ip++) {
        const bool north = L.ct[ip] > 0;   // theta below pi/2: reflected nodes across the north pole
        struct Tap { int idx, refl; double w; };
        auto taps = [&](int jc, std::vector<Tap> &v) {
            v.clear();
            const int row = ip * nphc + jc;
            for (int e = th.start[row]; e < th.start[row + 1]; e++) {
                const int idx = th.col[e] / nphc, jj = th.col[e] % nphc;
                int refl;
                if (jj == jc) refl = 0;
                else if (jj == (jc + half) % nphc) refl = 1;
                else return false;
                v.push_back({idx, refl, th.w[e]});
            }
            std::sort(v.begin(), v.end(), [](const Tap &x, const Tap &y) { return x.idx != y.idx ? x.idx < y.idx : x.refl < y.refl; });
            return true;
        };
        std::vector<Tap> t0, tj;
        if (!taps(0, t0)) return;
        for (int jc = 1; jc < nphc; jc++) {
            if (!taps(jc, tj) || tj.size() != t0.size()) return;
            for (size_t i = 0; i < t0.size(); i++)
                if (tj[i].idx != t0[i].idx || tj[i].refl != t0[i].refl || std::abs(tj[i].w - t0[i].w) > 1e-13 * (1 + std::abs(t0[i].w)))
                    return;
        }
        for (const Tap &x : t0) {
            const int e = x.refl ? (north ? nthc - 1 - x.idx : 3 * nthc - 1 - x.idx) : nthc + x.idx;
            ath[(size_t)ip * e_pad + e] += (float)x.w;
            ks_lo[ip / 16] = std::min(ks_lo[ip / 16], e / 4);
            ks_hi[ip / 16] = std::max(ks_hi[ip / 16], e / 4 + 1);
        }
    }
    for (int it = 0; it < nit; it++) {
        if (ks_lo[it] > ks_hi[it]) ks_lo[it] = ks_hi[it] = 0;
        if (ks_hi[it] - ks_lo[it] > 8) return;   // the kernel holds at most 8 k-steps of one tile
    }
    const int jc_pad = njt * 16;
    std::vector<float> bph((size_t)npt * 16 * jc_pad, 0.f);
    for (int jp = 0; jp < nphp; jp++)
        for (int e = ph.start[jp]; e < ph.start[jp + 1]; e++) bph[(size_t)jp * jc_pad + ph.col[e]] += (float)ph.w[e];
    for (int ip = 1; ip < nthp; ip++)
        for (int jp = 0; jp < nphp; jp++) {
            const int row = ip * nphp + jp;
            if (ph.start[row + 1] - ph.start[row] != ph.start[jp + 1] - ph.start[jp]) return;
            for (int e = ph.start[row], e0 = ph.start[jp]; e < ph.start[row + 1]; e++, e0++)
                if (ph.col[e] != ip * nphc + ph.col[e0] || ph.w[e] != ph.w[e0]) return;
        }
    std::vector<unsigned> bmask(njt, 0u);
    for (int jp = 0; jp < nphp; jp++)
        for (int j = 0; j < nphc; j++)
            if (bph[(size_t)jp * jc_pad + j] != 0.f) bmask[j / 16] |= 1u << (jp / 16);
    // ---- disaggregation
    SepStencil sep;
    if (!separable_disaggregation(L, C, tr.dis_phi[l], tr.dis_theta[l], sep)) return;
    const int nks = (nphp + 3) / 4, jp_pad = nks * 4, nip = (nthp + 15) / 16, ip_pad = nip * 16;
    if (nks > 64) return;
    std::vector<float> dph((size_t)njt * 16 * jp_pad, 0.f);
    for (int j = 0; j < nphc; j++)
        for (int t = 0; t < sep.tphi; t++)
            dph[(size_t)j * jp_pad + sep.phi_col[(size_t)j * sep.tphi + t]] += (float)sep.phi_w[(size_t)j * sep.tphi + t];
    std::vector<unsigned long long> kmask(njt, 0ull), kmask_s(njt, 0ull);
    for (int j = 0; j < nphc; j++) {
        const int js = (j + half) % nphc;
        for (int jp = 0; jp < nphp; jp++) {
            if (dph[(size_t)j * jp_pad + jp] != 0.f) kmask[j / 16] |= 1ull << (jp / 4);
            if (dph[(size_t)js * jp_pad + jp] != 0.f) kmask_s[j / 16] |= 1ull << (jp / 4);
        }
    }
    std::vector<float> rowf(ip_pad, 0.f), dthd((size_t)nict * 16 * ip_pad, 0.f), dthr((size_t)nict * 16 * ip_pad, 0.f);
    for (int ip = 0; ip < nthp; ip++) rowf[ip] = (float)sep.rowf[ip];
    for (int ic = 0; ic < nthc; ic++)
        for (int t = 0; t < sep.tth; t++) {
            const size_t k = (size_t)ic * sep.tth + t;
            if (sep.th_w[k] == 0) continue;
            if (sep.th_sh[k] == 0) dthd[(size_t)ic * ip_pad + sep.th_row[k]] += (float)sep.th_w[k];
            else if (sep.th_sh[k] == half) dthr[(size_t)ic * ip_pad + sep.th_row[k]] += (float)sep.th_w[k];
            else return;
        }
    std::vector<unsigned> dmask(nict, 0u), rmask_c(nict, 0u);
    unsigned rmask = 0;
    for (int ic = 0; ic < nthc; ic++)
        for (int ip = 0; ip < nthp; ip++) {
            if (dthd[(size_t)ic * ip_pad + ip] != 0.f) dmask[ic / 16] |= 1u << (ip / 16);
            if (dthr[(size_t)ic * ip_pad + ip] != 0.f) {
                rmask_c[ic / 16] |= 1u << (ip / 16);
                rmask |= 1u << (ip / 16);
            }
        }
    // ---- device tables
    StepMfma base;
    base.nth_p = nthp;
    base.nph_p = nphp;
    base.nth_c = nthc;
    base.nph_c = nphc;
    base.child_start = c->lv[l].child_start;
    base.parent = c->lv[l + 1].parent;
    base.oct = c->lv[l + 1].oct;
    base.shift = c->p32.lv[l].shift;
    base.njt = njt;
    agg = base;
    agg.nbox = L.nbox;
    agg.nit = nit;
    agg.ne = ne;
    agg.e_pad = e_pad;
    agg.jc_pad = jc_pad;
    agg.ext_row = c->upload(ext_row);
    agg.ext_sh = c->upload(ext_sh);
    agg.ks_lo = c->upload(ks_lo);
    agg.ks_hi = c->upload(ks_hi);
    agg.ath = c->upload(ath);
    agg.bph = c->upload(bph);
    agg.bmask = c->upload(bmask);
    agg.ok = 1;
    dis = base;
    dis.nbox = C.nbox;
    dis.nks = nks;
    dis.jp_pad = jp_pad;
    dis.nict = nict;
    dis.ip_pad = ip_pad;
    dis.rmask = rmask;
    dis.kmask = c->upload(kmask);
    dis.kmask_s = c->upload(kmask_s);
    dis.dph = c->upload(dph);
    dis.rowf = c->upload(rowf);
    dis.dthd = c->upload(dthd);
    dis.dthr = c->upload(dthr);
    dis.dmask = c->upload(dmask);
    dis.rmask_c = c->upload(rmask_c);
    dis.ok = 1;
}

template <class T>
void upload_level_tables(mlfma_ctx *c, Prec<T> &P, const std::vector<std::vector<cdouble>> &trans,
                         const std::vector<std::vector<cdouble>> &shift)
{
    const Tree &tr = c->tr;
    P.lv.assign(tr.levels, PrecLevel<T>());
    for (int l = 2; l < tr.levels; l++) {
        P.lv[l].trans = c->upload(cast_cvec<T>(trans[l]));
        if (l + 1 < tr.levels) {
            P.lv[l].shift = c->upload(cast_cvec<T>(shift[l]));
            P.lv[l].ath_w = c->upload(cast_vec<T>(tr.agg_theta[l].w));
            P.lv[l].aph_w = c->upload(cast_vec<T>(tr.agg_phi[l].w));
            P.lv[l].dph_w = c->upload(cast_vec<T>(tr.dis_phi[l].w));
            P.lv[l].dth_w = c->upload(cast_vec<T>(tr.dis_theta[l].w));
            plan_level_steps<T>(c, l, P.lv[l]);
        }
    }
}

// translation tiles of every level for one tile shape; allocations go to
// `list` (tuning trials) or to the handle
// The tiled translation's tables of every level for one tile shape, built on
// host threads (one per level) and kept while the handle is built: the
// autotuner's candidates of both precisions share them.
const std::vector<TransTiles> &tiles_for(mlfma_ctx *c, int tmax, int smax)
{
    auto &slot = c->tile_cache[{tmax, smax}];
    if (slot.empty()) {
        const Tree &tr = c->tr;
        slot.resize(tr.levels);
        std::vector<std::thread> pool;
        for (int l = 2; l < tr.levels; l++)
            pool.emplace_back([&, l] { build_translation_tiles(tr.lv[l], smax, tmax, slot[l]); });
        for (auto &t : pool) t.join();
    }
    return slot;
}

template <class T>
void upload_trans_tiles(mlfma_ctx *c, Prec<T> &P, int tmax, int smax, std::vector<void *> *list)
{
    const Tree &tr = c->tr;
    const std::vector<TransTiles> &tiles = tiles_for(c, tmax, smax);
    for (int l = 2; l < tr.levels; l++) {
        const TransTiles &tt = tiles[l];
        PrecLevel<T> &PL = P.lv[l];
        auto up = [&](const std::vector<int> &v) {
            int *d = c->dalloc<int>(v.size(), list);
            if (!v.empty()) HIPCHK(hipMemcpy(d, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice));
            return d;
        };
        PL.ntile = (int)tt.tile_tgt.size() - 1;
        PL.tile_tgt = up(tt.tile_tgt);
        PL.tile_bat = up(tt.tile_bat);
        PL.bat_src = up(tt.bat_src);
        PL.src = up(tt.src);
        PL.bat_row = up(tt.bat_row);
        PL.row = up(tt.row);
        PL.ent = up(tt.ent);
    }
    P.trans_tmax = tmax;
    P.trans_smax = smax;
}

// translation arguments of every level (only_level >= 0: that level alone)
template <class T>
TransArgs<T> trans_args(mlfma_ctx *c, Prec<T> &P, Workspace &w, int only_level)
{
    const Tree &tr = c->tr;
    TransArgs<T> ta;
    ta.smax = P.trans_smax;
    ta.tmax = P.trans_tmax;
    ta.rb = P.trans_rb;
    for (int l = 2; l < tr.levels; l++) {
        if (only_level >= 0 && l != only_level) continue;
        const PrecLevel<T> &PL = P.lv[l];
        TransLevel<T> &d = ta.lv[ta.nlev++];
        d.K = tr.lv[l].K;
        d.ntile = PL.ntile;
        d.tile_tgt = PL.tile_tgt;
        d.tile_bat = PL.tile_bat;
        d.bat_src = PL.bat_src;
        d.src = PL.src;
        d.bat_row = PL.bat_row;
        d.row = PL.row;
        d.ent = PL.ent;
        d.trans = PL.trans;
        d.U = (const cpx<T> *)w.U[l];
        d.V = (cpx<T> *)w.V[l];
    }
    return ta;
}

// arguments of the sibling-group translation with group table gi (0: 4
// targets, 1: 8 targets, 2: 8 targets of merged sibling sets)
template <class T>
GroupArgs<T> group_args(mlfma_ctx *c, Prec<T> &P, Workspace &w, int only_level, int gi, int rb, int rw, int lds = 0)
{
    const Tree &tr = c->tr;
    GroupArgs<T> ga;
    ga.tg = group_tg(gi);
    ga.rb = rb;
    ga.rw = rw;
    ga.lds = lds;
    for (int l = 2; l < tr.levels; l++) {
        if (only_level >= 0 && l != only_level) continue;
        const IntLevel &I = c->lv[l];
        GroupLevel<T> &d = ga.lv[ga.nlev++];
        d.K = tr.lv[l].K;
        d.ngroup = I.g_ngroup[gi];
        d.first_tgt = I.g_first[gi];
        d.count = I.g_count[gi];
        d.rec_start = I.g_rec[gi];
        d.src = I.g_src[gi];
        d.off = I.g_off[gi];
        d.trans = P.lv[l].trans;
        d.U = (const cpx<T> *)w.U[l];
        d.V = (cpx<T> *)w.V[l];
    }
    return ga;
}

// The sibling-group shape a call with nrhs right-hand sides runs: the tuned
// one (whose launcher narrows a shape wider than the call: eight lanes over
// the right-hand sides, or for 8-target groups and fewer than 8 of them the
// register kernel), except that a tuned LDS-operator shape on 16-target
// groups gives way, below 8 right-hand sides (its lanes would idle), to the
// register kernel on the merged 8-target groups with the default lane split.
struct TransShape {
    int gi, rb, rw, lds;
};
template <class T>
TransShape trans_shape(const Prec<T> &P, int nrhs)
{
    if (P.trans_group <= 0) return {0, 1, 0, 0};
    if (P.trans_lds && P.trans_gi == 3 && nrhs < 8) return {2, 1, 0, 0};
    return {P.trans_gi, P.trans_rb, P.trans_rw, P.trans_lds};
}

// the translation of all levels (or of only_level) with the tuned kernel
template <class T>
void launch_translation(mlfma_ctx *c, Prec<T> &P, Workspace &w, int only_level, int nrhs, hipStream_t st)
{
    if (P.trans_group > 0) {
        const TransShape gs = trans_shape(P, nrhs);
        if (!launch_translate_groups<T>(group_args<T>(c, P, w, only_level, gs.gi, gs.rb, gs.rw, gs.lds), nrhs, st))
            throw Error(MLFMA_ERR_STATE, "invalid sibling-group translation shape");
    } else if (!launch_translate_tiled<T>(trans_args<T>(c, P, w, only_level), nrhs, st)) {
        throw Error(MLFMA_ERR_STATE, "translation tiles missing");
    }
}

// Autotuner of the translation: every candidate of the LDS-tiled kernel
// (targets per tile 4/8/16, LDS batch of 16/32/64 KB, 1/2/4 right-hand sides
// per lane) that satisfies the kernel's limits and of the sibling-group
// kernel (4 or 8 targets per group, lanes and right-hand sides per lane), or
// with MLFMA_TRANS_MATRIX of the matrix-core kernel (16-target groups,
// samples and column tiles per wave), is timed on the device (HIP events, one warm-up and three timed launches of
// the translation of all levels with the right-hand-side count the handle
// is built for, capped at 16); the fastest is kept.
template <class T>
void tune_translation(mlfma_ctx *c, Prec<T> &P)
{
    const Tree &tr = c->tr;
    if (tr.levels < 3) {
        P.trans_rb = 1;
        upload_trans_tiles<T>(c, P, 8, 16, nullptr);
        return;
    }
    const int nrhs = std::min(c->opt.max_rhs, 16);
    hipStream_t st;
    HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    double best = 1e300;
    int bt = 0, bs = 0, bb = 1;
    for (int rb : {1, 2, 4}) {
        if (rb > 1 && (trans_rw(nrhs) != 4 || nrhs < 4 * rb)) continue;
        if (c->opt.trans_kernel != MLFMA_TRANS_AUTO && c->opt.trans_kernel != MLFMA_TRANS_TILED) break;
        for (int tmax : {4, 8, 16})
            for (int kb : {16, 32, 64}) {
                const int smax = (kb * 1024) / (int)(2 * 64 * rb * sizeof(cpx<T>));
                if (!trans_shape_ok(tmax, smax, rb)) continue;
                struct Trial {
                    mlfma_ctx *c;
                    unsigned long long b0;
                    std::vector<void *> list;
                    ~Trial()
                    {
                        for (void *p : list) (void)hipFree(p);
                        c->bytes = b0;
                    }
                } trial{c, c->bytes, {}};
                upload_trans_tiles<T>(c, P, tmax, smax, &trial.list);
                P.trans_rb = rb;
                const TransArgs<T> ta = trans_args<T>(c, P, c->ws, -1);
                if (!launch_translate_tiled<T>(ta, nrhs, st)) throw Error(MLFMA_ERR_HIP, "invalid translation tile shape");
                HIPCHK(hipEventRecord(e0, st));
                for (int i = 0; i < 3; i++) launch_translate_tiled<T>(ta, nrhs, st);
                HIPCHK(hipEventRecord(e1, st));
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) {
                    best = ms;
                    bt = tmax;
                    bs = smax;
                    bb = rb;
                }
            }
    }
    int bg = 0, bw = 0, bgi = 0, blds = 0;
    // sibling-group shapes: (lanes over the RHS, RHS per lane) within the
    // handle's right-hand sides (the default lane split always)
    const int shapes[9][2] = {{1, 1}, {2, 1}, {4, 1}, {4, 2}, {4, 4}, {8, 1}, {8, 2}, {16, 1}, {2, 8}};
    for (int gi : {0, 1, 2})
        for (const auto &sh : shapes) {
            if (c->opt.trans_kernel != MLFMA_TRANS_AUTO && c->opt.trans_kernel != MLFMA_TRANS_GROUPS) break;
            const int tg = group_tg(gi);
            const int rw = sh[0], rb = sh[1];
            const int def = trans_rw(nrhs);
            if (!(rw == def && rb == 1) && (rw * rb > nrhs || rw * rb < def)) continue;
            if (sizeof(T) == 8 && tg * rb > 8) continue;   // register budget of the double-precision sums
            if (rb == 8 && (tg != 4 || sizeof(T) != 4 || nrhs < 16)) continue;
            const GroupArgs<T> ga = group_args<T>(c, P, c->ws, -1, gi, rb, rw);
            if (!launch_translate_groups<T>(ga, nrhs, st)) throw Error(MLFMA_ERR_HIP, "invalid sibling-group shape");
            HIPCHK(hipEventRecord(e0, st));
            for (int i = 0; i < 3; i++) launch_translate_groups<T>(ga, nrhs, st);
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                bg = tg;
                bb = rb;
                bw = rw;
                bgi = gi;
                blds = 0;
            }
        }
    // the same with the operator values staged in LDS (merged groups of 8 or
    // 16 targets; shapes without a kernel are skipped)
    const int lshapes[4][2] = {{4, 4}, {8, 2}, {16, 1}, {8, 1}};
    for (int gi : {2, 3})
        for (const auto &sh : lshapes) {
            if (c->opt.trans_kernel != MLFMA_TRANS_AUTO && c->opt.trans_kernel != MLFMA_TRANS_GROUPS &&
                c->opt.trans_kernel != MLFMA_TRANS_LDS)
                break;
            const int rw = sh[0], rb = sh[1];
            if (rw * rb > nrhs && !(rw == trans_rw(nrhs) && rb == 1)) continue;
            const GroupArgs<T> ga = group_args<T>(c, P, c->ws, -1, gi, rb, rw, 1);
            if (!launch_translate_groups<T>(ga, nrhs, st)) continue;
            HIPCHK(hipEventRecord(e0, st));
            for (int i = 0; i < 3; i++) launch_translate_groups<T>(ga, nrhs, st);
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                bg = group_tg(gi);
                bb = rb;
                bw = rw;
                bgi = gi;
                blds = 1;
            }
        }
    // matrix-core kernel (16-target groups): (samples per wave, tiles of 16
    // columns per wave); two column tiles only where there are two.  Timed
    // only when asked for: on surface meshes a 16-target group's targets
    // share few sources (36-44 % of the target x source operand is nonzero
    // on a sphere of radius 8 wavelengths), so the matrix cores do 2-3x the
    // useful work and the kernel is slower than the sibling-group one.
    const int mshapes[4][2] = {{4, 1}, {8, 1}, {4, 2}, {8, 2}};
    const int dshapes[3][2] = {{4, 1}, {4, 2}, {2, 2}};
    for (int i = 0; i < (sizeof(T) == 4 ? 4 : 3); i++) {
        if (c->opt.trans_kernel != MLFMA_TRANS_MATRIX) break;
        const int qt = sizeof(T) == 4 ? mshapes[i][0] : dshapes[i][0];
        const int ct = sizeof(T) == 4 ? mshapes[i][1] : dshapes[i][1];
        if (ct == 2 && 2 * nrhs <= 16) continue;
        const GroupArgs<T> ga = group_args<T>(c, P, c->ws, -1, 3, qt, ct);
        if (!launch_translate_groups<T>(ga, nrhs, st)) throw Error(MLFMA_ERR_HIP, "invalid matrix-core translation shape");
        HIPCHK(hipEventRecord(e0, st));
        for (int k = 0; k < 3; k++) launch_translate_groups<T>(ga, nrhs, st);
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
            best = ms;
            bg = 16;
            bb = qt;
            bw = ct;
            bgi = 3;
            blds = 0;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    if (bg > 0) {
        // the tiled kernel's tables of its best shape are not needed; keep a
        // small valid set so that the kernel stays callable
        upload_trans_tiles<T>(c, P, 8, 16, nullptr);
        P.trans_group = bg;
        P.trans_rw = bw;
        P.trans_gi = bgi;
        P.trans_lds = blds;
    } else {
        upload_trans_tiles<T>(c, P, bt, bs, nullptr);
        P.trans_group = 0;
    }
    P.trans_rb = bb;
    P.trans_ms = best / 3;
}

void build_device_tables(mlfma_ctx *c)
{
    const Tree &tr = c->tr;
    const int N = c->r.n, leafl = tr.levels - 1;
    const double k = c->opt.wavenumber;
    c->perm = c->upload(tr.perm);
    c->iperm = c->upload(tr.iperm);
    c->leaf_of = c->upload(tr.leaf_of);
    c->box_start = c->upload(tr.box_start);
    c->near_start = c->upload(tr.near_start);
    c->near_box = c->upload(tr.near_box);
    {
        std::vector<int2> items;
        std::vector<int> off(1, 0), cols;
        for (size_t b = 0; b + 1 < tr.box_start.size(); b++) {
            const int rows = 2 * (tr.box_start[b + 1] - tr.box_start[b]);
            for (int t = 0; t * 16 < rows; t++) items.push_back(make_int2((int)b, t));
            for (int e = tr.near_start[b]; e < tr.near_start[b + 1]; e++)
                for (int i = tr.box_start[tr.near_box[e]]; i < tr.box_start[tr.near_box[e] + 1]; i++) cols.push_back(i);
            off.push_back((int)cols.size());
        }
        c->n_items = (int)items.size();
        c->items = c->upload(items);
        c->col_off = c->upload(off);
        c->cols = c->upload(cols);
    }
    c->lv.assign(tr.levels, IntLevel());
    std::vector<std::vector<cdouble>> trans(tr.levels), shift(tr.levels);
    for (int l = 2; l < tr.levels; l++) {
        const Level &L = tr.lv[l];
        IntLevel &I = c->lv[l];
        I.il_start = c->upload(L.il_start);
        I.il_box = c->upload(L.il_box);
        I.il_off = c->upload(L.il_off);
        I.parent = c->upload(L.parent);
        I.oct = c->upload(L.child_oct);
        for (int gi = 0; gi < NGROUP_TABLES; gi++) {
            GroupTiles gt;
            build_group_tiles(L, group_tg(gi), gt, gi >= 2);
            I.g_ngroup[gi] = (int)gt.first.size();
            I.g_first[gi] = c->upload(gt.first);
            I.g_count[gi] = c->upload(gt.count);
            I.g_rec[gi] = c->upload(gt.rec_start);
            I.g_src[gi] = c->upload(gt.src);
            I.g_off[gi] = c->upload(gt.off);
        }
        std::vector<double> khat;
        level_directions(L, khat);
        // translation operators for the 7^3 offsets (unused entries stay 0),
        // the offsets shared out over host threads (each writes its own rows)
        trans[l].assign(343 * (size_t)L.K, cdouble(0, 0));
        {
            const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
            auto work = [&](int first) {
                std::vector<cdouble> tl;
                for (int o = first; o < 343; o += nth) {
                    int d[3] = {o / 49 - 3, (o / 7) % 7 - 3, o % 7 - 3};
                    if (std::max(std::abs(d[0]), std::max(std::abs(d[1]), std::abs(d[2]))) < 2) continue;
                    double X[3] = {d[0] * L.a, d[1] * L.a, d[2] * L.a};
                    translation_table(k, L.L, X, khat, tl);
                    std::copy(tl.begin(), tl.end(), trans[l].begin() + (size_t)o * L.K);
                }
            };
            std::vector<std::thread> pool;
            for (int i = 1; i < nth; i++) pool.emplace_back(work, i);
            work(0);
            for (auto &t : pool) t.join();
        }
        if (l + 1 < tr.levels) {
            const Level &C = tr.lv[l + 1];
            std::vector<int> cs(L.nbox + 1, 0);
            for (int b = 0; b < C.nbox; b++) cs[C.parent[b] + 1]++;
            for (int b = 0; b < L.nbox; b++) cs[b + 1] += cs[b];
            I.child_start = c->upload(cs);
            // exp(+jk khat.(r_child - r_parent)), r_child - r_parent = (bit - 1/2) a_child
            shift[l].resize(8 * (size_t)L.K);
            for (int o = 0; o < 8; o++) {
                double off[3] = {((o >> 2) & 1) - 0.5, ((o >> 1) & 1) - 0.5, (o & 1) - 0.5};
                for (int q = 0; q < L.K; q++) {
                    double ph = k * C.a * (khat[3 * q] * off[0] + khat[3 * q + 1] * off[1] + khat[3 * q + 2] * off[2]);
                    shift[l][(size_t)o * L.K + q] = cdouble(std::cos(ph), std::sin(ph));
                }
            }
            I.ath_s = c->upload(tr.agg_theta[l].start);
            I.ath_c = c->upload(tr.agg_theta[l].col);
            I.aph_s = c->upload(tr.agg_phi[l].start);
            I.aph_c = c->upload(tr.agg_phi[l].col);
            I.dph_s = c->upload(tr.dis_phi[l].start);
            I.dph_c = c->upload(tr.dis_phi[l].col);
            I.dth_s = c->upload(tr.dis_theta[l].start);
            I.dth_c = c->upload(tr.dis_theta[l].col);
        }
    }
    upload_level_tables<double>(c, c->p64, trans, shift);
    upload_level_tables<float>(c, c->p32, trans, shift);
    for (int l = 2; l + 1 < tr.levels; l++) build_step_mfma(c, l, c->p32.lv[l].agg_m, c->p32.lv[l].dis_m);

    // geometry in internal RWG order (kept: near field, plane waves)
    {
        std::vector<int> rtri(2 * (size_t)N), rloc(2 * (size_t)N);
        std::vector<double> rcoef(2 * (size_t)N), tv(9 * (size_t)c->s.nt);
        for (int i = 0; i < N; i++) {
            int u = tr.perm[i];
            for (int h = 0; h < 2; h++) {
                rtri[2 * i + h] = c->r.tri[h][u];
                rloc[2 * i + h] = c->r.loc[h][u];
                rcoef[2 * i + h] = c->r.coef[h][u];
            }
        }
        for (int t = 0; t < c->s.nt; t++)
            for (int a = 0; a < 3; a++)
                for (int d = 0; d < 3; d++) tv[9 * (size_t)t + 3 * a + d] = c->s.v[3 * c->s.t[3 * t + a] + d];
        c->g_rtri = c->upload(rtri);
        c->g_rloc = c->upload(rloc);
        c->g_rcoef = c->upload(rcoef);
        c->g_tv = c->upload(tv);
        c->g_tn = c->upload(c->s.nrm);
        c->g_ta = c->upload(c->s.area);
    }
    if (tr.levels >= 3) {
        // leaf patterns on the device (double), then a single-precision copy
        const Level &L = tr.lv[leafl];
        std::vector<double> cen(3 * (size_t)N);
        for (int i = 0; i < N; i++)
            for (int d = 0; d < 3; d++) cen[3 * i + d] = L.centre[3 * tr.leaf_of[i] + d];
        std::vector<void *> tmp;
        const unsigned long long bytes_before = c->bytes;
        auto d_cen = c->dalloc<double>(cen.size(), &tmp);
        auto d_ct = c->dalloc<double>(L.ct.size(), &tmp);
        HIPCHK(hipMemcpy(d_cen, cen.data(), cen.size() * 8, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(d_ct, L.ct.data(), L.ct.size() * 8, hipMemcpyHostToDevice));
        const unsigned long long tmp_bytes = c->bytes - bytes_before;
        const size_t np = (size_t)N * L.K * 2;
        c->p64.R = c->dalloc<cpx<double>>(np);
        c->p64.Q = c->dalloc<cpx<double>>(np);
        c->p32.R = c->dalloc<cpx<float>>(np);
        c->p32.Q = c->dalloc<cpx<float>>(np);
        launch_patterns(N, L.K, L.nph, d_ct, k, c->g_rtri, c->g_rcoef, c->g_rloc, c->g_tv, c->g_tn, c->g_ta, d_cen,
                        c->p64.R, c->p64.Q, nullptr);
        HIPCHK(hipGetLastError());
        launch_to_float(c->p64.R, c->p32.R, (long long)np, nullptr);
        launch_to_float(c->p64.Q, c->p32.Q, (long long)np, nullptr);
        HIPCHK(hipGetLastError());
        HIPCHK(hipDeviceSynchronize());
        for (void *p : tmp) (void)hipFree(p);
        c->bytes -= tmp_bytes;
        // receive weights c0 * w_theta * 2 pi / nph, c0 = -k^2 / (16 pi^2)
        std::vector<double> wq(L.K);
        const double c0 = -k * k / (16 * M_PI * M_PI);
        for (int q = 0; q < L.K; q++) wq[q] = c0 * L.wt[q / L.nph] * (2 * M_PI / L.nph);
        c->p64.wq = c->upload(wq);
        c->p32.wq = c->upload(cast_vec<float>(wq));
    }
}

// ------------------------------------------------------------- near field
double tri_quality(const Surface &s, int t)
{
    double l2 = 0;
    for (int a = 0; a < 3; a++) {
        const double *p = &s.v[3 * s.t[3 * t + a]], *q = &s.v[3 * s.t[3 * t + (a + 1) % 3]];
        l2 += (p[0] - q[0]) * (p[0] - q[0]) + (p[1] - q[1]) * (p[1] - q[1]) + (p[2] - q[2]) * (p[2] - q[2]);
    }
    return 4 * std::sqrt(3.0) * s.area[t] / l2;   // 1 for the equilateral triangle
}

// Gauss order per dimension of a touching pair's rule, from the worse shape
// quality of its two triangles and the angle between their normals: the
// relative-coordinate integrands are smooth, and their smoothness degrades
// with elongated triangles and with folds between them.  Near-equilateral,
// nearly coplanar pairs (fine meshes of smooth surfaces) reach about 5e-12
// relative accuracy of the near field already at order 10, elongated or
// folded ones need 14 to 28 for the same.
int rule_order(double q, double cos_normals)
{
    if (q >= 0.95 && cos_normals >= 0.98) return 10;
    if (q >= 0.55) return 14;
    if (q >= 0.35) return 20;
    return 28;
}

void precompute_near(mlfma_ctx *c)
{
    const Surface &s = c->s;
    const Tree &tr = c->tr;
    const RwgTable &r = c->r;
    const int N = r.n, nt = s.nt, leafl = tr.levels - 1;
    const double k = c->opt.wavenumber;
    // ordered touching triangle pairs (CSR by test triangle)
    std::vector<std::vector<int>> vt(s.nv);
    for (int t = 0; t < nt; t++)
        for (int a = 0; a < 3; a++) vt[s.t[3 * t + a]].push_back(t);
    std::vector<int> tp_start(nt + 1, 0), tp_s;
    std::vector<TouchPair> pairs;
    std::vector<double> quality(nt);
    for (int t = 0; t < nt; t++) quality[t] = tri_quality(s, t);
    for (int t = 0; t < nt; t++) {
        std::vector<int> part;
        for (int a = 0; a < 3; a++)
            for (int u : vt[s.t[3 * t + a]]) part.push_back(u);
        std::sort(part.begin(), part.end());
        part.erase(std::unique(part.begin(), part.end()), part.end());
        for (int u : part) {
            TouchPair tp{};
            const int *tv = &s.t[3 * t], *uv = &s.t[3 * u];
            // shared vertices in the test triangle's cyclic order
            int sh_t[3], sh_u[3], ns = 0;
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++)
                    if (tv[a] == uv[b]) { sh_t[ns] = a; sh_u[ns] = b; ns++; }
            tp.rel = ns;
            if (ns == 3) {
                for (int a = 0; a < 3; a++) { tp.pi[a] = a; tp.qi[a] = sh_u[a]; }
            } else if (ns == 2) {
                // shared edge first, both triangles listing it in the same order
                tp.pi[0] = sh_t[0]; tp.pi[1] = sh_t[1]; tp.pi[2] = 3 - sh_t[0] - sh_t[1];
                tp.qi[0] = sh_u[0]; tp.qi[1] = sh_u[1]; tp.qi[2] = 3 - sh_u[0] - sh_u[1];
            } else {
                tp.pi[0] = sh_t[0]; tp.pi[1] = (sh_t[0] + 1) % 3; tp.pi[2] = (sh_t[0] + 2) % 3;
                tp.qi[0] = sh_u[0]; tp.qi[1] = (sh_u[0] + 1) % 3; tp.qi[2] = (sh_u[0] + 2) % 3;
            }
            for (int a = 0; a < 3; a++)
                for (int d = 0; d < 3; d++) {
                    tp.P[3 * a + d] = s.v[3 * tv[tp.pi[a]] + d];
                    tp.Q[3 * a + d] = s.v[3 * uv[tp.qi[a]] + d];
                }
            for (int d = 0; d < 3; d++) tp.nt[d] = s.nrm[3 * t + d];
            tp.At = s.area[t];
            tp.As = s.area[u];
            const double cn = s.nrm[3 * t] * s.nrm[3 * u] + s.nrm[3 * t + 1] * s.nrm[3 * u + 1] +
                              s.nrm[3 * t + 2] * s.nrm[3 * u + 2];
            tp.order = rule_order(std::min(quality[t], quality[u]), cn);
            pairs.push_back(tp);
            tp_s.push_back(u);
        }
        tp_start[t + 1] = (int)tp_s.size();
    }
    // Gauss-Legendre nodes/weights on [0, 1] for the orders used
    std::vector<double> gn;
    std::vector<int> goff(65, 0);
    for (int n : {10, 14, 20, 28}) {
        std::vector<double> x, w;
        gauss_legendre(n, x, w);
        goff[n] = (int)gn.size();
        for (int i = 0; i < n; i++) gn.push_back(0.5 * (x[i] + 1));
        for (int i = 0; i < n; i++) gn.push_back(0.5 * w[i]);
    }
    // slot layout: per leaf box, rows x (concatenated near columns)
    const Level &L = tr.lv[leafl];
    std::vector<long long> val_off(L.nbox + 1, 0);
    for (int b = 0; b < L.nbox; b++) {
        long long nc = 0;
        for (int e = tr.near_start[b]; e < tr.near_start[b + 1]; e++) {
            int nb = tr.near_box[e];
            nc += tr.box_start[nb + 1] - tr.box_start[nb];
        }
        val_off[b + 1] = val_off[b] + (long long)(tr.box_start[b + 1] - tr.box_start[b]) * nc;
    }
    const long long nslot = val_off[L.nbox];
    c->n_slots = nslot;
    c->n_touch = (long long)pairs.size();
    c->val_off = c->upload(val_off);
    c->p64.near_em = c->dalloc<cpx<double>>(2 * (size_t)nslot);
    c->p64.near_c = c->dalloc<cpx<double>>(2 * (size_t)nslot);
    c->p32.near_em = c->dalloc<cpx<float>>(2 * (size_t)nslot);
    c->p32.near_c = c->dalloc<cpx<float>>(2 * (size_t)nslot);
    std::vector<void *> tmp;
    auto up = [&](auto &h) {
        using E = typename std::remove_reference<decltype(h)>::type::value_type;
        E *d = c->dalloc<E>(h.size(), &tmp);
        if (!h.empty()) HIPCHK(hipMemcpy(d, h.data(), h.size() * sizeof(E), hipMemcpyHostToDevice));
        return d;
    };
    unsigned long long bytes_before = c->bytes;
    int *d_tps = up(tp_start), *d_tp_s = up(tp_s), *d_goff = up(goff);
    double *d_gn = up(gn);
    TouchPair *d_pairs = up(pairs);
    cpx<double> *d_touch = c->dalloc<cpx<double>>(36 * std::max<size_t>(pairs.size(), 1), &tmp);
    launch_touch((int)pairs.size(), d_pairs, k, d_gn, d_goff, d_touch, nullptr);
    HIPCHK(hipGetLastError());
    launch_slots(L.nbox, c->box_start, c->near_start, c->near_box, c->val_off, c->g_rtri, c->g_rloc, c->g_rcoef,
                 c->g_tv, c->g_tn, c->g_ta, d_tps, d_tp_s, d_touch, k, c->p64.near_em, c->p64.near_c, c->p32.near_em,
                 c->p32.near_c, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipDeviceSynchronize());
    for (void *p : tmp) (void)hipFree(p);
    c->bytes = bytes_before;
    // identity terms of the C block: Gram and n x Gram on common triangles,
    // 7-point rule (exact for these quadratic integrands)
    std::vector<std::map<int, std::pair<double, double>>> rows(N);
    const double s15 = std::sqrt(15.0), a7 = (6 - s15) / 21, b7 = (6 + s15) / 21;
    const double bary[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {a7, a7, 1 - 2 * a7}, {a7, 1 - 2 * a7, a7},
                               {1 - 2 * a7, a7, a7}, {b7, b7, 1 - 2 * b7}, {b7, 1 - 2 * b7, b7}, {1 - 2 * b7, b7, b7}};
    const double w7[7] = {9.0 / 40, (155 - s15) / 1200, (155 - s15) / 1200, (155 - s15) / 1200,
                          (155 + s15) / 1200, (155 + s15) / 1200, (155 + s15) / 1200};
    for (int t = 0; t < nt; t++) {
        const double *P[3] = {&s.v[3 * s.t[3 * t]], &s.v[3 * s.t[3 * t + 1]], &s.v[3 * s.t[3 * t + 2]]};
        const double *n = &s.nrm[3 * t];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                int um = r.tri_rwg[3 * (size_t)t + i], un = r.tri_rwg[3 * (size_t)t + j];
                double cm = r.tri[0][um] == t ? r.coef[0][um] : r.coef[1][um];
                double cn = r.tri[0][un] == t ? r.coef[0][un] : r.coef[1][un];
                double g = 0, gx = 0;
                for (int p = 0; p < 7; p++) {
                    double x[3], a[3], b[3], nb[3];
                    for (int d = 0; d < 3; d++) {
                        x[d] = bary[p][0] * P[0][d] + bary[p][1] * P[1][d] + bary[p][2] * P[2][d];
                        a[d] = x[d] - P[i][d];
                        b[d] = x[d] - P[j][d];
                    }
                    nb[0] = n[1] * b[2] - n[2] * b[1];
                    nb[1] = n[2] * b[0] - n[0] * b[2];
                    nb[2] = n[0] * b[1] - n[1] * b[0];
                    g += w7[p] * (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
                    gx += w7[p] * (a[0] * nb[0] + a[1] * nb[1] + a[2] * nb[2]);
                }
                auto &e = rows[tr.iperm[um]][tr.iperm[un]];
                e.first += cm * cn * s.area[t] * g;
                e.second += cm * cn * s.area[t] * gx;
            }
    }
    std::vector<int> id_start(N + 1, 0), id_col;
    std::vector<double> id_w;
    for (int m = 0; m < N; m++) {
        for (auto &kv : rows[m]) {
            id_col.push_back(kv.first);
            id_w.push_back(kv.second.first);
            id_w.push_back(kv.second.second);
        }
        id_start[m + 1] = (int)id_col.size();
    }
    c->n_id = (long long)id_col.size();
    c->id_start = c->upload(id_start);
    c->id_col = c->upload(id_col);
    c->p64.id_w = c->upload(id_w);
    c->p32.id_w = c->upload(cast_vec<float>(id_w));
    c->near_ready = true;
}

// ---------------------------------------------------------------- SAI
// Sparse approximate inverse of op's near field with patterns of k_nearest
// RWGs (sai.hpp).  Host: the patterns (the k nearest RWG centres inside the
// adjacent leaf boxes, ties at the k-th distance included), the leaf boxes
// whose rows touch each pattern, and the row-wise entry lists of the apply
// (user order).  Device: the least-squares columns in double precision,
// copied to single precision.
void build_sai(mlfma_ctx *c, int op, int k_nearest)
{
    const auto t0 = std::chrono::steady_clock::now();
    c->free_sai(op);     // a failed build leaves the op without an SAI
    const Tree &tr = c->tr;
    const RwgTable &r = c->r;
    const Surface &s = c->s;
    const int N = r.n;
    if ((long long)N * 2 * SAI_D >= (1LL << 31))
        throw Error(MLFMA_ERR_UNSUPPORTED, "too many RWGs for the SAI entry offsets");
    std::vector<double> ctr(3 * (size_t)N);
    for (int u = 0; u < N; u++) {
        const int n = tr.perm[u];
        for (int d = 0; d < 3; d++) ctr[3 * (size_t)u + d] = 0.5 * (s.v[3 * (size_t)r.a[n] + d] + s.v[3 * (size_t)r.b[n] + d]);
    }
    std::vector<int> pat_start(N + 1, 0), pat, rb_start(N + 1, 0), rb;
    std::vector<std::pair<double, int>> cand;
    std::vector<int> boxes;
    int maxp = 0;
    for (int u = 0; u < N; u++) {
        const int b = tr.leaf_of[u];
        cand.clear();
        for (int e = tr.near_start[b]; e < tr.near_start[b + 1]; e++) {
            const int nb = tr.near_box[e];
            for (int w = tr.box_start[nb]; w < tr.box_start[nb + 1]; w++) {
                const double dx = ctr[3 * (size_t)w] - ctr[3 * (size_t)u];
                const double dy = ctr[3 * (size_t)w + 1] - ctr[3 * (size_t)u + 1];
                const double dz = ctr[3 * (size_t)w + 2] - ctr[3 * (size_t)u + 2];
                cand.push_back({dx * dx + dy * dy + dz * dz, w});
            }
        }
        size_t take = cand.size();
        if ((int)cand.size() > k_nearest) {
            std::nth_element(cand.begin(), cand.begin() + (k_nearest - 1), cand.end());
            const double thr = cand[k_nearest - 1].first * (1 + 1e-9);
            take = std::partition(cand.begin(), cand.end(), [&](const std::pair<double, int> &q) {
                       return q.first <= thr;
                   }) - cand.begin();
        }
        if ((int)take > SAI_MAXP)
            throw Error(MLFMA_ERR_UNSUPPORTED, "SAI pattern of RWG " + std::to_string(tr.perm[u]) + " has " +
                                                   std::to_string(take) + " members (ties); at most " +
                                                   std::to_string(SAI_MAXP));
        std::vector<int> sel;
        for (size_t i = 0; i < take; i++) sel.push_back(cand[i].second);
        std::sort(sel.begin(), sel.end());
        maxp = std::max(maxp, (int)sel.size());
        boxes.clear();
        for (int w : sel) {
            const int pb = tr.leaf_of[w];
            for (int e = tr.near_start[pb]; e < tr.near_start[pb + 1]; e++) boxes.push_back(tr.near_box[e]);
        }
        std::sort(boxes.begin(), boxes.end());
        boxes.erase(std::unique(boxes.begin(), boxes.end()), boxes.end());
        pat.insert(pat.end(), sel.begin(), sel.end());
        rb.insert(rb.end(), boxes.begin(), boxes.end());
        pat_start[u + 1] = (int)pat.size();
        rb_start[u + 1] = (int)rb.size();
    }
    // apply lists: row (user) p of M gathers the columns (u, .) whose pattern holds p
    const long long nnz = (long long)pat.size();
    std::vector<int> row_start(N + 1, 0), ent_col(nnz), ent_val(nnz);
    for (int u = 0; u < N; u++)
        for (int e = pat_start[u]; e < pat_start[u + 1]; e++) row_start[tr.perm[pat[e]] + 1]++;
    for (int p = 0; p < N; p++) row_start[p + 1] += row_start[p];
    {
        std::vector<int> fill(row_start.begin(), row_start.end() - 1);
        for (int u = 0; u < N; u++)
            for (int e = pat_start[u]; e < pat_start[u + 1]; e++) {
                const int q = fill[tr.perm[pat[e]]]++;
                ent_col[q] = tr.perm[u];
                ent_val[q] = u * 2 * SAI_D + 2 * (e - pat_start[u]);
            }
    }
    SaiData &d = c->sai[op];
    const unsigned long long before = c->bytes;
    std::vector<void *> tmp;
    struct Free {
        std::vector<void *> &l;
        ~Free()
        {
            for (void *p : l) (void)hipFree(p);
        }
    } fr{tmp};
    auto up = [&](const std::vector<int> &h, std::vector<void *> *list) {
        int *p = c->dalloc<int>(h.size(), list);
        if (!h.empty()) HIPCHK(hipMemcpy(p, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice));
        return p;
    };
    try {
        d.M64 = c->dalloc<cpx<double>>((size_t)N * 2 * SAI_D, &d.allocs);
        d.M32 = c->dalloc<cpx<float>>((size_t)N * 2 * SAI_D, &d.allocs);
        d.row_start = up(row_start, &d.allocs);
        d.ent_col = up(ent_col, &d.allocs);
        d.ent_val = up(ent_val, &d.allocs);
        d.bytes = c->bytes - before;
        const unsigned long long kept = c->bytes;
        int *d_ps = up(pat_start, &tmp), *d_pat = up(pat, &tmp), *d_rs = up(rb_start, &tmp), *d_rb = up(rb, &tmp);
        int *d_status = up(std::vector<int>(1, 0), &tmp);
        const bool isc = op == MLFMA_OP_C;
        const int chunk = 32768;
        for (int u0 = 0; u0 < N; u0 += chunk)
            launch_sai_build(u0, std::min(chunk, N - u0), d_ps, d_pat, d_rs, d_rb, c->leaf_of, c->box_start,
                             c->near_start, c->near_box, c->val_off, isc ? c->p64.near_c : c->p64.near_em,
                             isc ? c->id_start : nullptr, c->id_col, c->p64.id_w, d.M64, d_status, nullptr);
        HIPCHK(hipGetLastError());
        launch_to_float(d.M64, d.M32, (long long)N * 2 * SAI_D, nullptr);
        HIPCHK(hipGetLastError());
        int status = 0;
        HIPCHK(hipMemcpy(&status, d_status, sizeof(int), hipMemcpyDeviceToHost));
        c->bytes = kept;
        if (status)
            throw Error(MLFMA_ERR_UNSUPPORTED, "SAI normal equations not positive definite for some RWG");
    } catch (...) {
        c->bytes = before + d.bytes;
        c->free_sai(op);
        throw;
    }
    d.k = k_nearest;
    d.maxp = maxp;
    d.nnz = nnz;
    d.ready = true;
    d.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// ---------------------------------------------------------------- workspace
// Layout of the per-product scratch for nrhs right-hand sides in elements of
// esz bytes (16: complex double, also used by the complex float path; 8:
// complex float only), every buffer starting on a 256-byte boundary: the
// internal vectors X and Y, the box patterns U and V of every level and the
// level-step intermediate.  Returns the bytes; with w and base set, points
// w's buffers into base.
unsigned long long layout_workspace(const mlfma_ctx *c, int nrhs, size_t esz, char *base, Workspace *w)
{
    const Tree &tr = c->tr;
    unsigned long long off = 0;
    auto take = [&](unsigned long long elems) -> void * {
        void *p = base ? base + off : nullptr;
        off += (std::max<unsigned long long>(elems, 1) * esz + 255) & ~255ULL;
        return p;
    };
    const unsigned long long N = (unsigned long long)c->r.n;
    void *X = take(N * 2 * nrhs), *Y = take(N * 2 * nrhs);
    if (w) {
        w->X = X;
        w->Y = Y;
        w->U.assign(tr.levels, nullptr);
        w->V.assign(tr.levels, nullptr);
    }
    unsigned long long midmax = 1;
    for (int l = 2; l < tr.levels; l++) {
        const Level &L = tr.lv[l];
        void *U = take((unsigned long long)L.nbox * L.K * 2 * nrhs);
        void *V = take((unsigned long long)L.nbox * L.K * 2 * nrhs);
        if (w) {
            w->U[l] = U;
            w->V[l] = V;
        }
        if (l + 1 < tr.levels) {
            const Level &C = tr.lv[l + 1];
            midmax = std::max<unsigned long long>(midmax, (unsigned long long)C.nbox * L.nth * C.nph * 2 * nrhs);
        }
    }
    void *mid = take(midmax);
    void *X2 = nullptr, *Y2 = nullptr;
    if (c->mixed) {   // complex float copies of X and Y
        const unsigned long long f = (N * 2 * nrhs * sizeof(cpx<float>) + esz - 1) / esz;
        X2 = take(f);
        Y2 = take(f);
    }
    if (w) {
        w->mid = mid;
        w->X2 = X2;
        w->Y2 = Y2;
        w->rhs = nrhs;
    }
    return off;
}

// Bytes of a workspace for nrhs right-hand sides (complex double units).
unsigned long long workspace_bytes(const mlfma_ctx *c, int nrhs)
{
    return layout_workspace(c, nrhs, sizeof(cpx<double>), nullptr, nullptr);
}

// Allocate w for nrhs right-hand sides (no budget check: the caller admits).
void alloc_workspace(const mlfma_ctx *c, Workspace &w, int nrhs)
{
    w.release();
    const unsigned long long need = workspace_bytes(c, nrhs);
    void *p = nullptr;
    HIPCHK(hipMalloc(&p, need));
    w.allocs.push_back(p);
    w.bytes = need;
    layout_workspace(c, nrhs, sizeof(cpx<double>), (char *)p, &w);
}

// Lay a workspace for nrhs right-hand sides over an existing arena of at
// least workspace_bytes(c, nrhs) bytes (no allocation).
void carve_workspace(const mlfma_ctx *c, Workspace &w, char *base, int nrhs)
{
    layout_workspace(c, nrhs, sizeof(cpx<double>), base, &w);
}

void ensure_workspace(mlfma_ctx *c, int nrhs)
{
    if (nrhs <= c->ws.rhs) return;
    c->free_ws();
    const unsigned long long need = workspace_bytes(c, nrhs);
    if (c->opt.hbm_budget_bytes && c->bytes + need > c->opt.hbm_budget_bytes)
        throw Error(MLFMA_ERR_OOM, "device memory budget exceeded by the workspace");
    try {
        alloc_workspace(c, c->ws, nrhs);
    } catch (...) {
        c->ws.release();      // the buffers allocated before the failure; c->bytes never counted them
        throw;
    }
    c->bytes += c->ws.bytes;
    if (!c->side) {
        HIPCHK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->join, hipEventDisableTiming));
    }
    c->ws.side = c->side;
    c->ws.fork = c->fork;
    c->ws.join = c->join;
}

// arguments of the fused step between parent level l and child level l + 1
template <class T>
LevelStep<T> step_args(mlfma_ctx *c, Prec<T> &P, int l, bool agg, int nrhs)
{
    const Tree &tr = c->tr;
    const Level &L = tr.lv[l], &C = tr.lv[l + 1];
    const IntLevel &I = c->lv[l];
    const PrecLevel<T> &PL = P.lv[l];
    const bool small = nrhs < 4;
    const StepPlan &pl = agg ? (small ? PL.agg1 : PL.agg) : (small ? PL.dis1 : PL.dis);
    LevelStep<T> a;
    a.nbox = agg ? L.nbox : C.nbox;
    a.nth_p = L.nth;
    a.nph_p = L.nph;
    a.nth_c = C.nth;
    a.nph_c = C.nph;
    a.rows = pl.rows;
    a.nchunk = pl.nchunk;
    a.wrows = pl.wrows;
    a.win = pl.win;
    a.rb = small ? 0 : (agg ? PL.agg_rb : PL.dis_rb);
    a.group = small || !agg ? 0 : PL.agg_group;
    a.pipe = small ? 0 : (agg ? PL.agg_pipe : PL.dis_pipe);
    a.taps = c->opt.interp_order;
    a.child_start = I.child_start;
    a.parent = c->lv[l + 1].parent;
    a.oct = c->lv[l + 1].oct;
    a.shift = PL.shift;
    if (agg) {
        a.c1 = I.ath_c;
        a.w1 = PL.ath_w;
        a.c2 = I.aph_c;
        a.w2 = PL.aph_w;
        // the separable form, for the pipelined kernel
        a.tphi = PL.ag_tphi;
        a.tth = PL.ag_tth;
        a.phi_col = PL.ag_phi_col;
        a.th_row = PL.ag_th_row;
        a.th_sh = PL.ag_th_sh;
        a.phi_w = PL.ag_phi_w;
        a.th_w = PL.ag_th_w;
    } else {
        a.tphi = PL.tphi;
        a.tth = PL.tth;
        a.phi_col = PL.phi_col;
        a.th_row = PL.th_row;
        a.th_sh = PL.th_sh;
        a.phi_w = PL.phi_w;
        a.rowf = PL.rowf;
        a.th_w = PL.th_w;
    }
    return a;
}

// Kernel shape of every vector level step (aggregation and disaggregation,
// each level on its own): 1, 2 or 4 right-hand sides per workgroup (for the
// aggregation also 2 or 4 children staged together, one right-hand side
// each), the two kernels through the global intermediate, or the pipelined
// kernel with 1 or 2 per pass,
// whichever runs the step fastest with the handle's right-hand-side count
// (capped at 16; one warm-up and three timed runs each, on zeroed patterns).
// Handles for fewer than four right-hand sides keep the launchers' default;
// the options can fix the choice (blocked kernels only, or pipelined ones
// wherever they fit).
template <class T>
void tune_step_rb(mlfma_ctx *c, Prec<T> &P)
{
    const Tree &tr = c->tr;
    if (c->opt.level_kernel == MLFMA_LEVELS_PIPELINED) {
        for (int l = 2; l + 1 < tr.levels; l++) {   // the widest passes; the launchers narrow them where needed
            P.lv[l].agg_pipe = 2;
            P.lv[l].dis_pipe = 4;
        }
        return;
    }
    const bool blocked = c->opt.level_kernel == MLFMA_LEVELS_BLOCKED;
    const int nrhs = std::min(c->opt.max_rhs, 16);
    if (nrhs < 4) return;
    hipStream_t st;
    HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    Workspace &w = c->ws;
    for (int l = 2; l < tr.levels; l++) {
        launch_zero<T>((cpx<T> *)w.U[l], (long long)tr.lv[l].nbox * tr.lv[l].K * 2 * nrhs, st);
        launch_zero<T>((cpx<T> *)w.V[l], (long long)tr.lv[l].nbox * tr.lv[l].K * 2 * nrhs, st);
    }
    for (int l = 2; l + 1 < tr.levels; l++) {
        for (int agg = 0; agg < 2; agg++) {
            int &rb = agg ? P.lv[l].agg_rb : P.lv[l].dis_rb;
            int &pipe = agg ? P.lv[l].agg_pipe : P.lv[l].dis_pipe;
            int dummy = 0;
            int &group = agg ? P.lv[l].agg_group : dummy;
            int &two = agg ? P.lv[l].agg_two : P.lv[l].dis_two;
            // (right-hand sides per workgroup, pipelined per pass, children per
            // group, two kernels through the global intermediate)
            const int cands[9][4] = {{1, 0, 0, 0}, {2, 0, 0, 0}, {4, 0, 0, 0}, {0, 1, 0, 0}, {0, 2, 0, 0},
                                     {0, 4, 0, 0}, {1, 0, 2, 0}, {1, 0, 4, 0}, {0, 0, 0, 1}};
            double best = 1e30;
            int pick[4] = {0, 0, 0, 0};
            for (const auto &cd : cands) {
                if ((cd[1] > 0 || cd[3] > 0) && blocked) continue;
                if (cd[2] > 0 && !agg) continue;
                rb = cd[0];
                pipe = cd[1];
                group = cd[2];
                two = cd[3];
                LevelStep<T> a = step_args<T>(c, P, l, agg != 0, nrhs);
                a.in = (const cpx<T> *)(agg ? w.U[l + 1] : w.V[l]);
                a.out = (cpx<T> *)(agg ? w.U[l] : w.V[l + 1]);
                auto run = [&] {
                    if (two) {
                        if (agg) agg_two<T>(c, P, w, l, nrhs, st);
                        else dis_two<T>(c, P, w, l, nrhs, st);
                        return true;
                    }
                    return agg ? launch_aggregate_step<T>(a, nrhs, st) : launch_disaggregate_step<T>(a, nrhs, st);
                };
                if (!run()) break;   // the step has no fused kernel: nothing to tune
                HIPCHK(hipEventRecord(e0, st));
                for (int i = 0; i < 3; i++) run();
                HIPCHK(hipEventRecord(e1, st));
                HIPCHK(hipEventSynchronize(e1));
                float t = 0;
                HIPCHK(hipEventElapsedTime(&t, e0, e1));
                if (t < best) {
                    best = t;
                    pick[0] = rb;
                    pick[1] = pipe;
                    pick[2] = group;
                    pick[3] = two;
                }
            }
            rb = pick[0];
            pipe = pick[1];
            group = pick[2];
            two = pick[3];
        }
    }
    HIPCHK(hipGetLastError());
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
}

// Level steps of complex64 products: the vector kernels (levels.hip) or the
// matrix-core ones (levels_mfma.hip), whichever runs the aggregation and
// disaggregation of all levels faster with the handle's right-hand-side
// count (capped at 16; one warm-up and three timed runs each), unless the
// options fix the choice.
void tune_level_steps(mlfma_ctx *c)
{
    Prec<float> &P = c->p32;
    const Tree &tr = c->tr;
    P.level_mfma = 0;
    bool any = false;
    for (int l = 2; l + 1 < tr.levels; l++) any |= P.lv[l].agg_m.ok && P.lv[l].dis_m.ok;
    if (!any || (c->opt.level_kernel != MLFMA_LEVELS_AUTO && c->opt.level_kernel != MLFMA_LEVELS_MATRIX)) return;
    if (c->opt.level_kernel == MLFMA_LEVELS_MATRIX) {
        P.level_mfma = 1;
        return;
    }
    const int nrhs = std::min(c->opt.max_rhs, 16);
    hipStream_t st;
    HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    Workspace &w = c->ws;
    // zeroed patterns: the timing must not depend on what the workspace held
    for (int l = 2; l < tr.levels; l++) {
        launch_zero<float>((cpx<float> *)w.U[l], (long long)tr.lv[l].nbox * tr.lv[l].K * 2 * nrhs, st);
        launch_zero<float>((cpx<float> *)w.V[l], (long long)tr.lv[l].nbox * tr.lv[l].K * 2 * nrhs, st);
    }
    auto steps = [&](int mfma) {
        P.level_mfma = mfma;
        for (int l = tr.levels - 2; l >= 2; l--) {
            if (mfma && launch_aggregate_mfma(P.lv[l].agg_m, (const cpx<float> *)w.U[l + 1], (cpx<float> *)w.U[l], nrhs,
                                              st))
                continue;
            LevelStep<float> a = step_args<float>(c, P, l, true, nrhs);
            a.in = (const cpx<float> *)w.U[l + 1];
            a.out = (cpx<float> *)w.U[l];
            launch_aggregate_step<float>(a, nrhs, st);
        }
        for (int l = 3; l < tr.levels; l++) {
            if (mfma && launch_disaggregate_mfma(P.lv[l - 1].dis_m, (const cpx<float> *)w.V[l - 1], (cpx<float> *)w.V[l],
                                                 nrhs, st))
                continue;
            LevelStep<float> a = step_args<float>(c, P, l - 1, false, nrhs);
            a.in = (const cpx<float> *)w.V[l - 1];
            a.out = (cpx<float> *)w.V[l];
            launch_disaggregate_step<float>(a, nrhs, st);
        }
    };
    double ms[2] = {0, 0};
    for (int mfma = 0; mfma < 2; mfma++) {
        steps(mfma);
        HIPCHK(hipEventRecord(e0, st));
        for (int i = 0; i < 3; i++) steps(mfma);
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        float t = 0;
        HIPCHK(hipEventElapsedTime(&t, e0, e1));
        ms[mfma] = t / 3;
    }
    HIPCHK(hipGetLastError());
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    P.step_ms[0] = ms[0];
    P.step_ms[1] = ms[1];
    P.level_mfma = ms[1] < ms[0] ? 1 : 0;
}

// One product, in three phases so that a batch of geometries can share the
// translation launch: begin (permutation, near field, radiation,
// aggregation), translate, end (disaggregation, receive, permutation).
template <class T>
struct MvRun {
    mlfma_ctx *c = nullptr;
    Workspace *w = nullptr;
    Prec<T> *P = nullptr;
    int op = 0, part = 0, nrhs = 0;
    hipStream_t st = nullptr;
    bool profile = false;
    int N = 0, leafl = 0, only_level = -1;
    bool want_near = false, far = false, overlap = false, fold = false;
    cpx<T> *X = nullptr, *Y = nullptr, *mid = nullptr;
    std::vector<hipEvent_t> ev;
    void mark(int i)
    {
        if (profile) HIPCHK(hipEventRecord(ev[i], st));
    }
    void near(hipStream_t sn)
    {
        const cpx<T> *vals = op == MLFMA_OP_EM ? P->near_em : P->near_c;
        const int *ids = op == MLFMA_OP_C ? c->id_start : nullptr;
        bool done = false;
        if (P->mfma_ends)
            done = launch_near_mfma<T>(c->n_items, c->items, c->box_start, c->col_off, c->cols, c->val_off, vals, ids,
                                    c->id_col, P->id_w, X, Y, nrhs, sn);
        if (!done && nrhs == 1) {
            launch_near_tile<T>(c->n_items, c->items, c->box_start, c->col_off, c->cols, c->val_off, vals, ids,
                                c->id_col, P->id_w, X, Y, sn);
            done = true;
        }
        if (!done)
            launch_near<T>(N, c->leaf_of, c->box_start, c->near_start, c->near_box, c->val_off, vals, ids, c->id_col,
                           P->id_w, X, Y, nrhs, sn);
    }
};

template <class T>
MvRun<T> mv_setup(mlfma_ctx *c, Workspace &w, Prec<T> &P, int op, int part, int nrhs, hipStream_t st, bool profile)
{
    MvRun<T> m;
    const Tree &tr = c->tr;
    m.c = c;
    m.w = &w;
    m.P = &P;
    m.op = op;
    m.part = part;
    m.nrhs = nrhs;
    m.st = st;
    m.profile = profile;
    m.N = c->r.n;
    m.leafl = tr.levels - 1;
    m.X = (cpx<T> *)w.X;
    m.Y = (cpx<T> *)w.Y;
    m.mid = (cpx<T> *)w.mid;
    if (profile) m.ev = c->take_events();
    m.only_level = part >= MLFMA_PART_LEVEL ? part - MLFMA_PART_LEVEL : -1;
    m.want_near = m.only_level < 0 && (part & MLFMA_PART_NEAR);
    const bool want_far = m.only_level >= 0 || (part & MLFMA_PART_FAR);
    m.far = tr.levels >= 3 && want_far;
    // the near field beside the far-field chain (stage timing keeps them in
    // sequence): forked after the radiation, whose memory traffic it would
    // otherwise compete with, so that it shares the GPU with the
    // latency-bound level steps and translation
    m.overlap = !profile && m.want_near && m.far && w.side;
    // with one right-hand side and the near field after the radiation, the
    // radiation reads x through the permutation (and stores the tree-order
    // copy the near field reads) and the receive writes y in user order: two
    // launches fewer on the critical path
    m.fold = m.overlap && nrhs == 1;
    return m;
}

// A level step as two kernels through the global intermediate (no LDS
// windows): aggregation from level l + 1 to l (theta, then phi and shift);
// disaggregation from level l to l + 1 (shift and phi, then theta).
template <class T>
void agg_two(mlfma_ctx *c, Prec<T> &P, Workspace &w, int l, int nrhs, hipStream_t st)
{
    const Tree &tr = c->tr;
    const Level &L = tr.lv[l], &C = tr.lv[l + 1];
    const IntLevel &I = c->lv[l];
    const int midlen = L.nth * C.nph, taps = c->opt.interp_order;
    cpx<T> *mid = (cpx<T> *)w.mid;
    if (!launch_interp_fixed<T>(taps, C.nbox, midlen, C.K, I.ath_c, P.lv[l].ath_w, (cpx<T> *)w.U[l + 1], mid, nrhs,
                                st))
        launch_interp<T>(C.nbox, midlen, C.K, I.ath_s, I.ath_c, P.lv[l].ath_w, (cpx<T> *)w.U[l + 1], mid, nrhs, false,
                         st);
    if (!launch_agg_phi_fixed<T>(taps, L.nbox, L.K, midlen, I.child_start, c->lv[l + 1].oct, P.lv[l].shift, I.aph_c,
                                 P.lv[l].aph_w, mid, (cpx<T> *)w.U[l], nrhs, st))
        launch_agg_phi<T>(L.nbox, L.K, midlen, I.child_start, c->lv[l + 1].oct, P.lv[l].shift, I.aph_s, I.aph_c,
                          P.lv[l].aph_w, mid, (cpx<T> *)w.U[l], nrhs, st);
}

template <class T>
void dis_two(mlfma_ctx *c, Prec<T> &P, Workspace &w, int l, int nrhs, hipStream_t st)
{
    const Tree &tr = c->tr;
    const Level &Pl = tr.lv[l], &L = tr.lv[l + 1];
    const IntLevel &Ip = c->lv[l];
    const int midlen = Pl.nth * L.nph;
    cpx<T> *mid = (cpx<T> *)w.mid;
    launch_disagg_mid<T>(L.nbox, midlen, Pl.K, c->lv[l + 1].parent, c->lv[l + 1].oct, P.lv[l].shift, Ip.dph_s,
                         Ip.dph_c, P.lv[l].dph_w, (cpx<T> *)w.V[l], mid, nrhs, st);
    launch_interp<T>(L.nbox, L.K, midlen, Ip.dth_s, Ip.dth_c, P.lv[l].dth_w, mid, (cpx<T> *)w.V[l + 1], nrhs, true,
                     st);
}

template <class T>
void mv_begin(MvRun<T> &m, const cpx<T> *x, long long ldx)
{
    mlfma_ctx *c = m.c;
    Workspace &w = *m.w;
    Prec<T> &P = *m.P;
    const Tree &tr = c->tr;
    const int nrhs = m.nrhs, leafl = m.leafl;
    hipStream_t st = m.st;
    const Level &Lf = tr.lv[leafl];
    m.mark(0);
    if (!m.fold) launch_perm_in<T>(x, ldx, m.X, c->perm, c->iperm, m.N, nrhs, st);
    m.mark(1);
    if (!m.want_near) launch_zero<T>(m.Y, (long long)m.N * 2 * nrhs, st);
    else if (!m.overlap) m.near(st);
    m.mark(2);
    if (m.fold) {
        launch_radiate1_user<T>(m.op, Lf.nbox, Lf.K, c->box_start, P.R, x, c->perm, m.N, m.X, (cpx<T> *)w.U[leafl], st);
    } else if (m.far) {
        bool done = false;
        if (P.mfma_ends)
            done = launch_radiate_mfma<T>(m.op, Lf.nbox, Lf.K, c->box_start, P.R, m.X, (cpx<T> *)w.U[leafl], nrhs, st);
        if (!done) launch_radiate<T>(m.op, Lf.nbox, Lf.K, c->box_start, P.R, m.X, (cpx<T> *)w.U[leafl], nrhs, st);
    }
    if (m.overlap) {
        HIPCHK(hipEventRecord(w.fork, st));
        HIPCHK(hipStreamWaitEvent(w.side, w.fork, 0));
        m.near(w.side);
        HIPCHK(hipEventRecord(w.join, w.side));
    }
    m.mark(3);
    if (m.far) {
        for (int l = leafl - 1; l >= 2; l--) {
            if constexpr (std::is_same<T, float>::value)
                if (P.level_mfma && P.lv[l].agg_m.ok &&
                    launch_aggregate_mfma(P.lv[l].agg_m, (const cpx<float> *)w.U[l + 1], (cpx<float> *)w.U[l], nrhs, st))
                    continue;
            LevelStep<T> a = step_args<T>(c, P, l, true, nrhs);
            a.in = (const cpx<T> *)w.U[l + 1];
            a.out = (cpx<T> *)w.U[l];
            if (!(nrhs >= 4 && P.lv[l].agg_two) && launch_aggregate_step<T>(a, nrhs, st)) continue;
            agg_two<T>(c, P, w, l, nrhs, st);
        }
    }
    m.mark(4);
}

// levels whose translation is not asked for (a single level's part) start at zero
template <class T>
void mv_clear_levels(MvRun<T> &m)
{
    const Tree &tr = m.c->tr;
    for (int l = 2; l <= m.leafl; l++)
        if (m.only_level >= 0 && l != m.only_level)
            launch_zero<T>((cpx<T> *)m.w->V[l], (long long)tr.lv[l].nbox * tr.lv[l].K * 2 * m.nrhs, m.st);
}

template <class T>
void mv_translate(MvRun<T> &m)
{
    if (m.far) {
        mv_clear_levels(m);
        launch_translation<T>(m.c, *m.P, *m.w, m.only_level, m.nrhs, m.st);
    }
    m.mark(5);
}

template <class T>
void mv_end(MvRun<T> &m, cpx<T> *y, long long ldy)
{
    mlfma_ctx *c = m.c;
    Workspace &w = *m.w;
    Prec<T> &P = *m.P;
    const Tree &tr = c->tr;
    const int nrhs = m.nrhs, leafl = m.leafl;
    hipStream_t st = m.st;
    const Level &Lf = tr.lv[leafl];
    if (m.far) {
        for (int l = 3; l <= leafl; l++) {
            if constexpr (std::is_same<T, float>::value)
                if (P.level_mfma && P.lv[l - 1].dis_m.ok &&
                    launch_disaggregate_mfma(P.lv[l - 1].dis_m, (const cpx<float> *)w.V[l - 1], (cpx<float> *)w.V[l],
                                             nrhs, st))
                    continue;
            LevelStep<T> a = step_args<T>(c, P, l - 1, false, nrhs);
            a.in = (const cpx<T> *)w.V[l - 1];
            a.out = (cpx<T> *)w.V[l];
            if (!(nrhs >= 4 && P.lv[l - 1].dis_two) && launch_disaggregate_step<T>(a, nrhs, st)) continue;
            dis_two<T>(c, P, w, l - 1, nrhs, st);
        }
    }
    m.mark(6);
    if (m.overlap) HIPCHK(hipStreamWaitEvent(st, w.join, 0));
    if (m.fold) {
        launch_receive1_user<T>(m.op, m.N, Lf.K, c->leaf_of, P.R, P.Q, P.wq, (cpx<T> *)w.V[leafl], m.Y, y, c->perm, st);
    } else if (m.far) {
        bool done = false;
        if (P.mfma_ends)
            done = launch_receive_mfma<T>(m.op, c->n_items, c->items, Lf.K, c->box_start, P.R, P.Q, P.wq,
                                       (cpx<T> *)w.V[leafl], m.Y, nrhs, st);
        if (!done)
            launch_receive<T>(m.op, m.N, Lf.K, c->leaf_of, P.R, P.Q, P.wq, (cpx<T> *)w.V[leafl], m.Y, nrhs, st);
    }
    m.mark(7);
    if (!m.fold) launch_perm_out<T>(m.Y, y, ldy, c->iperm, m.N, nrhs, st);
    m.mark(8);
    if (m.profile) c->ev_pending.push_back(m.ev);
}

template <class T>
void run_matvec(mlfma_ctx *c, Workspace &w, Prec<T> &P, int op, int part, int nrhs, const cpx<T> *x, long long ldx,
                cpx<T> *y, long long ldy, hipStream_t st, bool profile)
{
    MvRun<T> m = mv_setup<T>(c, w, P, op, part, nrhs, st, profile);
    mv_begin<T>(m, x, ldx);
    mv_translate<T>(m);
    mv_end<T>(m, y, ldy);
}

// One product in precision T of the vectors.  complex128 products whose
// near or far part is asked for in FP32 (the handle's options) run that part
// as a complex64 product of the same x rounded to single precision (part
// selection of run_matvec), added to the FP64 part; stage timing covers
// the FP64 part (the FP32 one when there is no FP64 part).
template <class T>
void product(mlfma_ctx *c, Workspace &w, int op, int part, int nrhs, const cpx<T> *x, long long ldx, cpx<T> *y,
             long long ldy, hipStream_t st, bool profile);
template <>
void product<float>(mlfma_ctx *c, Workspace &w, int op, int part, int nrhs, const cpx<float> *x, long long ldx,
                    cpx<float> *y, long long ldy, hipStream_t st, bool profile)
{
    run_matvec<float>(c, w, c->p32, op, part, nrhs, x, ldx, y, ldy, st, profile);
}
template <>
void product<double>(mlfma_ctx *c, Workspace &w, int op, int part, int nrhs, const cpx<double> *x, long long ldx,
                     cpx<double> *y, long long ldy, hipStream_t st, bool profile)
{
    if (!c->mixed) {
        run_matvec<double>(c, w, c->p64, op, part, nrhs, x, ldx, y, ldy, st, profile);
        return;
    }
    const bool near32 = c->opt.near_precision == MLFMA_PREC_FP32, far32 = c->opt.far_precision == MLFMA_PREC_FP32;
    const bool level = part >= MLFMA_PART_LEVEL;
    const bool want_near = !level && (part & MLFMA_PART_NEAR), want_far = level || (part & MLFMA_PART_FAR);
    int p64 = 0, p32 = 0;
    if (want_near) (near32 ? p32 : p64) |= MLFMA_PART_NEAR;
    if (want_far && !level) (far32 ? p32 : p64) |= MLFMA_PART_FAR;
    if (level) (far32 ? p32 : p64) = part;
    const long long n = 2LL * c->r.n;
    cpx<float> *xf = (cpx<float> *)w.X2, *yf = (cpx<float> *)w.Y2;
    if (p64) run_matvec<double>(c, w, c->p64, op, p64, nrhs, x, ldx, y, ldy, st, profile);
    if (p32) {
        launch_to_single(x, ldx, xf, n, n, nrhs, st);
        run_matvec<float>(c, w, c->p32, op, p32, nrhs, xf, n, yf, n, st, profile && !p64);
        launch_from_single(y, ldy, yf, n, n, nrhs, p64 != 0, st);
    }
}

template <class T>
const cpx<T> *sai_values(const SaiData &d);
template <>
const cpx<double> *sai_values<double>(const SaiData &d) { return d.M64; }
template <>
const cpx<float> *sai_values<float>(const SaiData &d) { return d.M32; }

// The HDG side of the hybrid solver's product (Sec. II-E, eq. 52, steps
// 2(b)-(e)): the sparse couplings D^{Lambda X} (n_hdg x 2N) and D^{X Lambda}
// (2N x n_hdg) in CSR form on the device, in both precisions, and the
// caller's solve with Q (the sparse-direct factorisation of the HDG block)
// over the caller's two n_hdg x max_rhs buffers.
struct HybridSide {
    long long n_hdg = 0, nnz_lx = 0, nnz_xl = 0;
    long long *lx_ptr = nullptr, *xl_ptr = nullptr;
    int *lx_col = nullptr, *xl_col = nullptr;
    cpx<double> *lx64 = nullptr, *xl64 = nullptr;
    cpx<float> *lx32 = nullptr, *xl32 = nullptr;
    mlfma_qsolve_fn solve = nullptr;
    void *user = nullptr;
    void *buf1 = nullptr, *buf2 = nullptr;
    long long ldbuf = 0, max_rhs = 0;
};

template <class T>
const cpx<T> *hy_vals(const HybridSide &h, bool lx);
template <>
const cpx<double> *hy_vals<double>(const HybridSide &h, bool lx) { return lx ? h.lx64 : h.xl64; }
template <>
const cpx<float> *hy_vals<float>(const HybridSide &h, bool lx) { return lx ? h.lx32 : h.xl32; }

// out -= D^{X Lambda} Q^{-1} D^{Lambda X} in, after out holds C in
template <class T>
void hybrid_correction(const HybridSide &hy, int n2, int nrhs, const cpx<T> *in, long long ldi, cpx<T> *out,
                       long long ldo, hipStream_t st)
{
    const int dtype = std::is_same<T, double>::value ? MLFMA_C128 : MLFMA_C64;
    cpx<T> *x1 = (cpx<T> *)hy.buf1, *x2 = (cpx<T> *)hy.buf2;
    launch_csr_spmm<T>(hy.n_hdg, nrhs, hy.lx_ptr, hy.lx_col, hy_vals<T>(hy, true), in, ldi, x1, hy.ldbuf, 1.0, false,
                       st);
    HIPCHK(hipGetLastError());
    const int rc = hy.solve(hy.user, dtype, hy.n_hdg, nrhs, x1, hy.ldbuf, x2, hy.ldbuf, (void *)st);
    if (rc != 0) throw Error(MLFMA_ERR_ARG, "the solve with Q returned " + std::to_string(rc));
    launch_csr_spmm<T>(n2, nrhs, hy.xl_ptr, hy.xl_col, hy_vals<T>(hy, false), x2, hy.ldbuf, out, ldo, -1.0, true, st);
    HIPCHK(hipGetLastError());
}

// Restarted GMRES(m) on y = A x (op, precision T), one Krylov space per
// right-hand-side column; every Arnoldi step is one batched product of all
// columns.  Classical Gram-Schmidt applied twice on the device (inner
// products in double), complex Givens rotations and the triangular solve on
// the host.  All columns iterate until the largest estimated relative
// residual reaches tol (or max_iters steps); relres returns the true
// relative residual ||b - A x|| / ||b|| of every column, recomputed at exit.
// With sai (right preconditioning) the Krylov space is built for A M and the
// solution is x0 + M V y; residuals and tol are those of A x = b itself.
// With hy the operator is the reduced matrix of eq. 52, C - D^{X Lambda}
// Q^{-1} D^{Lambda X} (op C).
template <class T>
void gmres(mlfma_ctx *c, Prec<T> &P, int op, int nrhs, const cpx<T> *b, long long ldb, cpx<T> *x, long long ldx,
           int m, int max_iters, double tol, int *iters_out, double *relres, const SaiData *sai, hipStream_t st,
           const HybridSide *hy = nullptr)
{
    typedef std::complex<double> C;
    const long long n = 2LL * c->r.n;
    const int nchunk = (int)std::min<long long>(256, std::max<long long>(1, n / 2048));
    std::vector<void *> list;
    struct Free {
        std::vector<void *> &l;
        ~Free()
        {
            for (void *p : l) (void)hipFree(p);
        }
    } fr{list};
    auto dev = [&](size_t bytes) {
        void *p = nullptr;
        HIPCHK(hipMalloc(&p, std::max<size_t>(bytes, 1)));
        list.push_back(p);
        return p;
    };
    const long long vstride = n * nrhs;
    cpx<T> *V = (cpx<T> *)dev(sizeof(cpx<T>) * (size_t)vstride * (m + 1));
    cpx<T> *w = (cpx<T> *)dev(sizeof(cpx<T>) * (size_t)vstride);
    cpx<double> *part = (cpx<double> *)dev(sizeof(cpx<double>) * (size_t)(m + 1) * nchunk * nrhs);
    cpx<double> *hd = (cpx<double> *)dev(sizeof(cpx<double>) * (size_t)(m + 1) * nrhs);
    cpx<double> *hd2 = (cpx<double> *)dev(sizeof(cpx<double>) * (size_t)(m + 1) * nrhs);
    cpx<double> *ca = (cpx<double> *)dev(sizeof(cpx<double>) * nrhs);
    cpx<double> *cb = (cpx<double> *)dev(sizeof(cpx<double>) * nrhs);
    auto matvec = [&](const cpx<T> *in, long long ldi, cpx<T> *out, long long ldo) {
        product<T>(c, c->ws, op, MLFMA_PART_ALL, nrhs, in, ldi, out, ldo, st, false);
        if (hy) hybrid_correction<T>(*hy, (int)n, nrhs, in, ldi, out, ldo, st);
    };
    cpx<T> *z = sai ? (cpx<T> *)dev(sizeof(cpx<T>) * (size_t)vstride) : nullptr;
    cpx<T> *tv = sai ? (cpx<T> *)dev(sizeof(cpx<T>) * (size_t)vstride) : nullptr;
    auto precond = [&](const cpx<T> *in, cpx<T> *out) {
        launch_sai_apply<T>(c->r.n, nrhs, sai->row_start, sai->ent_col, sai->ent_val, sai_values<T>(*sai), in, n,
                            out, n, st);
    };
    // w = A M v (or A v)
    auto opmul = [&](const cpx<T> *in, cpx<T> *out) {
        if (sai) {
            precond(in, z);
            matvec(z, n, out, n);
        } else {
            matvec(in, n, out, n);
        }
    };
    auto fetch = [&](const cpx<double> *d, int count, std::vector<C> &h) {
        std::vector<cpx<double>> tmp((size_t)count);
        HIPCHK(hipMemcpyAsync(tmp.data(), d, sizeof(cpx<double>) * count, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        h.resize(count);
        for (int i = 0; i < count; i++) h[i] = C(tmp[i].re, tmp[i].im);
    };
    auto put = [&](cpx<double> *d, const std::vector<C> &h) {
        std::vector<cpx<double>> tmp(h.size());
        for (size_t i = 0; i < h.size(); i++) tmp[i] = {h[i].real(), h[i].imag()};
        HIPCHK(hipMemcpyAsync(d, tmp.data(), sizeof(cpx<double>) * tmp.size(), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    };
    auto norms = [&](const cpx<T> *v, long long ld, std::vector<double> &out) {
        std::vector<C> d;
        krylov_dots<T>(v, 0, ld, 1, v, ld, n, nrhs, part, nchunk, hd, st);
        fetch(hd, nrhs, d);
        out.resize(nrhs);
        for (int r = 0; r < nrhs; r++) out[r] = std::sqrt(std::max(0.0, d[r].real()));
    };
    std::vector<double> bnorm;
    norms(b, ldb, bnorm);
    std::vector<C> ones(nrhs, C(1, 0)), mones(nrhs, C(-1, 0));
    int iters = 0;
    bool done = false;
    while (!done) {
        // r = b - A x, V_0 = r / |r|
        matvec(x, ldx, w, n);
        put(ca, ones);
        put(cb, mones);
        krylov_axpby<T>(ca, b, ldb, cb, w, n, V, n, n, nrhs, st);
        std::vector<double> beta;
        norms(V, n, beta);
        std::vector<C> sc(nrhs);
        for (int r = 0; r < nrhs; r++) sc[r] = beta[r] > 0 ? C(1.0 / beta[r], 0) : C(0, 0);
        put(ca, sc);
        krylov_axpby<T>(ca, V, n, nullptr, nullptr, 0, V, n, n, nrhs, st);
        // Hessenberg columns, rotations and right-hand side per column
        std::vector<std::vector<C>> H(nrhs, std::vector<C>((size_t)(m + 1) * m, C(0, 0)));
        std::vector<std::vector<double>> cs(nrhs, std::vector<double>(m, 1.0));
        std::vector<std::vector<C>> sn(nrhs, std::vector<C>(m, C(0, 0)));
        std::vector<std::vector<C>> g(nrhs, std::vector<C>(m + 1, C(0, 0)));
        double worst = 0;
        for (int r = 0; r < nrhs; r++) {
            g[r][0] = C(beta[r], 0);
            worst = std::max(worst, bnorm[r] > 0 ? beta[r] / bnorm[r] : 0.0);
        }
        if (worst <= tol) break;
        int j = 0;
        for (; j < m && iters < max_iters; j++) {
            opmul(V + (size_t)j * vstride, w);
            std::vector<C> h1, h2;
            krylov_dots<T>(V, vstride, n, j + 1, w, n, n, nrhs, part, nchunk, hd, st);
            krylov_combine<T>(V, vstride, n, j + 1, hd, -1.0, w, n, n, nrhs, st);
            krylov_dots<T>(V, vstride, n, j + 1, w, n, n, nrhs, part, nchunk, hd2, st);
            krylov_combine<T>(V, vstride, n, j + 1, hd2, -1.0, w, n, n, nrhs, st);
            fetch(hd, (j + 1) * nrhs, h1);
            fetch(hd2, (j + 1) * nrhs, h2);
            std::vector<double> hn;
            norms(w, n, hn);
            for (int r = 0; r < nrhs; r++) sc[r] = hn[r] > 0 ? C(1.0 / hn[r], 0) : C(0, 0);
            put(ca, sc);
            krylov_axpby<T>(ca, w, n, nullptr, nullptr, 0, V + (size_t)(j + 1) * vstride, n, n, nrhs, st);
            iters++;
            worst = 0;
            for (int r = 0; r < nrhs; r++) {
                std::vector<C> col(j + 2);
                for (int i = 0; i <= j; i++) col[i] = h1[i * nrhs + r] + h2[i * nrhs + r];
                col[j + 1] = C(hn[r], 0);
                for (int i = 0; i < j; i++) {   // earlier rotations
                    const C a = col[i], bb = col[i + 1];
                    col[i] = cs[r][i] * a + sn[r][i] * bb;
                    col[i + 1] = -std::conj(sn[r][i]) * a + cs[r][i] * bb;
                }
                const C a = col[j];
                const double bb = col[j + 1].real(), t = std::sqrt(std::norm(a) + bb * bb);
                if (t == 0) {
                    cs[r][j] = 1;
                    sn[r][j] = 0;
                } else if (std::abs(a) == 0) {
                    cs[r][j] = 0;
                    sn[r][j] = 1;
                } else {
                    cs[r][j] = std::abs(a) / t;
                    sn[r][j] = (a / std::abs(a)) * (bb / t);
                }
                col[j] = cs[r][j] * a + sn[r][j] * col[j + 1];
                col[j + 1] = 0;
                for (int i = 0; i <= j; i++) H[r][(size_t)i * m + j] = col[i];
                g[r][j + 1] = -std::conj(sn[r][j]) * g[r][j];
                g[r][j] = cs[r][j] * g[r][j];
                worst = std::max(worst, bnorm[r] > 0 ? std::abs(g[r][j + 1]) / bnorm[r] : 0.0);
            }
            if (worst <= tol) {
                j++;
                done = true;
                break;
            }
        }
        if (iters >= max_iters) done = true;
        // x += V y with H y = g (upper triangular, j columns)
        if (j > 0) {
            std::vector<C> y((size_t)j * nrhs, C(0, 0));
            for (int r = 0; r < nrhs; r++)
                for (int i = j - 1; i >= 0; i--) {
                    C s = g[r][i];
                    for (int k = i + 1; k < j; k++) s -= H[r][(size_t)i * m + k] * y[(size_t)k * nrhs + r];
                    const C d = H[r][(size_t)i * m + i];
                    y[(size_t)i * nrhs + r] = std::abs(d) > 0 ? s / d : C(0, 0);
                }
            put(hd, y);
            if (sai) {
                // x += M (V y)
                HIPCHK(hipMemsetAsync(tv, 0, sizeof(cpx<T>) * (size_t)vstride, st));
                krylov_combine<T>(V, vstride, n, j, hd, 1.0, tv, n, n, nrhs, st);
                precond(tv, z);
                put(ca, ones);
                put(cb, ones);
                krylov_axpby<T>(ca, x, ldx, cb, z, n, x, ldx, n, nrhs, st);
            } else {
                krylov_combine<T>(V, vstride, n, j, hd, 1.0, x, ldx, n, nrhs, st);
            }
        }
    }
    // true residual
    matvec(x, ldx, w, n);
    put(ca, ones);
    put(cb, mones);
    krylov_axpby<T>(ca, b, ldb, cb, w, n, w, n, n, nrhs, st);
    std::vector<double> rn;
    norms(w, n, rn);
    for (int r = 0; r < nrhs; r++) relres[r] = bnorm[r] > 0 ? rn[r] / bnorm[r] : 0.0;
    if (iters_out) *iters_out = iters;
}

int fail(const Error &e)
{
    g_last_error = e.what();
    return e.code;
}

// Checks and runs mlfma_gmres_precond; with hy, on the reduced operator of
// eq. 52 (op C only).
int gmres_entry(mlfma_handle h, int op, int dtype, long long nrhs, const void *b, long long ldb, void *x,
                long long ldx, int restart, int max_iters, double tol, int precond, int *iters, double *relres,
                void *hip_stream, const HybridSide *hy)
{
    g_last_error.clear();
    if (!h) return fail(Error(MLFMA_ERR_ARG, "NULL handle"));
    if (!h->near_ready) return fail(Error(MLFMA_ERR_STATE, "mlfma_precompute_nearfield has not been called"));
    if (op != MLFMA_OP_C && op != MLFMA_OP_EM) return fail(Error(MLFMA_ERR_ARG, "unknown op"));
    if (dtype != MLFMA_C128 && dtype != MLFMA_C64) return fail(Error(MLFMA_ERR_ARG, "unknown dtype"));
    const long long N2 = 2LL * h->r.n;
    if (nrhs < 1 || nrhs > 4096 || !b || !x || !relres || ldb < N2 || ldx < N2 || restart < 1 || restart > 512 ||
        max_iters < 1 || !(tol > 0))
        return fail(Error(MLFMA_ERR_ARG, "bad nrhs, pointer, leading dimension, restart, max_iters or tol"));
    if (hy && (op != MLFMA_OP_C || nrhs > hy->max_rhs))
        return fail(Error(MLFMA_ERR_ARG, "the hybrid operator is op C with at most max_rhs columns"));
    if (precond != MLFMA_PRECOND_NONE && precond != MLFMA_PRECOND_SAI)
        return fail(Error(MLFMA_ERR_ARG, "unknown preconditioner"));
    const SaiData *sai = nullptr;
    if (precond == MLFMA_PRECOND_SAI) {
        if (!h->sai[op].ready) return fail(Error(MLFMA_ERR_STATE, "mlfma_sai_build has not been called for this op"));
        sai = &h->sai[op];
    }
    const size_t esz = dtype == MLFMA_C128 ? 16 : 8;
    const char *bb = (const char *)b, *xb = (const char *)x;
    if (bb < xb + (size_t)(ldx * (nrhs - 1) + N2) * esz && xb < bb + (size_t)(ldb * (nrhs - 1) + N2) * esz)
        return fail(Error(MLFMA_ERR_ARG, "b and x overlap"));
    try {
        DeviceGuard g(h->device);
        HIPCHK(hipGetLastError());
        ensure_workspace(h, (int)nrhs);
        hipStream_t st = (hipStream_t)hip_stream;
        if (dtype == MLFMA_C128)
            gmres<double>(h, h->p64, op, (int)nrhs, (const cpx<double> *)b, ldb, (cpx<double> *)x, ldx, restart,
                          max_iters, tol, iters, relres, sai, st, hy);
        else
            gmres<float>(h, h->p32, op, (int)nrhs, (const cpx<float> *)b, ldb, (cpx<float> *)x, ldx, restart,
                         max_iters, tol, iters, relres, sai, st, hy);
        HIPCHK(hipGetLastError());
        return MLFMA_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

}  // namespace

// =================================================================== C ABI
namespace mlfma {
namespace {

template <class T>
Prec<T> &prec_of(mlfma_ctx *c)
{
    if constexpr (std::is_same<T, double>::value) return c->p64;
    else return c->p32;
}

// Items in lockstep: every item's first phase, then the translations of all
// items' levels as sibling-group work lists (at most TRANS_MAXLEV levels per
// launch) with the shape tuned for the item with the most translation work,
// then every item's last phase.
template <class T>
void batch_fused(const mlfma_batch_item *items, int n, hipStream_t st)
{
    // the items' own phases run concurrently on their handles' batch
    // streams, forked from st before and after the shared translations
    auto fork = [&] {
        HIPCHK(hipEventRecord(items[0].h->bfork, st));
        for (int i = 0; i < n; i++) HIPCHK(hipStreamWaitEvent(items[i].h->bstream, items[0].h->bfork, 0));
    };
    auto join = [&] {
        for (int i = 0; i < n; i++) {
            HIPCHK(hipEventRecord(items[i].h->bjoin, items[i].h->bstream));
            HIPCHK(hipStreamWaitEvent(st, items[i].h->bjoin, 0));
        }
    };
    std::vector<MvRun<T>> runs;
    runs.reserve(n);
    for (int i = 0; i < n; i++) {
        mlfma_ctx *h = items[i].h;
        runs.push_back(mv_setup<T>(h, h->ws, prec_of<T>(h), items[i].op, MLFMA_PART_ALL, (int)items[i].nrhs,
                                   h->bstream, false));
    }
    fork();
    for (int i = 0; i < n; i++) mv_begin<T>(runs[i], (const cpx<T> *)items[i].x, items[i].ldx);
    join();
    const int nrhs = (int)items[0].nrhs;
    int ref = 0;
    long long most = -1;
    for (int i = 0; i < n; i++) {
        long long work = 0;
        const Tree &tr = items[i].h->tr;
        for (int l = 2; l < tr.levels; l++) work += (long long)tr.lv[l].il_start[tr.lv[l].nbox] * tr.lv[l].K;
        if (work > most) {
            most = work;
            ref = i;
        }
    }
    const Prec<T> &PR = prec_of<T>(items[ref].h);
    const TransShape gs = trans_shape(PR, nrhs);
    const int gi = gs.gi, rb = gs.rb, rw = gs.rw, lds = gs.lds;
    GroupArgs<T> ga;
    ga.tg = group_tg(gi);
    ga.rb = rb;
    ga.rw = rw;
    ga.lds = lds;
    auto flush = [&] {
        if (ga.nlev > 0 && !launch_translate_groups<T>(ga, nrhs, st))
            throw Error(MLFMA_ERR_STATE, "invalid sibling-group translation shape");
        ga.nlev = 0;
    };
    for (int i = 0; i < n; i++) {
        if (!runs[i].far) continue;
        mlfma_ctx *h = items[i].h;
        const GroupArgs<T> one = group_args<T>(h, prec_of<T>(h), h->ws, -1, gi, rb, rw, lds);
        for (int l = 0; l < one.nlev; l++) {
            if (ga.nlev == TRANS_MAXLEV) flush();
            ga.lv[ga.nlev++] = one.lv[l];
        }
    }
    flush();
    fork();
    for (int i = 0; i < n; i++) mv_end<T>(runs[i], (cpx<T> *)items[i].y, items[i].ldy);
    join();
}

}  // namespace
}  // namespace mlfma

extern "C" {

const char *mlfma_last_error(void) { return g_last_error.c_str(); }

int mlfma_options_default(mlfma_options *opt)
{
    if (!opt) return MLFMA_ERR_ARG;
    opt->wavenumber = 2 * M_PI;
    opt->leaf_size = 0.25;
    opt->digits = 3;
    opt->interp_order = 8;
    opt->leaf_extra_L = 2;
    opt->max_rhs = 1;
    opt->device = -1;
    opt->hbm_budget_bytes = 0;
    opt->trans_kernel = MLFMA_TRANS_AUTO;
    opt->level_kernel = MLFMA_LEVELS_AUTO;
    opt->near_precision = MLFMA_PREC_DTYPE;
    opt->far_precision = MLFMA_PREC_DTYPE;
    return MLFMA_OK;
}

int mlfma_build_tree(const double *verts, long long n_verts, const int *tris, long long n_tris,
                     const mlfma_options *opt, mlfma_handle *out)
{
    g_last_error.clear();
    if (!out) return fail(Error(MLFMA_ERR_ARG, "out handle pointer is NULL"));
    *out = nullptr;
    try {
        std::unique_ptr<mlfma_ctx> c(new mlfma_ctx());
        static std::atomic<long long> next_uid{1};
        c->uid = next_uid++;
        if (opt) c->opt = *opt;
        else mlfma_options_default(&c->opt);
        if (c->opt.max_rhs < 1) throw Error(MLFMA_ERR_ARG, "max_rhs must be >= 1");
        if (c->opt.trans_kernel < MLFMA_TRANS_AUTO || c->opt.trans_kernel > MLFMA_TRANS_LDS)
            throw Error(MLFMA_ERR_ARG, "unknown translation kernel");
        if (c->opt.level_kernel < MLFMA_LEVELS_AUTO || c->opt.level_kernel > MLFMA_LEVELS_PIPELINED)
            throw Error(MLFMA_ERR_ARG, "unknown level-step kernel");
        for (int pr : {c->opt.near_precision, c->opt.far_precision})
            if (pr < MLFMA_PREC_DTYPE || pr > MLFMA_PREC_FP32) throw Error(MLFMA_ERR_ARG, "unknown precision");
        c->mixed = c->opt.near_precision == MLFMA_PREC_FP32 || c->opt.far_precision == MLFMA_PREC_FP32;
        build_surface(c->s, verts, n_verts, tris, n_tris);
        build_rwg(c->s, c->r);
        build_tree(c->s, c->r, c->opt.wavenumber, c->opt.leaf_size, c->opt.digits, c->opt.interp_order,
                   c->opt.leaf_extra_L, c->tr);
        check_touching_near(c->s, c->r, c->tr);
        int dev = c->opt.device;
        if (dev < 0) HIPCHK(hipGetDevice(&dev));
        c->device = dev;
        DeviceGuard g(dev);
        build_device_tables(c.get());
        ensure_workspace(c.get(), c->opt.max_rhs);
        tune_translation<double>(c.get(), c->p64);
        tune_translation<float>(c.get(), c->p32);
        c->tile_cache.clear();
        tune_step_rb<double>(c.get(), c->p64);
        tune_step_rb<float>(c.get(), c->p32);
        tune_level_steps(c.get());
        *out = c.release();
        return MLFMA_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error(MLFMA_ERR_OOM, "host memory exhausted"));
    } catch (const std::exception &e) {
        return fail(Error(MLFMA_ERR_HIP, e.what()));
    }
}

int mlfma_precompute_nearfield(mlfma_handle h)
{
    g_last_error.clear();
    if (!h) return fail(Error(MLFMA_ERR_ARG, "NULL handle"));
    try {
        DeviceGuard g(h->device);
        if (!h->near_ready) precompute_near(h);
        return MLFMA_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error(MLFMA_ERR_OOM, "host memory exhausted"));
    }
}

int mlfma_matvec_part(mlfma_handle h, int op, int dtype, int part, long long nrhs, const void *x, long long ldx,
                      void *y, long long ldy, void *hip_stream)
{
    g_last_error.clear();
    if (!h) return fail(Error(MLFMA_ERR_ARG, "NULL handle"));
    if (!h->near_ready) return fail(Error(MLFMA_ERR_STATE, "mlfma_precompute_nearfield has not been called"));
    if (op != MLFMA_OP_C && op != MLFMA_OP_EM) return fail(Error(MLFMA_ERR_ARG, "unknown op"));
    if (dtype != MLFMA_C128 && dtype != MLFMA_C64) return fail(Error(MLFMA_ERR_ARG, "unknown dtype"));
    if (!(part >= 1 && part <= 3) && !(part >= MLFMA_PART_LEVEL + 2 && part < MLFMA_PART_LEVEL + h->tr.levels))
        return fail(Error(MLFMA_ERR_ARG, "unknown part"));
    const long long N2 = 2LL * h->r.n;
    if (nrhs < 1 || nrhs > (1 << 20) || !x || !y || ldx < N2 || ldy < N2)
        return fail(Error(MLFMA_ERR_ARG, "bad nrhs, pointer or leading dimension"));
    const size_t esz = dtype == MLFMA_C128 ? 16 : 8;
    const char *xb = (const char *)x, *yb = (const char *)y;
    if (xb < yb + (size_t)(ldy * (nrhs - 1) + N2) * esz && yb < xb + (size_t)(ldx * (nrhs - 1) + N2) * esz)
        return fail(Error(MLFMA_ERR_ARG, "x and y overlap"));
    try {
        DeviceGuard g(h->device);
        HIPCHK(hipGetLastError());
        ensure_workspace(h, (int)nrhs);
        hipStream_t st = (hipStream_t)hip_stream;
        if (dtype == MLFMA_C128)
            product<double>(h, h->ws, op, part, (int)nrhs, (const cpx<double> *)x, ldx, (cpx<double> *)y,
                            ldy, st, h->prof);
        else
            product<float>(h, h->ws, op, part, (int)nrhs, (const cpx<float> *)x, ldx, (cpx<float> *)y,
                           ldy, st, h->prof);
        HIPCHK(hipGetLastError());
        return MLFMA_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

int mlfma_matvec_batch_fused(const mlfma_batch_item *items, int n_items, void *hip_stream)
{
    g_last_error.clear();
    if (n_items < 0 || (n_items > 0 && !items)) return fail(Error(MLFMA_ERR_ARG, "bad item list"));
    if (n_items == 0) return MLFMA_OK;
    for (int i = 0; i < n_items; i++) {
        const mlfma_batch_item &it = items[i];
        const std::string at = "item " + std::to_string(i) + ": ";
        if (!it.h) return fail(Error(MLFMA_ERR_ARG, at + "NULL handle"));
        if (!it.h->near_ready)
            return fail(Error(MLFMA_ERR_STATE, at + "mlfma_precompute_nearfield has not been called"));
        if (it.h->device != items[0].h->device) return fail(Error(MLFMA_ERR_ARG, at + "geometry on another device"));
        for (int j = 0; j < i; j++)
            if (items[j].h == it.h) return fail(Error(MLFMA_ERR_ARG, at + "geometry already in the batch"));
        if (it.h->mixed) return fail(Error(MLFMA_ERR_ARG, at + "handle with FP32 parts of complex128 products"));
        if (it.op != MLFMA_OP_C && it.op != MLFMA_OP_EM) return fail(Error(MLFMA_ERR_ARG, at + "unknown op"));
        if (it.dtype != MLFMA_C128 && it.dtype != MLFMA_C64) return fail(Error(MLFMA_ERR_ARG, at + "unknown dtype"));
        if (it.dtype != items[0].dtype || it.nrhs != items[0].nrhs)
            return fail(Error(MLFMA_ERR_ARG, at + "dtype or nrhs differs from item 0"));
        const long long N2 = 2LL * it.h->r.n;
        if (it.nrhs < 1 || it.nrhs > (1 << 20) || !it.x || !it.y || it.ldx < N2 || it.ldy < N2)
            return fail(Error(MLFMA_ERR_ARG, at + "bad nrhs, pointer or leading dimension"));
        const size_t esz = it.dtype == MLFMA_C128 ? 16 : 8;
        const char *xb = (const char *)it.x, *yb = (const char *)it.y;
        if (xb < yb + (size_t)(it.ldy * (it.nrhs - 1) + N2) * esz &&
            yb < xb + (size_t)(it.ldx * (it.nrhs - 1) + N2) * esz)
            return fail(Error(MLFMA_ERR_ARG, at + "x and y overlap"));
    }
    try {
        DeviceGuard g(items[0].h->device);
        HIPCHK(hipGetLastError());
        for (int i = 0; i < n_items; i++) {
            mlfma_ctx *h = items[i].h;
            ensure_workspace(h, (int)items[i].nrhs);
            if (!h->bstream) {
                HIPCHK(hipStreamCreateWithFlags(&h->bstream, hipStreamNonBlocking));
                HIPCHK(hipEventCreateWithFlags(&h->bfork, hipEventDisableTiming));
                HIPCHK(hipEventCreateWithFlags(&h->bjoin, hipEventDisableTiming));
            }
        }
        hipStream_t st = (hipStream_t)hip_stream;
        if (items[0].dtype == MLFMA_C128) batch_fused<double>(items, n_items, st);
        else batch_fused<float>(items, n_items, st);
        HIPCHK(hipGetLastError());
        return MLFMA_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

int mlfma_matvec_batch(const mlfma_batch_item *items, int n_items, void *hip_stream)
{
    g_last_error.clear();
    if (n_items < 0 || (n_items > 0 && !items)) return fail(Error(MLFMA_ERR_ARG, "bad item list"));
    if (n_items == 0) return MLFMA_OK;
    // every item is checked before anything is enqueued
    for (int i = 0; i < n_items; i++) {
        const mlfma_batch_item &it = items[i];
        const std::string at = "item " + std::to_string(i) + ": ";
        if (!it.h) return fail(Error(MLFMA_ERR_ARG, at + "NULL handle"));
        if (!it.h->near_ready)
            return fail(Error(MLFMA_ERR_STATE, at + "mlfma_precompute_nearfield has not been called"));
        if (it.h->device != items[0].h->device) return fail(Error(MLFMA_ERR_ARG, at + "geometry on another device"));
        if (it.op != MLFMA_OP_C && it.op != MLFMA_OP_EM) return fail(Error(MLFMA_ERR_ARG, at + "unknown op"));
        if (it.dtype != MLFMA_C128 && it.dtype != MLFMA_C64) return fail(Error(MLFMA_ERR_ARG, at + "unknown dtype"));
        const long long N2 = 2LL * it.h->r.n;
        if (it.nrhs < 1 || it.nrhs > (1 << 20) || !it.x || !it.y || it.ldx < N2 || it.ldy < N2)
            return fail(Error(MLFMA_ERR_ARG, at + "bad nrhs, pointer or leading dimension"));
        const size_t esz = it.dtype == MLFMA_C128 ? 16 : 8;
        const char *xb = (const char *)it.x, *yb = (const char *)it.y;
        if (xb < yb + (size_t)(it.ldy * (it.nrhs - 1) + N2) * esz &&
            yb < xb + (size_t)(it.ldx * (it.nrhs - 1) + N2) * esz)
            return fail(Error(MLFMA_ERR_ARG, at + "x and y overlap"));
    }
    try {
        DeviceGuard g(items[0].h->device);
        HIPCHK(hipGetLastError());
        // geometries in order of first appearance, with their widest product
        std::vector<std::pair<mlfma_handle, long long>> hs;
        for (int i = 0; i < n_items; i++) {
            auto f = std::find_if(hs.begin(), hs.end(), [&](const auto &p) { return p.first == items[i].h; });
            if (f == hs.end()) hs.push_back({items[i].h, items[i].nrhs});
            else f->second = std::max(f->second, items[i].nrhs);
        }
        for (auto &p : hs) {
            ensure_workspace(p.first, (int)p.second);
            if (!p.first->bstream) {
                HIPCHK(hipStreamCreateWithFlags(&p.first->bstream, hipStreamNonBlocking));
                HIPCHK(hipEventCreateWithFlags(&p.first->bfork, hipEventDisableTiming));
                HIPCHK(hipEventCreateWithFlags(&p.first->bjoin, hipEventDisableTiming));
            }
        }
        hipStream_t st = (hipStream_t)hip_stream;
        const bool fork = hs.size() > 1;
        if (fork) {
            HIPCHK(hipEventRecord(hs[0].first->bfork, st));
            for (auto &p : hs) HIPCHK(hipStreamWaitEvent(p.first->bstream, hs[0].first->bfork, 0));
        }
        for (int i = 0; i < n_items; i++) {
            const mlfma_batch_item &it = items[i];
            mlfma_ctx *h = it.h;
            hipStream_t s = fork ? h->bstream : st;
            if (it.dtype == MLFMA_C128)
                product<double>(h, h->ws, it.op, MLFMA_PART_ALL, (int)it.nrhs, (const cpx<double> *)it.x,
                                it.ldx, (cpx<double> *)it.y, it.ldy, s, h->prof);
            else
                product<float>(h, h->ws, it.op, MLFMA_PART_ALL, (int)it.nrhs, (const cpx<float> *)it.x,
                               it.ldx, (cpx<float> *)it.y, it.ldy, s, h->prof);
        }
        if (fork)
            for (auto &p : hs) {
                HIPCHK(hipEventRecord(p.first->bjoin, p.first->bstream));
                HIPCHK(hipStreamWaitEvent(st, p.first->bjoin, 0));
            }
        HIPCHK(hipGetLastError());
        return MLFMA_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

// ------------------------------------------------------------ graph capture
struct mlfma_graph_s {
    mlfma_handle h = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    long long ws_gen = 0;
};

int mlfma_graph_create(mlfma_handle h, int op, int dtype, long long nrhs, const void *x, long long ldx, void *y,
                       long long ldy, mlfma_graph *out)
{
    g_last_error.clear();
    if (!out) return fail(Error(MLFMA_ERR_ARG, "out graph pointer is NULL"));
    *out = nullptr;
    if (!h) return fail(Error(MLFMA_ERR_ARG, "NULL handle"));
    if (!h->near_ready) return fail(Error(MLFMA_ERR_STATE, "mlfma_precompute_nearfield has not been called"));
    if (op != MLFMA_OP_C && op != MLFMA_OP_EM) return fail(Error(MLFMA_ERR_ARG, "unknown op"));
    if (dtype != MLFMA_C128 && dtype != MLFMA_C64) return fail(Error(MLFMA_ERR_ARG, "unknown dtype"));
    const long long N2 = 2LL * h->r.n;
    if (nrhs < 1 || nrhs > (1 << 20) || !x || !y || ldx < N2 || ldy < N2)
        return fail(Error(MLFMA_ERR_ARG, "bad nrhs, pointer or leading dimension"));
    const size_t esz = dtype == MLFMA_C128 ? 16 : 8;
    const char *xb = (const char *)x, *yb = (const char *)y;
    if (xb < yb + (size_t)(ldy * (nrhs - 1) + N2) * esz && yb < xb + (size_t)(ldx * (nrhs - 1) + N2) * esz)
        return fail(Error(MLFMA_ERR_ARG, "x and y overlap"));
    std::unique_ptr<mlfma_graph_s> g(new mlfma_graph_s());
    hipStream_t cs = nullptr;
    try {
        DeviceGuard dg(h->device);
        HIPCHK(hipGetLastError());
        ensure_workspace(h, (int)nrhs);
        HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        try {
            if (dtype == MLFMA_C128)
                product<double>(h, h->ws, op, MLFMA_PART_ALL, (int)nrhs, (const cpx<double> *)x, ldx,
                                (cpx<double> *)y, ldy, cs, false);
            else
                product<float>(h, h->ws, op, MLFMA_PART_ALL, (int)nrhs, (const cpx<float> *)x, ldx,
                               (cpx<float> *)y, ldy, cs, false);
        } catch (...) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(cs, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            throw;
        }
        HIPCHK(hipStreamEndCapture(cs, &g->graph));
        HIPCHK(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
        (void)hipStreamDestroy(cs);
        cs = nullptr;
        g->h = h;
        g->ws_gen = h->ws_gen;
        *out = g.release();
        return MLFMA_OK;
    } catch (const Error &e) {
        if (cs) (void)hipStreamDestroy(cs);
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        return fail(e);
    }
}

int mlfma_graph_launch(mlfma_graph g, void *hip_stream)
{
    g_last_error.clear();
    if (!g || !g->exec) return fail(Error(MLFMA_ERR_ARG, "NULL graph"));
    if (g->ws_gen != g->h->ws_gen)
        return fail(Error(MLFMA_ERR_STATE, "the handle's workspace was reallocated after the capture"));
    try {
        DeviceGuard dg(g->h->device);
        HIPCHK(hipGraphLaunch(g->exec, (hipStream_t)hip_stream));
        return MLFMA_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

int mlfma_gmres(mlfma_handle h, int op, int dtype, long long nrhs, const void *b, long long ldb, void *x,
                long long ldx, int restart, int max_iters, double tol, int *iters, double *relres, void *hip_stream)
{
    return mlfma_gmres_precond(h, op, dtype, nrhs, b, ldb, x, ldx, restart, max_iters, tol, MLFMA_PRECOND_NONE,
                               iters, relres, hip_stream);
}

int mlfma_gmres_precond(mlfma_handle h, int op, int dtype, long long nrhs, const void *b, long long ldb, void *x,
                        long long ldx, int restart, int max_iters, double tol, int precond, int *iters,
                        double *relres, void *hip_stream)
{
    return gmres_entry(h, op, dtype, nrhs, b, ldb, x, ldx, restart, max_iters, tol, precond, iters, relres,
                       hip_stream, nullptr);
}

// ------------------------------------------------------ hybrid product
struct mlfma_hybrid_s {
    mlfma_handle h = nullptr;
    HybridSide side;
    std::vector<void *> allocs;
};

int mlfma_hybrid_create(mlfma_handle h, long long n_hdg, const long long *dlx_ptr, const int *dlx_col,
                        const double *dlx_val, const long long *dxl_ptr, const int *dxl_col, const double *dxl_val,
                        mlfma_qsolve_fn solve, void *user, void *buf1, void *buf2, long long ldbuf,
                        long long max_rhs, mlfma_hybrid *out)
{
    g_last_error.clear();
    if (!out) return fail(Error(MLFMA_ERR_ARG, "out pointer is NULL"));
    *out = nullptr;
    if (!h || !solve || !buf1 || !buf2 || !dlx_ptr || !dxl_ptr) return fail(Error(MLFMA_ERR_ARG, "NULL argument"));
    const long long N2 = 2LL * h->r.n;
    if (n_hdg < 1 || n_hdg > (1LL << 31) - 1 || max_rhs < 1 || max_rhs > 4096 || ldbuf < n_hdg)
        return fail(Error(MLFMA_ERR_ARG, "bad n_hdg, max_rhs or buffer leading dimension"));
    // CSR checks: row pointers start at 0 and never decrease, columns in range
    auto check = [&](const long long *ptr, const int *col, const double *val, long long rows, long long ncols,
                     const char *what) {
        if (ptr[0] != 0) throw Error(MLFMA_ERR_ARG, std::string(what) + ": row pointers must start at 0");
        for (long long i = 0; i < rows; i++)
            if (ptr[i + 1] < ptr[i]) throw Error(MLFMA_ERR_ARG, std::string(what) + ": decreasing row pointers");
        const long long nnz = ptr[rows];
        if (nnz > 0 && (!col || !val)) throw Error(MLFMA_ERR_ARG, std::string(what) + ": NULL columns or values");
        for (long long k = 0; k < nnz; k++)
            if (col[k] < 0 || col[k] >= ncols) throw Error(MLFMA_ERR_ARG, std::string(what) + ": column out of range");
        return nnz;
    };
    std::unique_ptr<mlfma_hybrid_s> hy(new mlfma_hybrid_s());
    try {
        const long long nlx = check(dlx_ptr, dlx_col, dlx_val, n_hdg, N2, "D^{Lambda X}");
        const long long nxl = check(dxl_ptr, dxl_col, dxl_val, N2, n_hdg, "D^{X Lambda}");
        DeviceGuard g(h->device);
        auto up = [&](const void *src, size_t bytes) {
            void *d = nullptr;
            HIPCHK(hipMalloc(&d, std::max<size_t>(bytes, 1)));
            hy->allocs.push_back(d);
            if (bytes) HIPCHK(hipMemcpy(d, src, bytes, hipMemcpyHostToDevice));
            return d;
        };
        auto single = [](const double *v, long long nnz) {
            std::vector<cpx<float>> f((size_t)nnz);
            for (long long k = 0; k < nnz; k++) f[(size_t)k] = {(float)v[2 * k], (float)v[2 * k + 1]};
            return f;
        };
        HybridSide &sd = hy->side;
        sd.n_hdg = n_hdg;
        sd.nnz_lx = nlx;
        sd.nnz_xl = nxl;
        sd.lx_ptr = (long long *)up(dlx_ptr, sizeof(long long) * (size_t)(n_hdg + 1));
        sd.xl_ptr = (long long *)up(dxl_ptr, sizeof(long long) * (size_t)(N2 + 1));
        sd.lx_col = (int *)up(dlx_col, sizeof(int) * (size_t)nlx);
        sd.xl_col = (int *)up(dxl_col, sizeof(int) * (size_t)nxl);
        sd.lx64 = (cpx<double> *)up(dlx_val, sizeof(cpx<double>) * (size_t)nlx);
        sd.xl64 = (cpx<double> *)up(dxl_val, sizeof(cpx<double>) * (size_t)nxl);
        const std::vector<cpx<float>> lx32 = single(dlx_val, nlx), xl32 = single(dxl_val, nxl);
        sd.lx32 = (cpx<float> *)up(lx32.data(), sizeof(cpx<float>) * lx32.size());
        sd.xl32 = (cpx<float> *)up(xl32.data(), sizeof(cpx<float>) * xl32.size());
        sd.solve = solve;
        sd.user = user;
        sd.buf1 = buf1;
        sd.buf2 = buf2;
        sd.ldbuf = ldbuf;
        sd.max_rhs = max_rhs;
        hy->h = h;
        *out = hy.release();
        return MLFMA_OK;
    } catch (const Error &e) {
        for (void *p : hy->allocs) (void)hipFree(p);
        return fail(e);
    }
}

int mlfma_hybrid_matvec(mlfma_hybrid hy, int dtype, long long nrhs, const void *x, long long ldx, void *y,
                        long long ldy, void *hip_stream)
{
    g_last_error.clear();
    if (!hy) return fail(Error(MLFMA_ERR_ARG, "NULL hybrid operator"));
    if (nrhs > hy->side.max_rhs) return fail(Error(MLFMA_ERR_ARG, "nrhs exceeds the solve buffers' max_rhs"));
    const int rc = mlfma_matvec_part(hy->h, MLFMA_OP_C, dtype, MLFMA_PART_ALL, nrhs, x, ldx, y, ldy, hip_stream);
    if (rc != MLFMA_OK) return rc;
    try {
        DeviceGuard g(hy->h->device);
        const int n2 = 2 * hy->h->r.n;
        hipStream_t st = (hipStream_t)hip_stream;
        if (dtype == MLFMA_C128)
            hybrid_correction<double>(hy->side, n2, (int)nrhs, (const cpx<double> *)x, ldx, (cpx<double> *)y, ldy, st);
        else
            hybrid_correction<float>(hy->side, n2, (int)nrhs, (const cpx<float> *)x, ldx, (cpx<float> *)y, ldy, st);
        return MLFMA_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

int mlfma_hybrid_gmres(mlfma_hybrid hy, int dtype, long long nrhs, const void *b, long long ldb, void *x,
                       long long ldx, int restart, int max_iters, double tol, int precond, int *iters,
                       double *relres, void *hip_stream)
{
    g_last_error.clear();
    if (!hy) return fail(Error(MLFMA_ERR_ARG, "NULL hybrid operator"));
    return gmres_entry(hy->h, MLFMA_OP_C, dtype, nrhs, b, ldb, x, ldx, restart, max_iters, tol, precond, iters,
                       relres, hip_stream, &hy->side);
}

int mlfma_hybrid_destroy(mlfma_hybrid hy)
{
    if (!hy) return MLFMA_OK;
    {
        DeviceGuard g(hy->h->device);
        (void)hipDeviceSynchronize();
        for (void *p : hy->allocs) (void)hipFree(p);
    }
    delete hy;
    return MLFMA_OK;
}

int mlfma_graph_destroy(mlfma_graph g)
{
    if (!g) return MLFMA_OK;
    {
        DeviceGuard dg(g->h->device);
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
    }
    delete g;
    return MLFMA_OK;
}

int mlfma_matvec_LK(mlfma_handle h, int op, int dtype, long long nrhs, const void *x, long long ldx, void *y,
                    long long ldy, void *hip_stream)
{
    return mlfma_matvec_part(h, op, dtype, MLFMA_PART_ALL, nrhs, x, ldx, y, ldy, hip_stream);
}

int mlfma_release(mlfma_handle h)
{
    if (!h) return MLFMA_OK;
    {
        DeviceGuard g(h->device);
        (void)hipDeviceSynchronize();
        delete h;
    }
    return MLFMA_OK;
}

int mlfma_query(mlfma_handle h, long long *n_rwg, int *levels, unsigned long long *hbm_bytes)
{
    if (!h) return fail(Error(MLFMA_ERR_ARG, "NULL handle"));
    if (n_rwg) *n_rwg = h->r.n;
    if (levels) *levels = h->tr.levels;
    if (hbm_bytes) *hbm_bytes = h->bytes;
    return MLFMA_OK;
}

int mlfma_rwg_table(mlfma_handle h, int *edge_ab, int *tri_pm)
{
    if (!h) return fail(Error(MLFMA_ERR_ARG, "NULL handle"));
    for (int n = 0; n < h->r.n; n++) {
        if (edge_ab) {
            edge_ab[2 * n] = h->r.a[n];
            edge_ab[2 * n + 1] = h->r.b[n];
        }
        if (tri_pm) {
            tri_pm[2 * n] = h->r.tri[0][n];
            tri_pm[2 * n + 1] = h->r.tri[1][n];
        }
    }
    return MLFMA_OK;
}

int mlfma_level_info(mlfma_handle h, int level, long long info[6])
{
    if (!h || !info || level < 2 || level >= h->tr.levels) return fail(Error(MLFMA_ERR_ARG, "bad level"));
    const Level &L = h->tr.lv[level];
    info[0] = L.nbox;
    info[1] = L.L;
    info[2] = L.K;
    info[3] = (long long)L.il_box.size();
    info[4] = (long long)std::llround(L.a * 1e6);
    info[5] = 0;
    return MLFMA_OK;
}

int mlfma_tuning(mlfma_handle h, int dtype, int shape[4], double *ms)
{
    if (!h || !shape || (dtype != MLFMA_C128 && dtype != MLFMA_C64)) return fail(Error(MLFMA_ERR_ARG, "bad argument"));
    const int group = dtype == MLFMA_C64 ? h->p32.trans_group : h->p64.trans_group;
    shape[0] = group > 0 ? group : (dtype == MLFMA_C64 ? h->p32.trans_tmax : h->p64.trans_tmax);
    const int merged = (dtype == MLFMA_C64 ? h->p32.trans_gi : h->p64.trans_gi) >= 2;
    const int lds = dtype == MLFMA_C64 ? h->p32.trans_lds : h->p64.trans_lds;
    shape[1] = group > 0 ? (lds ? -2 : -merged) : (dtype == MLFMA_C64 ? h->p32.trans_smax : h->p64.trans_smax);
    shape[2] = dtype == MLFMA_C64 ? h->p32.trans_rb : h->p64.trans_rb;
    shape[3] = group > 0 ? (dtype == MLFMA_C64 ? h->p32.trans_rw : h->p64.trans_rw) : 0;
    if (ms) *ms = dtype == MLFMA_C64 ? h->p32.trans_ms : h->p64.trans_ms;
    return MLFMA_OK;
}

int mlfma_tuning_steps(mlfma_handle h, int *matrix_cores, double ms[2])
{
    if (!h) return fail(Error(MLFMA_ERR_ARG, "NULL handle"));
    if (matrix_cores) *matrix_cores = h->p32.level_mfma;
    if (ms) {
        ms[0] = h->p32.step_ms[0];
        ms[1] = h->p32.step_ms[1];
    }
    return MLFMA_OK;
}

int mlfma_tuning_level(mlfma_handle h, int dtype, int level, int shape[5])
{
    if (!h || !shape || (dtype != MLFMA_C128 && dtype != MLFMA_C64)) return fail(Error(MLFMA_ERR_ARG, "bad argument"));
    if (level < 2 || level + 1 >= h->tr.levels) return fail(Error(MLFMA_ERR_ARG, "level out of range"));
    auto get = [&](const auto &P) {
        const auto &PL = P.lv[level];
        shape[0] = PL.agg_rb;
        shape[1] = PL.agg_pipe;
        shape[2] = PL.dis_rb;
        shape[3] = PL.dis_pipe;
        shape[4] = PL.agg_group;
    };
    if (dtype == MLFMA_C64) get(h->p32);
    else get(h->p64);
    return MLFMA_OK;
}

int mlfma_near_info(mlfma_handle h, long long info[4])
{
    if (!h || !info) return fail(Error(MLFMA_ERR_ARG, "NULL argument"));
    if (!h->near_ready) return fail(Error(MLFMA_ERR_STATE, "near field not computed"));
    info[0] = h->n_slots;
    info[1] = h->n_id;
    info[2] = h->n_touch;
    info[3] = h->tr.lv[h->tr.levels - 1].nbox;
    return MLFMA_OK;
}

int mlfma_profile(mlfma_handle h, int enable)
{
    if (!h) return fail(Error(MLFMA_ERR_ARG, "NULL handle"));
    try {
        DeviceGuard g(h->device);
        h->drain_events();
        if (enable) {
            for (double &v : h->stage_ms) v = 0;
            h->prof_calls = 0;
        }
        h->prof = enable != 0;
        return MLFMA_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

int mlfma_profile_read(mlfma_handle h, double ms[8], long long *calls)
{
    if (!h) return fail(Error(MLFMA_ERR_ARG, "NULL handle"));
    try {
        DeviceGuard g(h->device);
        h->drain_events();
        if (ms)
            for (int s = 0; s < MLFMA_STAGES; s++) ms[s] = h->stage_ms[s];
        if (calls) *calls = h->prof_calls;
        return MLFMA_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

int mlfma_plane_wave_rhs(mlfma_handle h, int dtype, long long nrhs, const double *khat, const double *pol, void *b,
                         long long ldb, void *hip_stream)
{
    g_last_error.clear();
    if (!h || !khat || !pol || !b || nrhs < 1 || ldb < 2LL * h->r.n || (dtype != MLFMA_C128 && dtype != MLFMA_C64))
        return fail(Error(MLFMA_ERR_ARG, "bad arguments"));
    try {
        DeviceGuard g(h->device);
        std::vector<double> dirs(6 * (size_t)nrhs);
        for (long long r = 0; r < nrhs; r++)
            for (int d = 0; d < 3; d++) {
                dirs[6 * r + d] = khat[3 * r + d];
                dirs[6 * r + 3 + d] = pol[3 * r + d];
            }
        std::vector<void *> tmp;
        const unsigned long long before = h->bytes;
        double *d_dirs = h->dalloc<double>(dirs.size(), &tmp);
        HIPCHK(hipMemcpy(d_dirs, dirs.data(), dirs.size() * 8, hipMemcpyHostToDevice));
        hipStream_t st = (hipStream_t)hip_stream;
        launch_plane_wave(dtype == MLFMA_C64, h->r.n, (int)nrhs, h->opt.wavenumber, h->perm, h->g_rtri, h->g_rloc,
                          h->g_rcoef, h->g_tv, h->g_tn, h->g_ta, d_dirs, b, ldb, st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        for (void *p : tmp) (void)hipFree(p);
        h->bytes = before;
        return MLFMA_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

int mlfma_far_field(mlfma_handle h, int dtype, long long nrhs, const void *x, long long ldx, long long ndir,
                    const double *dirs, void *F, void *hip_stream)
{
    g_last_error.clear();
    if (!h || !x || !F || !dirs || nrhs < 1 || nrhs > 65535 || ndir < 1 || ndir > (1LL << 30) ||
        ldx < 2LL * h->r.n || (dtype != MLFMA_C128 && dtype != MLFMA_C64))
        return fail(Error(MLFMA_ERR_ARG, "bad arguments"));
    for (long long d = 0; d < ndir; d++) {
        const double n2 = dirs[3 * d] * dirs[3 * d] + dirs[3 * d + 1] * dirs[3 * d + 1] + dirs[3 * d + 2] * dirs[3 * d + 2];
        if (!(std::abs(n2 - 1.0) <= 1e-9)) return fail(Error(MLFMA_ERR_ARG, "directions must be unit vectors"));
    }
    std::vector<void *> tmp;
    const unsigned long long before = h->bytes;
    struct Free {
        mlfma_ctx *h;
        std::vector<void *> &l;
        unsigned long long b;
        ~Free()
        {
            for (void *p : l) (void)hipFree(p);
            h->bytes = b;
        }
    } fr{h, tmp, before};
    try {
        DeviceGuard g(h->device);
        double *d_dirs = h->dalloc<double>(3 * (size_t)ndir, &tmp);
        HIPCHK(hipMemcpy(d_dirs, dirs, 3 * (size_t)ndir * 8, hipMemcpyHostToDevice));
        hipStream_t st = (hipStream_t)hip_stream;
        launch_far_field(dtype == MLFMA_C64, h->r.n, h->opt.wavenumber, h->perm, h->g_rtri, h->g_rloc, h->g_rcoef,
                         h->g_tv, h->g_ta, d_dirs, (int)ndir, x, ldx, F, (int)nrhs, st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        return MLFMA_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

int mlfma_sai_build(mlfma_handle h, int op, int k_nearest)
{
    g_last_error.clear();
    if (!h) return fail(Error(MLFMA_ERR_ARG, "NULL handle"));
    if (op != MLFMA_OP_C && op != MLFMA_OP_EM) return fail(Error(MLFMA_ERR_ARG, "unknown op"));
    if (k_nearest < 1 || k_nearest > SAI_MAXP) return fail(Error(MLFMA_ERR_ARG, "k_nearest outside 1..32"));
    if (!h->near_ready) return fail(Error(MLFMA_ERR_STATE, "mlfma_precompute_nearfield has not been called"));
    try {
        DeviceGuard g(h->device);
        HIPCHK(hipGetLastError());
        build_sai(h, op, k_nearest);
        return MLFMA_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

int mlfma_sai_apply(mlfma_handle h, int op, int dtype, long long nrhs, const void *x, long long ldx, void *y,
                    long long ldy, void *hip_stream)
{
    g_last_error.clear();
    if (!h) return fail(Error(MLFMA_ERR_ARG, "NULL handle"));
    if (op != MLFMA_OP_C && op != MLFMA_OP_EM) return fail(Error(MLFMA_ERR_ARG, "unknown op"));
    if (dtype != MLFMA_C128 && dtype != MLFMA_C64) return fail(Error(MLFMA_ERR_ARG, "unknown dtype"));
    const long long N2 = 2LL * h->r.n;
    if (nrhs < 1 || nrhs > 65535 || !x || !y || ldx < N2 || ldy < N2)
        return fail(Error(MLFMA_ERR_ARG, "bad nrhs, pointer or leading dimension"));
    if (!h->sai[op].ready) return fail(Error(MLFMA_ERR_STATE, "mlfma_sai_build has not been called for this op"));
    const size_t esz = dtype == MLFMA_C128 ? 16 : 8;
    const char *xb = (const char *)x, *yb = (const char *)y;
    if (xb < yb + (size_t)(ldy * (nrhs - 1) + N2) * esz && yb < xb + (size_t)(ldx * (nrhs - 1) + N2) * esz)
        return fail(Error(MLFMA_ERR_ARG, "x and y overlap"));
    try {
        DeviceGuard g(h->device);
        const SaiData &d = h->sai[op];
        hipStream_t st = (hipStream_t)hip_stream;
        if (dtype == MLFMA_C128)
            launch_sai_apply<double>(h->r.n, (int)nrhs, d.row_start, d.ent_col, d.ent_val, d.M64,
                                     (const cpx<double> *)x, ldx, (cpx<double> *)y, ldy, st);
        else
            launch_sai_apply<float>(h->r.n, (int)nrhs, d.row_start, d.ent_col, d.ent_val, d.M32,
                                    (const cpx<float> *)x, ldx, (cpx<float> *)y, ldy, st);
        HIPCHK(hipGetLastError());
        return MLFMA_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

int mlfma_sai_info(mlfma_handle h, int op, long long *nnz, int *max_pattern, double *build_ms,
                   unsigned long long *bytes)
{
    g_last_error.clear();
    if (!h) return fail(Error(MLFMA_ERR_ARG, "NULL handle"));
    if (op != MLFMA_OP_C && op != MLFMA_OP_EM) return fail(Error(MLFMA_ERR_ARG, "unknown op"));
    const SaiData &d = h->sai[op];
    if (!d.ready) return fail(Error(MLFMA_ERR_STATE, "mlfma_sai_build has not been called for this op"));
    if (nnz) *nnz = d.nnz;
    if (max_pattern) *max_pattern = d.maxp;
    if (build_ms) *build_ms = d.build_ms;
    if (bytes) *bytes = d.bytes;
    return MLFMA_OK;
}

int mlfma_translation_operator(double k, int L, const double X[3], long long nk, const double *khat, double *out)
{
    if (!(k > 0) || L < 0 || !X || nk < 0 || (nk && (!khat || !out))) return fail(Error(MLFMA_ERR_ARG, "bad args"));
    std::vector<double> kh(khat, khat + 3 * nk);
    std::vector<cdouble> o;
    translation_table(k, L, X, kh, o);
    for (long long q = 0; q < nk; q++) {
        out[2 * q] = o[q].real();
        out[2 * q + 1] = o[q].imag();
    }
    return MLFMA_OK;
}

}  // extern "C"

// ============================================================ scratch product
// The product of mlfma_matvec_LK with its per-product scratch laid over
// caller-provided device memory instead of the handle's workspace: no
// allocation, no second stream (the near field runs on hip_stream), no
// stage timing.  Used by the allocation-free entry point (noalloc.hip).
namespace mlfma {

int handle_device(mlfma_handle h) { return h ? h->device : -1; }

int set_error(int code, const char *msg) { return fail(Error(code, msg)); }

int matvec_in_scratch(mlfma_handle h, int op, int dtype, long long nrhs, const void *x, long long ldx, void *y,
                      long long ldy, void *hip_stream, void *scratch, unsigned long long cap)
{
    g_last_error.clear();
    if (!h) return fail(Error(MLFMA_ERR_ARG, "NULL handle"));
    if (!h->near_ready) return fail(Error(MLFMA_ERR_STATE, "mlfma_precompute_nearfield has not been called"));
    if (op != MLFMA_OP_C && op != MLFMA_OP_EM) return fail(Error(MLFMA_ERR_ARG, "unknown op"));
    if (dtype != MLFMA_C128 && dtype != MLFMA_C64) return fail(Error(MLFMA_ERR_ARG, "unknown dtype"));
    const long long N2 = 2LL * h->r.n;
    if (nrhs < 1 || nrhs > (1 << 20) || !x || !y || ldx < N2 || ldy < N2)
        return fail(Error(MLFMA_ERR_ARG, "bad nrhs, pointer or leading dimension"));
    const size_t esz = dtype == MLFMA_C128 ? 16 : 8;
    const char *xb = (const char *)x, *yb = (const char *)y;
    if (xb < yb + (size_t)(ldy * (nrhs - 1) + N2) * esz && yb < xb + (size_t)(ldx * (nrhs - 1) + N2) * esz)
        return fail(Error(MLFMA_ERR_ARG, "x and y overlap"));
    const unsigned long long need = layout_workspace(h, (int)nrhs, esz, nullptr, nullptr);
    if (!scratch || need > cap)
        return fail(Error(MLFMA_ERR_ARG, "the product needs " + std::to_string(need) +
                                             " bytes of scratch, more than the " + std::to_string(cap) +
                                             " bytes available"));
    try {
        DeviceGuard g(h->device);
        HIPCHK(hipGetLastError());
        Workspace w;
        layout_workspace(h, (int)nrhs, esz, (char *)scratch, &w);
        hipStream_t st = (hipStream_t)hip_stream;
        if (dtype == MLFMA_C128)
            product<double>(h, w, op, MLFMA_PART_ALL, (int)nrhs, (const cpx<double> *)x, ldx,
                            (cpx<double> *)y, ldy, st, false);
        else
            product<float>(h, w, op, MLFMA_PART_ALL, (int)nrhs, (const cpx<float> *)x, ldx,
                           (cpx<float> *)y, ldy, st, false);
        HIPCHK(hipGetLastError());
        return MLFMA_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

}  // namespace mlfma

// ====================================================================== serving
// Continuous batching: client threads submit products for resident
// geometries; a scheduler thread merges queued requests of the same
// (geometry, op, dtype) into one multi-RHS product, admits it to a free
// launch slot (a stream and a workspace arena; arenas are bounded by the
// memory budget), gathers the requests' columns into the slot's batch buffer,
// runs the product and scatters the columns back; a poller thread retires
// finished slots.  Requests that arrive while others run are admitted as
// soon as a slot frees, so work on different geometries overlaps on the GPU.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    long long ticket = 0;
    mlfma_handle h = nullptr;
    int op = 0, dtype = 0, nrhs = 0;
    const void *x = nullptr;
    void *y = nullptr;
    long long ldx = 0, ldy = 0;
    hipEvent_t ready = nullptr;   // recorded on the caller's stream at submit: x and y are usable after it
    Clock::time_point t_submit, t_start, t_done;
    int state = 0;        // 0 queued, 1 running, 2 done, < 0 error code
    int batch_rhs = 0;    // right-hand sides of the product it ran in
    std::string error;    // why the request failed (state < 0)
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    char *arena = nullptr;
    unsigned long long arena_bytes = 0;
    char *xb = nullptr, *yb = nullptr;
    unsigned long long io_bytes = 0;
    bool busy = false;
    std::vector<Request *> reqs;
    // captured products of this slot's arena: (geometry uid, op, dtype, rhs)
    std::map<std::tuple<long long, int, int, int>, hipGraphExec_t> graphs;
};

constexpr size_t SLOT_GRAPHS_MAX = 64;

void clear_graphs(Slot &sl)
{
    for (auto &kv : sl.graphs) (void)hipGraphExecDestroy(kv.second);
    sl.graphs.clear();
}

}  // namespace

struct mlfma_server_s {
    mlfma_server_opts opt{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<long long, Request *> reqs;
    std::vector<Slot> slots;
    unsigned long long arena_total = 0;
    long long next_ticket = 1;
    long long launches = 0, batched_requests = 0;
    bool stop = false;
    int waiters = 0;                   // threads inside mlfma_server_wait
    std::vector<hipEvent_t> free_events;   // pool of the requests' ready events
    std::thread sched, poll;
    hipStream_t capture = nullptr;     // stream the scheduler captures products on
    long long graph_captures = 0;
};

namespace {

unsigned long long io_bytes_for(mlfma_handle h, int rhs) { return 2ULL * h->r.n * rhs * sizeof(cpx<double>); }

// Runs on the scheduler thread with the lock released.
void launch_batch(mlfma_server_s *S, Slot &slot, std::vector<Request *> &batch, int total)
{
    mlfma_handle h = batch[0]->h;
    const int op = batch[0]->op, dtype = batch[0]->dtype;
    const size_t esz = dtype == MLFMA_C128 ? 16 : 8;
    const long long N2 = 2LL * h->r.n;
    // nothing of a request is read or written before the caller's work that
    // preceded its submission
    for (Request *r : batch) HIPCHK(hipStreamWaitEvent(slot.stream, r->ready, 0));
    int col = 0;
    for (Request *r : batch) {
        HIPCHK(hipMemcpy2DAsync(slot.xb + (size_t)col * N2 * esz, N2 * esz, r->x, r->ldx * esz, N2 * esz, r->nrhs,
                                hipMemcpyDeviceToDevice, slot.stream));
        col += r->nrhs;
    }
    Workspace w;
    carve_workspace(h, w, slot.arena, total);
    auto run = [&](hipStream_t st) {
        if (dtype == MLFMA_C128)
            product<double>(h, w, op, MLFMA_PART_ALL, total, (const cpx<double> *)slot.xb, N2,
                            (cpx<double> *)slot.yb, N2, st, false);
        else
            product<float>(h, w, op, MLFMA_PART_ALL, total, (const cpx<float> *)slot.xb, N2,
                           (cpx<float> *)slot.yb, N2, st, false);
    };
    if (S->opt.use_graphs) {
        // replay the product captured for this slot, geometry, op, dtype and
        // width; capture it the first time
        const auto key = std::make_tuple(h->uid, op, dtype, total);
        auto it = slot.graphs.find(key);
        if (it == slot.graphs.end()) {
            if (slot.graphs.size() >= SLOT_GRAPHS_MAX) clear_graphs(slot);
            hipGraph_t graph = nullptr;
            HIPCHK(hipStreamBeginCapture(S->capture, hipStreamCaptureModeThreadLocal));
            try {
                run(S->capture);
            } catch (...) {
                (void)hipStreamEndCapture(S->capture, &graph);
                if (graph) (void)hipGraphDestroy(graph);
                throw;
            }
            HIPCHK(hipStreamEndCapture(S->capture, &graph));
            hipGraphExec_t exec = nullptr;
            const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HIPCHK(e);
            it = slot.graphs.emplace(key, exec).first;
            S->graph_captures++;
        }
        HIPCHK(hipGraphLaunch(it->second, slot.stream));
    } else {
        run(slot.stream);
    }
    col = 0;
    for (Request *r : batch) {
        HIPCHK(hipMemcpy2DAsync(r->y, r->ldy * esz, slot.yb + (size_t)col * N2 * esz, N2 * esz, N2 * esz, r->nrhs,
                                hipMemcpyDeviceToDevice, slot.stream));
        col += r->nrhs;
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(slot.done, slot.stream));
}

void scheduler_loop(mlfma_server_s *S)
{
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (!S->stop) {
        if (S->queue.empty()) {
            S->cv_sched.wait(lk);
            continue;
        }
        Request *r0 = S->queue.front();
        mlfma_handle h = r0->h;
        const int maxb = std::max(S->opt.max_batch_rhs, r0->nrhs);
        const unsigned long long need = workspace_bytes(h, maxb), ion = io_bytes_for(h, maxb);
        // a free slot whose arena fits, else a free slot that may grow within the budget
        int pick = -1;
        for (size_t i = 0; i < S->slots.size(); i++)
            if (!S->slots[i].busy && S->slots[i].arena_bytes >= need && S->slots[i].io_bytes >= ion) { pick = (int)i; break; }
        bool grow = false;
        if (pick < 0)
            for (size_t i = 0; i < S->slots.size(); i++) {
                const Slot &sl = S->slots[i];
                if (sl.busy) continue;
                unsigned long long after = S->arena_total - sl.arena_bytes - 2 * sl.io_bytes + need + 2 * ion;
                if (!S->opt.hbm_budget_bytes || after <= S->opt.hbm_budget_bytes) { pick = (int)i; grow = true; break; }
            }
        if (pick < 0 && S->opt.hbm_budget_bytes) {
            // room may be made by releasing the arenas of other idle slots
            unsigned long long idle = 0;
            int cand = -1;
            for (size_t i = 0; i < S->slots.size(); i++)
                if (!S->slots[i].busy) {
                    idle += S->slots[i].arena_bytes + 2 * S->slots[i].io_bytes;
                    if (cand < 0) cand = (int)i;
                }
            if (cand >= 0 && S->arena_total - idle + need + 2 * ion <= S->opt.hbm_budget_bytes) {
                const Slot &cs = S->slots[cand];
                for (size_t i = 0; i < S->slots.size(); i++) {
                    if (S->arena_total - cs.arena_bytes - 2 * cs.io_bytes + need + 2 * ion <= S->opt.hbm_budget_bytes)
                        break;
                    Slot &sl = S->slots[i];
                    if (sl.busy || (int)i == cand || !sl.arena_bytes) continue;
                    clear_graphs(sl);
                    (void)hipFree(sl.arena);
                    (void)hipFree(sl.xb);
                    (void)hipFree(sl.yb);
                    sl.arena = sl.xb = sl.yb = nullptr;
                    S->arena_total -= sl.arena_bytes + 2 * sl.io_bytes;
                    sl.arena_bytes = sl.io_bytes = 0;
                }
                pick = cand;
                grow = true;
            }
        }
        if (pick < 0) {
            bool any_busy = false;
            for (auto &sl : S->slots) any_busy |= sl.busy;
            if (!any_busy) {          // can never fit: fail the request
                S->queue.pop_front();
                r0->error = "the request's product does not fit the memory budget";
                r0->state = MLFMA_ERR_OOM;
                r0->t_done = Clock::now();
                S->cv_done.notify_all();
                continue;
            }
            S->cv_sched.wait(lk);     // admitted when a slot frees
            continue;
        }
        // merge queued requests of the same geometry, op and dtype
        std::vector<Request *> batch;
        int total = 0;
        for (auto it = S->queue.begin(); it != S->queue.end();) {
            Request *r = *it;
            if (r->h == h && r->op == r0->op && r->dtype == r0->dtype && total + r->nrhs <= maxb) {
                batch.push_back(r);
                total += r->nrhs;
                it = S->queue.erase(it);
            } else {
                ++it;
            }
        }
        Slot &slot = S->slots[pick];
        slot.busy = true;
        const auto now = Clock::now();
        for (Request *r : batch) {
            r->state = 1;
            r->t_start = now;
            r->batch_rhs = total;
        }
        lk.unlock();
        int err = 0;
        std::string why;
        try {
            if (grow) {
                clear_graphs(slot);
                if (slot.arena) (void)hipFree(slot.arena);
                if (slot.xb) (void)hipFree(slot.xb);
                if (slot.yb) (void)hipFree(slot.yb);
                slot.arena = slot.xb = slot.yb = nullptr;
                lk.lock();
                S->arena_total -= slot.arena_bytes + 2 * slot.io_bytes;
                slot.arena_bytes = slot.io_bytes = 0;
                lk.unlock();
                HIPCHK(hipMalloc((void **)&slot.arena, need));
                HIPCHK(hipMalloc((void **)&slot.xb, ion));
                HIPCHK(hipMalloc((void **)&slot.yb, ion));
                lk.lock();
                slot.arena_bytes = need;
                slot.io_bytes = ion;
                S->arena_total += need + 2 * ion;
                lk.unlock();
            }
            launch_batch(S, slot, batch, total);
        } catch (const Error &e) {
            err = e.code;
            why = e.what();
            // copies and kernels already queued may still use the requests'
            // buffers: the caller learns of the failure only once they are done
            (void)hipStreamSynchronize(slot.stream);
        }
        lk.lock();
        S->launches++;
        S->batched_requests += (long long)batch.size();
        if (err) {
            for (Request *r : batch) {
                r->error = why;
                r->state = err;
                r->t_done = Clock::now();
            }
            slot.busy = false;
            S->cv_done.notify_all();
        } else {
            slot.reqs = batch;
        }
    }
}

void poller_loop(mlfma_server_s *S)
{
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (!S->stop) {
        bool any = false;
        for (auto &sl : S->slots) {
            if (!sl.busy || sl.reqs.empty()) continue;
            any = true;
            hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            const auto now = Clock::now();
            for (Request *r : sl.reqs) {
                if (q != hipSuccess) r->error = std::string("device error: ") + hipGetErrorString(q);
                r->state = q == hipSuccess ? 2 : MLFMA_ERR_HIP;
                r->t_done = now;
            }
            sl.reqs.clear();
            sl.busy = false;
            S->cv_done.notify_all();
            S->cv_sched.notify_all();
        }
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(any ? 20 : 200));
        lk.lock();
    }
}

}  // namespace

extern "C" {

int mlfma_server_opts_default(mlfma_server_opts *o)
{
    if (!o) return MLFMA_ERR_ARG;
    o->streams = 4;
    o->max_batch_rhs = 16;
    o->device = -1;
    o->hbm_budget_bytes = 0;
    o->use_graphs = 1;
    return MLFMA_OK;
}

int mlfma_server_create(const mlfma_server_opts *opt, mlfma_server *out)
{
    g_last_error.clear();
    if (!out) return fail(Error(MLFMA_ERR_ARG, "NULL output"));
    *out = nullptr;
    try {
        std::unique_ptr<mlfma_server_s> S(new mlfma_server_s());
        if (opt) S->opt = *opt;
        else mlfma_server_opts_default(&S->opt);
        if (S->opt.streams < 1 || S->opt.streams > 16 || S->opt.max_batch_rhs < 1)
            throw Error(MLFMA_ERR_ARG, "streams must be 1..16 and max_batch_rhs >= 1");
        int dev = S->opt.device;
        if (dev < 0) HIPCHK(hipGetDevice(&dev));
        S->device = dev;
        DeviceGuard g(dev);
        S->slots.resize(S->opt.streams);
        for (auto &sl : S->slots) {
            HIPCHK(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
        }
        HIPCHK(hipStreamCreateWithFlags(&S->capture, hipStreamNonBlocking));
        mlfma_server_s *raw = S.get();
        S->sched = std::thread(scheduler_loop, raw);
        S->poll = std::thread(poller_loop, raw);
        *out = S.release();
        return MLFMA_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

int mlfma_server_submit(mlfma_server s, mlfma_handle h, int op, int dtype, long long nrhs, const void *x,
                        long long ldx, void *y, long long ldy, void *hip_stream, long long *ticket)
{
    g_last_error.clear();
    if (!s || !h || !ticket) return fail(Error(MLFMA_ERR_ARG, "NULL argument"));
    if (!h->near_ready) return fail(Error(MLFMA_ERR_STATE, "mlfma_precompute_nearfield has not been called"));
    if (op != MLFMA_OP_C && op != MLFMA_OP_EM) return fail(Error(MLFMA_ERR_ARG, "unknown op"));
    if (dtype != MLFMA_C128 && dtype != MLFMA_C64) return fail(Error(MLFMA_ERR_ARG, "unknown dtype"));
    if (h->device != s->device) return fail(Error(MLFMA_ERR_ARG, "geometry lives on another device"));
    const long long N2 = 2LL * h->r.n;
    if (nrhs < 1 || nrhs > (1 << 16) || !x || !y || ldx < N2 || ldy < N2)
        return fail(Error(MLFMA_ERR_ARG, "bad nrhs, pointer or leading dimension"));
    hipEvent_t ready = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return fail(Error(MLFMA_ERR_STATE, "the server is being destroyed"));
        if (!s->free_events.empty()) {
            ready = s->free_events.back();
            s->free_events.pop_back();
        }
    }
    try {
        DeviceGuard g(s->device);
        if (!ready) HIPCHK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
        HIPCHK(hipEventRecord(ready, (hipStream_t)hip_stream));
    } catch (const Error &e) {
        if (ready) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->free_events.push_back(ready);
        }
        return fail(e);
    }
    Request *r = new Request();
    r->ready = ready;
    r->h = h;
    r->op = op;
    r->dtype = dtype;
    r->nrhs = (int)nrhs;
    r->x = x;
    r->y = y;
    r->ldx = ldx;
    r->ldy = ldy;
    r->t_submit = Clock::now();
    long long t = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            s->free_events.push_back(ready);
            delete r;
            return fail(Error(MLFMA_ERR_STATE, "the server is being destroyed"));
        }
        t = r->ticket = s->next_ticket++;
        s->reqs[r->ticket] = r;
        s->queue.push_back(r);
    }
    s->cv_sched.notify_all();
    *ticket = t;
    return MLFMA_OK;
}

int mlfma_server_wait(mlfma_server s, long long ticket, double timeout_s, double *latency_s, int *batch_rhs)
{
    g_last_error.clear();
    if (!s) return fail(Error(MLFMA_ERR_ARG, "NULL server"));
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(Error(MLFMA_ERR_ARG, "unknown ticket"));
    Request *r = it->second;
    auto pred = [&] { return r->state == 2 || r->state < 0; };
    s->waiters++;
    bool finished = true;
    if (timeout_s < 0) s->cv_done.wait(lk, pred);
    else finished = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred);
    if (!finished) {
        s->waiters--;
        s->cv_done.notify_all();
        lk.unlock();
        return fail(Error(MLFMA_ERR_STATE, "request not finished within the timeout"));
    }
    const int st = r->state;
    if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    if (batch_rhs) *batch_rhs = r->batch_rhs;
    s->reqs.erase(it);
    const std::string why = r->error;
    if (r->ready) s->free_events.push_back(r->ready);
    delete r;
    s->waiters--;
    s->cv_done.notify_all();     // mlfma_server_destroy waits for the last waiter to leave
    lk.unlock();
    if (st < 0) return fail(Error(st, why.empty() ? "request failed" : why));
    return MLFMA_OK;
}

int mlfma_server_stats(mlfma_server s, long long out[5])
{
    if (!s || !out) return fail(Error(MLFMA_ERR_ARG, "NULL argument"));
    std::lock_guard<std::mutex> lk(s->mu);
    out[0] = s->launches;
    out[1] = s->batched_requests;
    out[2] = (long long)s->arena_total;
    out[3] = (long long)s->queue.size();
    out[4] = s->graph_captures;
    return MLFMA_OK;
}

int mlfma_server_destroy(mlfma_server s)
{
    if (!s) return MLFMA_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_sched.notify_all();
    s->cv_done.notify_all();
    if (s->sched.joinable()) s->sched.join();
    if (s->poll.joinable()) s->poll.join();
    {
        DeviceGuard g(s->device);
        for (auto &sl : s->slots) {
            if (sl.stream) (void)hipStreamSynchronize(sl.stream);
            clear_graphs(sl);
            if (sl.arena) (void)hipFree(sl.arena);
            if (sl.xb) (void)hipFree(sl.xb);
            if (sl.yb) (void)hipFree(sl.yb);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        if (s->capture) (void)hipStreamDestroy(s->capture);
    }
    {
        // requests still queued or running fail; threads waiting for them
        // return before the server is freed
        std::unique_lock<std::mutex> lk(s->mu);
        for (auto &kv : s->reqs)
            if (kv.second->state == 0 || kv.second->state == 1) {
                kv.second->error = "the server was destroyed before the request finished";
                kv.second->state = MLFMA_ERR_STATE;
                kv.second->t_done = Clock::now();
            }
        s->cv_done.notify_all();
        s->cv_done.wait(lk, [&] { return s->waiters == 0; });
    }
    {
        DeviceGuard g(s->device);
        for (auto &kv : s->reqs) {
            if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
            delete kv.second;
        }
        for (auto e : s->free_events) (void)hipEventDestroy(e);
    }
    delete s;
    return MLFMA_OK;
}

}  // extern "C"
