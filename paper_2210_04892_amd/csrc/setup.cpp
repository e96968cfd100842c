// Host-side set-up: surface checks, RWG table, octree over RWG centres,
// per-level k-space sampling, Lagrange interpolation stencils and the
// diagonal translation operators of the multilevel plane-wave expansion.
#include "setup.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>
#include <unordered_map>

#include "../../include/mlfma.h"

namespace mlfma {

static inline void sub3(const double *a, const double *b, double *o)
{
    o[0] = a[0] - b[0];
    o[1] = a[1] - b[1];
    o[2] = a[2] - b[2];
}
static inline void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

void build_surface(Surface &s, const double *verts, long long nv, const int *tris, long long nt)
{
    if (!verts || !tris || nv < 4 || nt < 4 || nv > (1LL << 30) || nt > (1LL << 30))
        throw Error(MLFMA_ERR_ARG, "mesh arrays missing or sizes out of range");
    s.nv = (int)nv;
    s.nt = (int)nt;
    s.v.assign(verts, verts + 3 * nv);
    s.t.assign(tris, tris + 3 * nt);
    s.area.resize(nt);
    s.nrm.resize(3 * nt);
    double maxa = 0;
    for (int i = 0; i < s.nt; i++) {
        for (int c = 0; c < 3; c++)
            if (s.t[3 * i + c] < 0 || s.t[3 * i + c] >= s.nv)
                throw Error(MLFMA_ERR_MESH, "triangle " + std::to_string(i) + " has a vertex index out of range");
        const double *p0 = &s.v[3 * s.t[3 * i]], *p1 = &s.v[3 * s.t[3 * i + 1]], *p2 = &s.v[3 * s.t[3 * i + 2]];
        double e1[3], e2[3], c[3];
        sub3(p1, p0, e1);
        sub3(p2, p0, e2);
        cross3(e1, e2, c);
        double n2 = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        s.area[i] = 0.5 * n2;
        maxa = std::max(maxa, s.area[i]);
        for (int k = 0; k < 3; k++) s.nrm[3 * i + k] = n2 > 0 ? c[k] / n2 : 0.0;
    }
    for (int i = 0; i < s.nt; i++)
        if (!(s.area[i] > 1e-12 * maxa))
            throw Error(MLFMA_ERR_MESH, "degenerate triangle " + std::to_string(i));
}

void build_rwg(const Surface &s, RwgTable &r)
{
    // every directed edge (p -> q) of a counter-clockwise triangle, keyed by
    // the undirected pair; a closed oriented 2-manifold uses each undirected
    // edge exactly twice, once in each direction
    struct Use { int tri, loc, dir; };
    std::unordered_map<uint64_t, std::vector<Use>> edges;
    edges.reserve(3 * (size_t)s.nt);
    for (int i = 0; i < s.nt; i++)
        for (int j = 0; j < 3; j++) {
            int p = s.t[3 * i + (j + 1) % 3], q = s.t[3 * i + (j + 2) % 3];
            int a = std::min(p, q), b = std::max(p, q);
            edges[((uint64_t)a << 32) | (uint32_t)b].push_back({i, j, p < q ? 1 : -1});
        }
    std::vector<uint64_t> keys;
    keys.reserve(edges.size());
    for (auto &kv : edges) {
        if (kv.second.size() != 2)
            throw Error(MLFMA_ERR_MESH, "edge used by " + std::to_string(kv.second.size()) +
                                            " triangles: the surface must be a closed 2-manifold");
        if (kv.second[0].dir == kv.second[1].dir)
            throw Error(MLFMA_ERR_MESH, "neighbouring triangles with opposite orientation");
        keys.push_back(kv.first);
    }
    std::sort(keys.begin(), keys.end());
    r.n = (int)keys.size();
    r.a.resize(r.n);
    r.b.resize(r.n);
    for (int h = 0; h < 2; h++) {
        r.tri[h].resize(r.n);
        r.loc[h].resize(r.n);
        r.coef[h].resize(r.n);
    }
    r.tri_rwg.assign(3 * (size_t)s.nt, -1);
    for (int n = 0; n < r.n; n++) {
        uint64_t key = keys[n];
        r.a[n] = (int)(key >> 32);
        r.b[n] = (int)(key & 0xffffffffu);
        const double *va = &s.v[3 * r.a[n]], *vb = &s.v[3 * r.b[n]];
        double d[3];
        sub3(vb, va, d);
        double len = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        for (const Use &u : edges[key]) {
            int h = u.dir == 1 ? 0 : 1;       // a -> b counter-clockwise: T+
            r.tri[h][n] = u.tri;
            r.loc[h][n] = u.loc;
            r.coef[h][n] = (h == 0 ? 1.0 : -1.0) * len / (2.0 * s.area[u.tri]);
            r.tri_rwg[3 * (size_t)u.tri + u.loc] = n;
        }
    }
    // Disconnected scatterers may share the mesh (the BI equations then hold
    // on each closed surface, Sec. II-E remarks): every connected surface --
    // triangles joined through their RWGs -- must enclose a positive volume.
    std::vector<int> root(s.nt);
    for (int i = 0; i < s.nt; i++) root[i] = i;
    auto find = [&](int a) {
        while (root[a] != a) a = root[a] = root[root[a]];
        return a;
    };
    for (int n = 0; n < r.n; n++) {
        const int a = find(r.tri[0][n]), b = find(r.tri[1][n]);
        if (a != b) root[std::max(a, b)] = std::min(a, b);
    }
    std::vector<double> vol6(s.nt, 0.0);
    for (int i = 0; i < s.nt; i++) {
        const double *p0 = &s.v[3 * s.t[3 * i]], *p1 = &s.v[3 * s.t[3 * i + 1]], *p2 = &s.v[3 * s.t[3 * i + 2]];
        double pc[3];
        cross3(p1, p2, pc);
        vol6[find(i)] += p0[0] * pc[0] + p0[1] * pc[1] + p0[2] * pc[2];
    }
    for (int i = 0; i < s.nt; i++)
        if (root[i] == i && !(vol6[i] > 0))
            throw Error(MLFMA_ERR_MESH, "enclosed volume of a closed surface is not positive: triangles must be "
                                        "counter-clockwise seen from outside");
}

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; i++) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double pp = 1;
        for (int it = 0; it < 100; it++) {
            double p0 = 1, p1 = z;
            for (int l = 2; l <= n; l++) {
                double p2 = ((2.0 * l - 1) * z * p1 - (l - 1.0) * p0) / l;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) p0 = 1, p1 = z;
            pp = n * (z * p1 - p0) / (z * z - 1);
            double dz = p1 / pp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1, p1 = z;
        for (int l = 2; l <= n; l++) {
            double p2 = ((2.0 * l - 1) * z * p1 - (l - 1.0) * p0) / l;
            p0 = p1;
            p1 = p2;
        }
        pp = n * (z * p1 - p0) / (z * z - 1);
        x[n - 1 - i] = z;                     // ascending
        w[n - 1 - i] = 2.0 / ((1 - z * z) * pp * pp);
    }
}

int truncation(double k, double a, int digits)
{
    double kD = k * std::sqrt(3.0) * a;
    return (int)std::ceil(kD + 1.8 * std::pow((double)digits, 2.0 / 3.0) * std::cbrt(kD));
}

static uint64_t morton(int x, int y, int z)
{
    uint64_t c = 0;
    for (int b = 0; b < 21; b++) {
        c |= (uint64_t)((x >> b) & 1) << (3 * b + 2);
        c |= (uint64_t)((y >> b) & 1) << (3 * b + 1);
        c |= (uint64_t)((z >> b) & 1) << (3 * b);
    }
    return c;
}

static uint64_t coord_key(int x, int y, int z)
{
    return ((uint64_t)(uint32_t)(x + 1) << 42) | ((uint64_t)(uint32_t)(y + 1) << 21) | (uint64_t)(uint32_t)(z + 1);
}

// Lagrange weights of the nodes xs at the point x0
static void lagrange(const std::vector<double> &xs, double x0, std::vector<double> &w)
{
    int p = (int)xs.size();
    w.assign(p, 1.0);
    for (int s = 0; s < p; s++)
        for (int t = 0; t < p; t++)
            if (t != s) w[s] *= (x0 - xs[t]) / (xs[s] - xs[t]);
}

static Csr transpose(const Csr &a)
{
    Csr t;
    t.rows = a.cols;
    t.cols = a.rows;
    t.start.assign(t.rows + 1, 0);
    for (int c : a.col) t.start[c + 1]++;
    for (int i = 0; i < t.rows; i++) t.start[i + 1] += t.start[i];
    t.col.resize(a.col.size());
    t.w.resize(a.w.size());
    std::vector<int> fill(t.start.begin(), t.start.end() - 1);
    for (int r = 0; r < a.rows; r++)
        for (int e = a.start[r]; e < a.start[r + 1]; e++) {
            int pos = fill[a.col[e]]++;
            t.col[pos] = r;
            t.w[pos] = a.w[e];
        }
    return t;
}

// Stencils between child level c and parent level p (see Tree).
static void build_stencils(const Level &c, const Level &p, int order, Csr &ath, Csr &aph, Csr &dph, Csr &dth)
{
    // child theta nodes extended across both poles: (-theta, phi + pi) and
    // (2 pi - theta, phi + pi) are the same directions as (theta, phi); the
    // theta and phi unit vectors change sign there, so both components flip
    struct Node { double th; int idx; int refl; };
    std::vector<Node> ext;
    for (int i = 0; i < c.nth; i++) {
        double th = std::acos(c.ct[i]);
        ext.push_back({th, i, 0});
        ext.push_back({-th, i, 1});
        ext.push_back({2 * M_PI - th, i, 1});
    }
    std::sort(ext.begin(), ext.end(), [](const Node &x, const Node &y) { return x.th < y.th; });
    const int half = c.nph / 2;
    ath.rows = p.nth * c.nph;
    ath.cols = c.K;
    ath.start.assign(1, 0);
    std::vector<double> xs, w;
    for (int ip = 0; ip < p.nth; ip++) {
        double th = std::acos(p.ct[ip]);
        // window of `order` consecutive extended nodes closest to th
        int pos = (int)(std::lower_bound(ext.begin(), ext.end(), th, [](const Node &n, double v) { return n.th < v; }) -
                        ext.begin());
        int lo = pos, hi = pos;   // [lo, hi)
        while (hi - lo < order) {
            bool take_lo = lo > 0 && (hi >= (int)ext.size() || th - ext[lo - 1].th <= ext[hi].th - th);
            if (take_lo) lo--; else hi++;
        }
        xs.clear();
        for (int s = lo; s < hi; s++) xs.push_back(ext[s].th);
        lagrange(xs, th, w);
        for (int jc = 0; jc < c.nph; jc++) {
            for (int s = lo; s < hi; s++) {
                const Node &n = ext[s];
                int jj = n.refl ? (jc + half) % c.nph : jc;
                ath.col.push_back(n.idx * c.nph + jj);
                ath.w.push_back(n.refl ? -w[s - lo] : w[s - lo]);
            }
            ath.start.push_back((int)ath.col.size());
        }
    }
    aph.rows = p.K;
    aph.cols = p.nth * c.nph;
    aph.start.assign(1, 0);
    const double dc = 2 * M_PI / c.nph;
    for (int ip = 0; ip < p.nth; ip++)
        for (int jp = 0; jp < p.nph; jp++) {
            double ph = 2 * M_PI * jp / p.nph;
            int j0 = (int)std::floor(ph / dc) - (order / 2 - 1);
            xs.clear();
            for (int s = 0; s < order; s++) xs.push_back((j0 + s) * dc);
            lagrange(xs, ph, w);
            for (int s = 0; s < order; s++) {
                int j = ((j0 + s) % c.nph + c.nph) % c.nph;
                aph.col.push_back(ip * c.nph + j);
                aph.w.push_back(w[s]);
            }
            aph.start.push_back((int)aph.col.size());
        }
    // anterpolation: W_c^-1 A_theta^T A_phi^T W_p (quadrature weights W)
    dph = transpose(aph);
    for (int r = 0; r < dph.rows; r++)
        for (int e = dph.start[r]; e < dph.start[r + 1]; e++) {
            int kp = dph.col[e];
            dph.w[e] *= p.wt[kp / p.nph] * (2 * M_PI / p.nph);
        }
    dth = transpose(ath);
    for (int r = 0; r < dth.rows; r++)
        for (int e = dth.start[r]; e < dth.start[r + 1]; e++)
            dth.w[e] /= c.wt[r / c.nph] * (2 * M_PI / c.nph);
}

void build_tree(const Surface &s, const RwgTable &r, double k, double leaf, int digits, int order, int leaf_extra_L,
                Tree &tr)
{
    if (!(leaf > 0) || !(k > 0) || digits < 1 || order < 2 || order > 16 || leaf_extra_L < 0)
        throw Error(MLFMA_ERR_ARG, "invalid wavenumber, leaf size, digits or interpolation order");
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int i = 0; i < s.nv; i++)
        for (int c = 0; c < 3; c++) {
            lo[c] = std::min(lo[c], s.v[3 * i + c]);
            hi[c] = std::max(hi[c], s.v[3 * i + c]);
        }
    double extent = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    int levels = (int)std::ceil(std::log2(extent / leaf)) + 1;
    if (levels < 1) levels = 1;
    if (levels > 20) throw Error(MLFMA_ERR_ARG, "too many octree levels");
    tr.levels = levels;
    tr.leaf = leaf;
    tr.side = leaf * std::ldexp(1.0, levels - 1);
    const int nb = 1 << (levels - 1);
    for (int c = 0; c < 3; c++) tr.origin[c] = 0.5 * (lo[c] + hi[c]) - 0.5 * tr.side;
    // leaf box of every RWG centre (edge midpoint)
    const int N = r.n;
    std::vector<int> lc(3 * (size_t)N);
    std::vector<uint64_t> code(N);
    for (int n = 0; n < N; n++) {
        for (int c = 0; c < 3; c++) {
            double centre = 0.5 * (lo[c] + hi[c]);
            double origin = centre - 0.5 * tr.side;
            double mid = 0.5 * (s.v[3 * r.a[n] + c] + s.v[3 * r.b[n] + c]);
            int b = (int)std::floor((mid - origin) / leaf);
            lc[3 * n + c] = std::min(std::max(b, 0), nb - 1);
        }
        code[n] = morton(lc[3 * n], lc[3 * n + 1], lc[3 * n + 2]);
    }
    tr.perm.resize(N);
    std::iota(tr.perm.begin(), tr.perm.end(), 0);
    std::stable_sort(tr.perm.begin(), tr.perm.end(), [&](int x, int y) { return code[x] < code[y]; });
    tr.iperm.resize(N);
    for (int i = 0; i < N; i++) tr.iperm[tr.perm[i]] = i;
    // boxes of every level, leaf upwards
    tr.lv.assign(levels, Level());
    const int leafl = levels - 1;
    std::vector<uint64_t> prev_codes;   // codes of the level below
    for (int l = leafl; l >= 0; l--) {
        Level &L = tr.lv[l];
        L.lev = l;
        L.a = tr.side / std::ldexp(1.0, l);
        int sh = leafl - l;
        std::vector<uint64_t> codes;
        for (int i = 0; i < N; i++) {
            uint64_t cc = code[tr.perm[i]] >> (3 * sh);
            if (codes.empty() || codes.back() != cc) codes.push_back(cc);
        }
        L.nbox = (int)codes.size();
        L.coord.resize(3 * (size_t)L.nbox);
        L.centre.resize(3 * (size_t)L.nbox);
        for (int b = 0; b < L.nbox; b++) {
            // any RWG of the box gives the coordinates
            int x = 0, y = 0, z = 0;
            uint64_t cc = codes[b];
            for (int bit = 0; bit < 21; bit++) {
                x |= (int)((cc >> (3 * bit + 2)) & 1) << bit;
                y |= (int)((cc >> (3 * bit + 1)) & 1) << bit;
                z |= (int)((cc >> (3 * bit)) & 1) << bit;
            }
            L.coord[3 * b] = x;
            L.coord[3 * b + 1] = y;
            L.coord[3 * b + 2] = z;
            for (int c = 0; c < 3; c++) L.centre[3 * b + c] = tr.origin[c] + (L.coord[3 * b + c] + 0.5) * L.a;
        }
        if (l == leafl) {
            tr.box_start.assign(1, 0);
            tr.leaf_of.resize(N);
            int b = 0;
            for (int i = 0; i < N; i++) {
                uint64_t cc = code[tr.perm[i]];
                while (codes[b] != cc) {
                    tr.box_start.push_back(i);
                    b++;
                }
                tr.leaf_of[i] = b;
            }
            tr.box_start.push_back(N);
        }
        if (l < leafl) {
            Level &C = tr.lv[l + 1];
            C.parent.resize(C.nbox);
            C.child_oct.resize(C.nbox);
            int pb = 0;
            for (int b = 0; b < C.nbox; b++) {
                uint64_t pc = prev_codes[b] >> 3;
                while (codes[pb] != pc) pb++;
                C.parent[b] = pb;
                C.child_oct[b] = (int)(prev_codes[b] & 7);
            }
        }
        prev_codes.swap(codes);
    }
    // near lists at the leaf level and interaction lists at levels >= 2
    std::vector<std::unordered_map<uint64_t, int>> where(levels);
    for (int l = 0; l < levels; l++) {
        Level &L = tr.lv[l];
        for (int b = 0; b < L.nbox; b++)
            where[l][coord_key(L.coord[3 * b], L.coord[3 * b + 1], L.coord[3 * b + 2])] = b;
    }
    {
        Level &L = tr.lv[leafl];
        tr.near_start.assign(1, 0);
        for (int b = 0; b < L.nbox; b++) {
            std::vector<int> lst;
            for (int dx = -1; dx <= 1; dx++)
                for (int dy = -1; dy <= 1; dy++)
                    for (int dz = -1; dz <= 1; dz++) {
                        auto it = where[leafl].find(coord_key(L.coord[3 * b] + dx, L.coord[3 * b + 1] + dy,
                                                              L.coord[3 * b + 2] + dz));
                        if (it != where[leafl].end()) lst.push_back(it->second);
                    }
            std::sort(lst.begin(), lst.end());
            tr.near_box.insert(tr.near_box.end(), lst.begin(), lst.end());
            tr.near_start.push_back((int)tr.near_box.size());
        }
    }
    for (int l = 2; l < levels; l++) {
        Level &L = tr.lv[l];
        Level &P = tr.lv[l - 1];
        // children of every parent box
        std::vector<std::vector<int>> kids(P.nbox);
        for (int b = 0; b < L.nbox; b++) kids[L.parent[b]].push_back(b);
        L.il_start.assign(1, 0);
        for (int b = 0; b < L.nbox; b++) {
            int pbx = L.parent[b];
            std::vector<std::pair<int, int>> lst;
            for (int dx = -1; dx <= 1; dx++)
                for (int dy = -1; dy <= 1; dy++)
                    for (int dz = -1; dz <= 1; dz++) {
                        auto it = where[l - 1].find(coord_key(P.coord[3 * pbx] + dx, P.coord[3 * pbx + 1] + dy,
                                                              P.coord[3 * pbx + 2] + dz));
                        if (it == where[l - 1].end()) continue;
                        for (int src : kids[it->second]) {
                            int ox = L.coord[3 * b] - L.coord[3 * src];
                            int oy = L.coord[3 * b + 1] - L.coord[3 * src + 1];
                            int oz = L.coord[3 * b + 2] - L.coord[3 * src + 2];
                            if (std::max(std::abs(ox), std::max(std::abs(oy), std::abs(oz))) < 2) continue;
                            lst.push_back({src, (ox + 3) * 49 + (oy + 3) * 7 + (oz + 3)});
                        }
                    }
            std::sort(lst.begin(), lst.end());
            for (auto &pr : lst) {
                L.il_box.push_back(pr.first);
                L.il_off.push_back(pr.second);
            }
            L.il_start.push_back((int)L.il_box.size());
        }
    }
    // k-space sampling: L+1 Gauss-Legendre nodes in cos(theta), 2L+2 azimuths
    for (int l = 2; l < levels; l++) {
        Level &L = tr.lv[l];
        L.L = truncation(k, L.a, digits) + (l == leafl ? leaf_extra_L : 0);
        L.nth = L.L + 1;
        L.nph = 2 * L.L + 2;
        L.K = L.nth * L.nph;
        std::vector<double> x, w;
        gauss_legendre(L.nth, x, w);
        L.ct.resize(L.nth);
        L.wt.resize(L.nth);
        for (int i = 0; i < L.nth; i++) {       // theta ascending = cos(theta) descending
            L.ct[i] = x[L.nth - 1 - i];
            L.wt[i] = w[L.nth - 1 - i];
        }
    }
    tr.agg_theta.assign(levels, Csr());
    tr.agg_phi.assign(levels, Csr());
    tr.dis_phi.assign(levels, Csr());
    tr.dis_theta.assign(levels, Csr());
    for (int l = 2; l + 1 < levels; l++) {
        const Level &C = tr.lv[l + 1];
        if (order > C.nph || order > 3 * C.nth)
            throw Error(MLFMA_ERR_ARG, "interpolation order exceeds the samples of level " + std::to_string(l + 1));
        build_stencils(C, tr.lv[l], order, tr.agg_theta[l], tr.agg_phi[l], tr.dis_phi[l], tr.dis_theta[l]);
        // the forward stencils have exactly `order` taps per row (the fixed-size kernels rely on it)
        for (const Csr *a : {&tr.agg_theta[l], &tr.agg_phi[l]})
            for (int r = 0; r < a->rows; r++)
                if (a->start[r + 1] - a->start[r] != order)
                    throw Error(MLFMA_ERR_ARG, "interpolation stencil with a wrong number of taps");
    }
}

void check_touching_near(const Surface &s, const RwgTable &r, const Tree &tr)
{
    const int leafl = tr.levels - 1;
    const Level &L = tr.lv[leafl];
    std::vector<std::vector<int>> vt(s.nv);
    for (int i = 0; i < s.nt; i++)
        for (int c = 0; c < 3; c++) vt[s.t[3 * i + c]].push_back(i);
    auto box_of = [&](int user) { return tr.leaf_of[tr.iperm[user]]; };
    for (int v = 0; v < s.nv; v++)
        for (int t1 : vt[v])
            for (int t2 : vt[v])
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) {
                        int b1 = box_of(r.tri_rwg[3 * (size_t)t1 + i]), b2 = box_of(r.tri_rwg[3 * (size_t)t2 + j]);
                        for (int c = 0; c < 3; c++)
                            if (std::abs(L.coord[3 * b1 + c] - L.coord[3 * b2 + c]) > 1)
                                throw Error(MLFMA_ERR_TREE,
                                            "triangles sharing a vertex carry RWGs in non-adjacent leaf boxes: "
                                            "the leaf boxes are too small for this mesh");
                    }
}

void level_directions(const Level &l, std::vector<double> &khat)
{
    khat.resize(3 * (size_t)l.K);
    for (int i = 0; i < l.nth; i++) {
        double c = l.ct[i], sn = std::sqrt(std::max(0.0, 1 - c * c));
        for (int j = 0; j < l.nph; j++) {
            double ph = 2 * M_PI * j / l.nph;
            size_t q = (size_t)i * l.nph + j;
            khat[3 * q] = sn * std::cos(ph);
            khat[3 * q + 1] = sn * std::sin(ph);
            khat[3 * q + 2] = c;
        }
    }
}

void translation_table(double k, int L, const double X[3], const std::vector<double> &khat, std::vector<cdouble> &out)
{
    double R = std::sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
    double x = k * R;
    // spherical Bessel functions: y_l upward, j_l downward (Miller) normalised by j_0
    std::vector<double> jl(L + 1), yl(L + 1);
    yl[0] = -std::cos(x) / x;
    if (L >= 1) yl[1] = -std::cos(x) / (x * x) - std::sin(x) / x;
    for (int l = 1; l < L; l++) yl[l + 1] = (2 * l + 1) / x * yl[l] - yl[l - 1];
    int top = L + 30 + (int)x;
    double jp1 = 0, jc = 1e-300, scale_hit = 0;
    std::vector<double> tmp(top + 2, 0.0);
    tmp[top + 1] = jp1;
    tmp[top] = jc;
    for (int l = top; l >= 1; l--) {
        double jm1 = (2 * l + 1) / x * tmp[l] - tmp[l + 1];
        tmp[l - 1] = jm1;
        if (std::fabs(jm1) > 1e250) {     // rescale to avoid overflow
            for (int q = l - 1; q <= top + 1; q++) tmp[q] *= 1e-250;
        }
    }
    (void)scale_hit;
    // normalise with j_0 or j_1, whichever is larger (they never vanish together)
    const double j0 = std::sin(x) / x, j1 = std::sin(x) / (x * x) - std::cos(x) / x;
    double norm = std::fabs(j0) >= std::fabs(j1) ? j0 / tmp[0] : j1 / tmp[1];
    for (int l = 0; l <= L; l++) jl[l] = tmp[l] * norm;
    std::vector<cdouble> coef(L + 1);
    const cdouble mj[4] = {1.0, cdouble(0, -1), -1.0, cdouble(0, 1)};   // (-j)^l
    for (int l = 0; l <= L; l++) coef[l] = mj[l % 4] * (2.0 * l + 1) * cdouble(jl[l], -yl[l]);
    size_t nk = khat.size() / 3;
    out.resize(nk);
    for (size_t q = 0; q < nk; q++) {
        double c = (khat[3 * q] * X[0] + khat[3 * q + 1] * X[1] + khat[3 * q + 2] * X[2]) / R;
        double p0 = 1, p1 = c;
        cdouble acc = coef[0] * p0;
        if (L >= 1) acc += coef[1] * p1;
        for (int l = 1; l < L; l++) {
            double p2 = ((2 * l + 1) * c * p1 - l * p0) / (l + 1);
            p0 = p1;
            p1 = p2;
            acc += coef[l + 1] * p1;
        }
        out[q] = acc;
    }
}



// ---------------------------------------------------------- translation tiles
void build_translation_tiles(const Level &L, int smax, int tmax, TransTiles &t)
{
    if (smax < 1 || smax > 255 || tmax < 1) throw Error(MLFMA_ERR_ARG, "bad translation tile limits");
    if (343LL * L.K >= (1LL << 23)) throw Error(MLFMA_ERR_ARG, "too many samples for the translation tables");
    t = TransTiles();
    t.tile_tgt.push_back(0);
    t.tile_bat.push_back(0);
    t.bat_src.push_back(0);
    std::vector<int> uni;
    int A0 = 0;
    while (A0 < L.nbox) {
        // the tile: consecutive targets of one 4x4x4 block, at most tmax of them
        int A1 = A0 + 1;
        auto block = [&](int A) {
            return std::array<int, 3>{L.coord[3 * A] >> 2, L.coord[3 * A + 1] >> 2, L.coord[3 * A + 2] >> 2};
        };
        while (A1 < L.nbox && A1 - A0 < tmax && block(A1) == block(A0)) A1++;
        uni.clear();
        for (int A = A0; A < A1; A++)
            for (int e = L.il_start[A]; e < L.il_start[A + 1]; e++) uni.push_back(L.il_box[e]);
        std::sort(uni.begin(), uni.end());
        uni.erase(std::unique(uni.begin(), uni.end()), uni.end());
        const int nbat = std::max(1, (int)((uni.size() + smax - 1) / smax));
        for (int b = 0; b < nbat; b++) {
            const int s0 = b * smax, s1 = std::min((int)uni.size(), s0 + smax);
            t.src.insert(t.src.end(), uni.begin() + s0, uni.begin() + s1);
            t.bat_src.push_back((int)t.src.size());
            t.bat_row.push_back((int)t.row.size());
            for (int A = A0; A < A1; A++) {
                t.row.push_back((int)t.ent.size());
                for (int e = L.il_start[A]; e < L.il_start[A + 1]; e++) {
                    const int pos = (int)(std::lower_bound(uni.begin(), uni.end(), L.il_box[e]) - uni.begin());
                    if (pos >= s0 && pos < s1) t.ent.push_back(((L.il_off[e] * L.K) << 8) | (pos - s0));
                }
            }
            t.row.push_back((int)t.ent.size());
        }
        t.tile_tgt.push_back(A1);
        t.tile_bat.push_back((int)t.bat_row.size());
        A0 = A1;
    }
}

void build_group_tiles(const Level &L, int tg, GroupTiles &g, bool merge)
{
    if (tg < 1 || tg > 16) throw Error(MLFMA_ERR_ARG, "bad sibling group size");
    g = GroupTiles();
    g.tg = tg;
    g.rec_start.push_back(0);
    std::vector<std::pair<int, int>> ent;   // (source box, target slot * 512 + offset id)
    int A0 = 0;
    while (A0 < L.nbox) {
        int A1 = A0 + 1;
        while (A1 < L.nbox && A1 - A0 < tg && L.parent[A1] == L.parent[A0]) A1++;
        // with merge, a whole sibling set takes the following whole sibling
        // sets while the group has room
        const bool whole = (A1 >= L.nbox || L.parent[A1] != L.parent[A1 - 1]) &&
                           (A0 == 0 || L.parent[A0] != L.parent[A0 - 1]);
        while (merge && whole && A1 < L.nbox) {
            int B1 = A1 + 1;
            while (B1 < L.nbox && L.parent[B1] == L.parent[A1]) B1++;
            if (B1 - A0 > tg) break;
            A1 = B1;
        }
        ent.clear();
        for (int A = A0; A < A1; A++)
            for (int e = L.il_start[A]; e < L.il_start[A + 1]; e++) {
                if (L.il_off[e] < 0 || L.il_off[e] >= 343) throw Error(MLFMA_ERR_ARG, "bad interaction offset");
                ent.push_back({L.il_box[e], (A - A0) * 512 + L.il_off[e]});
            }
        std::sort(ent.begin(), ent.end());
        for (size_t i = 0; i < ent.size(); i++) {
            if (i == 0 || ent[i].first != ent[i - 1].first) {
                g.src.push_back(ent[i].first);
                g.off.insert(g.off.end(), tg, -1);
            }
            g.off[(g.src.size() - 1) * tg + ent[i].second / 512] = ent[i].second % 512;
        }
        g.first.push_back(A0);
        g.count.push_back(A1 - A0);
        g.rec_start.push_back((int)g.src.size());
        A0 = A1;
    }
}

// ------------------------------------------------------- level-step chunks
void plan_theta_chunks(const Csr &theta, int n_out, int nph, int rows0,
                       const std::function<size_t(int, int)> &lds, size_t lds_max, ChunkPlan &pl)
{
    pl = ChunkPlan();
    if (n_out < 1 || nph < 1 || theta.rows != n_out * nph) return;
    // input theta rows [lo, hi) of each output theta row
    std::vector<int> lo(n_out, 1 << 30), hi(n_out, -1);
    for (int o = 0; o < n_out; o++)
        for (int r = o * nph; r < (o + 1) * nph; r++)
            for (int e = theta.start[r]; e < theta.start[r + 1]; e++) {
                lo[o] = std::min(lo[o], theta.col[e] / nph);
                hi[o] = std::max(hi[o], theta.col[e] / nph + 1);
            }
    for (int rows = std::max(1, std::min(rows0, n_out)); rows >= 1; rows = rows > 1 ? rows / 2 : 0) {
        std::vector<int> win;
        int wrows = 0;
        for (int r0 = 0; r0 < n_out; r0 += rows) {
            int a = 1 << 30, b = -1;
            for (int o = r0; o < std::min(n_out, r0 + rows); o++) {
                a = std::min(a, lo[o]);
                b = std::max(b, hi[o]);
            }
            if (b < a) a = b = 0;
            win.push_back(a);
            win.push_back(b);
            wrows = std::max(wrows, b - a);
        }
        if (lds(wrows, rows) <= lds_max) {
            pl.rows = rows;
            pl.nchunk = (n_out + rows - 1) / rows;
            pl.wrows = wrows;
            pl.win = std::move(win);
            return;
        }
    }
}

// -------------------------------------------- separable aggregation stencils
bool separable_aggregation(const Level &P, const Level &C, const Csr &aph, const Csr &ath, SepStencil &o)
{
    o = SepStencil();
    const int nthp = P.nth, nphp = P.nph, nphc = C.nph;
    if (ath.rows != nthp * nphc || aph.rows != nthp * nphp) return false;
    auto same = [](double a, double b) { return a == b; };
    // theta: taps of (parent row ip, child column 0), then every column j
    for (int ip = 0; ip < nthp; ip++) o.tth = std::max(o.tth, ath.start[ip * nphc + 1] - ath.start[ip * nphc]);
    for (int jp = 0; jp < nphp; jp++) o.tphi = std::max(o.tphi, aph.start[jp + 1] - aph.start[jp]);
    if (o.tth < 1 || o.tphi < 1) return false;
    o.th_row.assign((size_t)nthp * o.tth, 0);
    o.th_sh.assign((size_t)nthp * o.tth, 0);
    o.th_w.assign((size_t)nthp * o.tth, 0.0);
    for (int ip = 0; ip < nthp; ip++) {
        const int r0 = ip * nphc, n0 = ath.start[r0 + 1] - ath.start[r0];
        if (n0 != o.tth) return false;
        for (int t = 0; t < n0; t++) {
            const int e = ath.start[r0] + t;
            o.th_row[(size_t)ip * o.tth + t] = ath.col[e] / nphc;
            o.th_sh[(size_t)ip * o.tth + t] = ath.col[e] % nphc;
            o.th_w[(size_t)ip * o.tth + t] = ath.w[e];
        }
        for (int j = 1; j < nphc; j++) {
            const int r = ip * nphc + j;
            if (ath.start[r + 1] - ath.start[r] != n0) return false;
            for (int t = 0; t < n0; t++) {
                const int e = ath.start[r] + t;
                const int row = ath.col[e] / nphc, sh = ((ath.col[e] % nphc - j) % nphc + nphc) % nphc;
                if (row != o.th_row[(size_t)ip * o.tth + t] || sh != o.th_sh[(size_t)ip * o.tth + t] ||
                    !same(ath.w[e], o.th_w[(size_t)ip * o.tth + t]))
                    return false;
            }
        }
    }
    // phi: taps of (parent row 0, parent column jp), then every row ip
    o.phi_col.assign((size_t)nphp * o.tphi, 0);
    o.phi_w.assign((size_t)nphp * o.tphi, 0.0);
    for (int jp = 0; jp < nphp; jp++) {
        const int n0 = aph.start[jp + 1] - aph.start[jp];
        if (n0 != o.tphi) return false;
        for (int t = 0; t < n0; t++) {
            const int e = aph.start[jp] + t;
            o.phi_col[(size_t)jp * o.tphi + t] = aph.col[e];
            o.phi_w[(size_t)jp * o.tphi + t] = aph.w[e];
        }
        for (int ip = 1; ip < nthp; ip++) {
            const int r = ip * nphp + jp;
            if (aph.start[r + 1] - aph.start[r] != n0) return false;
            for (int t = 0; t < n0; t++) {
                const int e = aph.start[r] + t;
                if (aph.col[e] != ip * nphc + o.phi_col[(size_t)jp * o.tphi + t] ||
                    !same(aph.w[e], o.phi_w[(size_t)jp * o.tphi + t]))
                    return false;
            }
        }
    }
    return true;
}

// ------------------------------------------ separable disaggregation stencils
bool separable_disaggregation(const Level &P, const Level &C, const Csr &dph, const Csr &dth, SepStencil &o)
{
    o = SepStencil();
    const int nthp = P.nth, nphp = P.nph, nthc = C.nth, nphc = C.nph;
    if (dph.rows != nthp * nphc || dth.rows != nthc * nphc) return false;
    auto close = [](double a, double b) { return std::abs(a - b) <= 1e-12 * std::max(1.0, std::max(std::abs(a), std::abs(b))); };
    // phi: row factor = the parent row's quadrature weight
    o.rowf.resize(nthp);
    for (int ip = 0; ip < nthp; ip++) o.rowf[ip] = P.wt[ip] * (2 * M_PI / nphp);
    for (int j = 0; j < nphc; j++) o.tphi = std::max(o.tphi, dph.start[j + 1] - dph.start[j]);
    o.phi_col.assign((size_t)nphc * o.tphi, 0);
    o.phi_w.assign((size_t)nphc * o.tphi, 0.0);
    for (int j = 0; j < nphc; j++)
        for (int e = dph.start[j], t = 0; e < dph.start[j + 1]; e++, t++) {
            o.phi_col[(size_t)j * o.tphi + t] = dph.col[e];
            o.phi_w[(size_t)j * o.tphi + t] = dph.w[e] / o.rowf[0];
        }
    for (int ip = 1; ip < nthp; ip++)
        for (int j = 0; j < nphc; j++) {
            const int r = ip * nphc + j;
            if (dph.start[r + 1] - dph.start[r] != dph.start[j + 1] - dph.start[j]) return false;
            for (int e = dph.start[r], t = 0; e < dph.start[r + 1]; e++, t++)
                if (dph.col[e] != ip * nphp + o.phi_col[(size_t)j * o.tphi + t] ||
                    !close(dph.w[e], o.rowf[ip] * o.phi_w[(size_t)j * o.tphi + t]))
                    return false;
        }
    // theta: per child row, (parent row, column shift, weight), in a fixed order
    struct Tap { int row, sh; double w; };
    auto taps_of = [&](int ic, int j) {
        std::vector<Tap> v;
        const int r = ic * nphc + j;
        for (int e = dth.start[r]; e < dth.start[r + 1]; e++)
            v.push_back({dth.col[e] / nphc, ((dth.col[e] % nphc - j) % nphc + nphc) % nphc, dth.w[e]});
        std::sort(v.begin(), v.end(), [](const Tap &x, const Tap &y) { return x.row != y.row ? x.row < y.row : x.sh < y.sh; });
        return v;
    };
    std::vector<std::vector<Tap>> t0(nthc);
    for (int ic = 0; ic < nthc; ic++) {
        t0[ic] = taps_of(ic, 0);
        if (t0[ic].empty()) return false;
        o.tth = std::max(o.tth, (int)t0[ic].size());
    }
    o.th_row.assign((size_t)nthc * o.tth, 0);
    o.th_sh.assign((size_t)nthc * o.tth, 0);
    o.th_w.assign((size_t)nthc * o.tth, 0.0);
    for (int ic = 0; ic < nthc; ic++) {
        const int n0 = (int)t0[ic].size();
        for (int t = 0; t < o.tth; t++) {
            const Tap &x = t0[ic][std::min(t, n0 - 1)];
            o.th_row[(size_t)ic * o.tth + t] = x.row;
            o.th_sh[(size_t)ic * o.tth + t] = x.sh;
            o.th_w[(size_t)ic * o.tth + t] = t < n0 ? x.w : 0.0;
        }
        for (int j = 1; j < nphc; j++) {
            const std::vector<Tap> v = taps_of(ic, j);
            if ((int)v.size() != n0) return false;
            for (int t = 0; t < n0; t++)
                if (v[t].row != t0[ic][t].row || v[t].sh != t0[ic][t].sh || !close(v[t].w, t0[ic][t].w)) return false;
        }
    }
    return true;
}

}  // namespace mlfma
