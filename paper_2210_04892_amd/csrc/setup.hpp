// Host-side geometry, octree and k-space set-up of the MLFMA matvec.
#pragma once
#include <complex>
#include <cstdint>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

namespace mlfma {

using cdouble = std::complex<double>;

// error carried from the set-up code to the C boundary
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

struct Surface {
    int nv = 0, nt = 0;
    std::vector<double> v;      // nv x 3
    std::vector<int> t;         // nt x 3
    std::vector<double> area;   // nt
    std::vector<double> nrm;    // nt x 3, unit outward normal
};

// RWG functions in the canonical (user) order.
struct RwgTable {
    int n = 0;
    std::vector<int> a, b;          // edge endpoints, a < b
    std::vector<int> tri[2];        // T+ and T-
    std::vector<int> loc[2];        // local vertex index of the free vertex in T+ / T-
    std::vector<double> coef[2];    // +l/(2A+) and -l/(2A-): f = coef * (r - p)
    std::vector<int> tri_rwg;       // nt x 3: RWG on the edge opposite local vertex j
};

// One octree level (only non-empty boxes are kept, in Morton order).
struct Level {
    int lev = 0;
    double a = 0;                   // box edge
    int nbox = 0;
    std::vector<int> coord;         // nbox x 3 integer box coordinates
    std::vector<double> centre;     // nbox x 3
    std::vector<int> parent;        // index into the level above (lev - 1)
    std::vector<int> child_oct;     // octant of this box inside its parent (0..7)
    // k-space sampling (levels >= 2)
    int L = 0, nth = 0, nph = 0, K = 0;
    std::vector<double> ct, wt;     // cos(theta) Gauss-Legendre nodes/weights, theta ascending
    // interaction list (levels >= 2), CSR over boxes: source box and offset id
    std::vector<int> il_start, il_box, il_off;
};

// Sparse matrix with real weights in CSR form (rows -> (column, weight)).
struct Csr {
    int rows = 0, cols = 0;
    std::vector<int> start, col;
    std::vector<double> w;
};

struct Tree {
    int levels = 0;                 // root = 0 .. leaf = levels - 1
    double leaf = 0, side = 0, origin[3] = {0, 0, 0};
    std::vector<int> perm;          // internal index -> user RWG index (Morton order)
    std::vector<int> iperm;         // user RWG index -> internal index
    std::vector<int> leaf_of;       // internal index -> leaf box
    std::vector<Level> lv;          // per level
    std::vector<int> box_start;     // leaf boxes: RWG ranges (nbox_leaf + 1)
    std::vector<int> near_start, near_box;   // leaf near lists (Chebyshev distance <= 1, incl. self)
    // interpolation stencils for the step from level l+1 (child) to l (parent)
    std::vector<Csr> agg_theta, agg_phi, dis_phi, dis_theta;   // indexed by parent level l
};

// Interaction lists regrouped for the tiled translation.  A tile is a run of
// consecutive target boxes (Morton order) inside one 4x4x4 block of the level;
// the union of their source boxes is split into batches of at most `smax`
// boxes, each small enough to be staged whole in LDS.  For batch b and the
// tile's j-th target, ent[row[bat_row[b] + j] .. row[bat_row[b] + j + 1]) are
// the target's interaction-list entries whose source lies in the batch, each
// packed as ((offset id * K) << 8) | (position of the source inside the
// batch), K = the level's samples (so the first field is the operator's row
// start in the 343 x K table).
struct TransTiles {
    std::vector<int> tile_tgt;  // ntile + 1: first target box of each tile
    std::vector<int> tile_bat;  // ntile + 1: first batch of each tile
    std::vector<int> bat_src;   // nbatch + 1: first entry of each batch in src
    std::vector<int> src;       // source boxes of every batch
    std::vector<int> bat_row;   // nbatch: position of the batch's row pointers in row
    std::vector<int> row;       // row pointers into ent
    std::vector<int> ent;       // packed entries
};
void build_translation_tiles(const Level &L, int smax, int tmax, TransTiles &t);

// Interaction lists regrouped by sibling groups for the register-blocked
// translation.  A group is a run of at most `tg` consecutive boxes (Morton
// order) with one parent; siblings share most of their interaction lists
// (children of the parent's neighbours), so every source of the group's
// union is read once and applied to all of the group's targets.  Group g
// has targets first[g] .. first[g] + count[g] - 1 and source records
// rec_start[g] .. rec_start[g + 1] - 1; record r is source box src[r] and,
// for target slot j < tg, offset id off[r * tg + j] (0..342, the 7 x 7 x 7
// window of the operator table) or -1 when the source is not in that
// target's interaction list.  Records are sorted by source box.  With
// merge, a whole sibling set also takes the following whole sibling sets
// (consecutive in Morton order) while the group has room: fewer groups,
// more targets each, sources shared by more of them.
struct GroupTiles {
    int tg = 0;
    std::vector<int> first, count, rec_start, src, off;
};
void build_group_tiles(const Level &L, int tg, GroupTiles &g, bool merge = false);

// Theta-row chunks for a level step done in LDS.  `theta` is the step's theta
// stencil, whose rows are (output theta row) * nph + phi column and whose
// columns are (input theta row) * nph + phi column.  Output theta rows are cut
// into chunks of `rows`; win[2 c], win[2 c + 1] bound the input theta rows
// chunk c needs and wrows is the widest window.  The largest rows <= rows0
// whose footprint lds(wrows, rows) is at most lds_max is taken (rows = 0 if
// none is).
struct ChunkPlan {
    int rows = 0, nchunk = 0, wrows = 0;
    std::vector<int> win;
};
void plan_theta_chunks(const Csr &theta, int n_out, int nph, int rows0,
                       const std::function<size_t(int, int)> &lds, size_t lds_max, ChunkPlan &pl);

// The disaggregation stencils of one step in separable form: the transposed
// phi stencil is the same for every parent theta row up to the row's
// quadrature weight, and the transposed theta stencil of a child theta row is
// the same for every phi column up to the half-turn shift of the pole
// extension.  Rows are padded with zero weights to a common width.
//   intermediate(ip, j) = rowf[ip] * sum_t phi_w[j][t] * parent(ip, phi_col[j][t])
//   child(ic, j) = sum_t th_w[ic][t] * intermediate(th_row[ic][t], (j + th_sh[ic][t]) mod nph_c)
struct SepStencil {
    int tphi = 0, tth = 0;
    std::vector<int> phi_col, th_row, th_sh;
    std::vector<double> phi_w, rowf, th_w;
};
// false when the step's stencils are not separable in this way
bool separable_disaggregation(const Level &parent, const Level &child, const Csr &dph, const Csr &dth,
                              SepStencil &out);
// The aggregation stencils of one step in the same form (rowf empty), taps in
// the stencils' own order: the theta stencil of a parent theta row is the
// same for every child phi column up to the half-turn shift, and the phi
// stencil of a parent phi column the same for every parent theta row:
//   intermediate(ip, j) = sum_t th_w[ip][t] * child(th_row[ip][t], (j + th_sh[ip][t]) mod nph_c)
//   parent(ip, jp) = sum_t phi_w[jp][t] * intermediate(ip, phi_col[jp][t])
bool separable_aggregation(const Level &parent, const Level &child, const Csr &aph, const Csr &ath,
                           SepStencil &out);

void build_surface(Surface &s, const double *verts, long long nv, const int *tris, long long nt);
void build_rwg(const Surface &s, RwgTable &r);
void build_tree(const Surface &s, const RwgTable &r, double k, double leaf, int digits, int interp_order,
                int leaf_extra_L, Tree &tr);
void check_touching_near(const Surface &s, const RwgTable &r, const Tree &tr);

// translation operator sum for one level and offset, at the level's samples
void translation_table(double k, int L, const double X[3], const std::vector<double> &khat,
                       std::vector<cdouble> &out);
// unit vectors of the level's samples, sample index = itheta * nph + iphi
void level_directions(const Level &l, std::vector<double> &khat);
// truncation rule
int truncation(double k, double box_edge, int digits);
// Gauss-Legendre nodes/weights on [-1, 1], ascending
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);

}  // namespace mlfma
