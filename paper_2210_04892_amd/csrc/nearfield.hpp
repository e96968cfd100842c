// Set-up kernels (double precision): patterns and near-field blocks.
#pragma once
#include "device.hpp"

namespace mlfma {

// One ordered pair of triangles that share at least one vertex, with both
// triangles' vertices reordered so that the shared ones come first and in
// the same order (rel = number of shared vertices: 1, 2 or 3).
struct TouchPair {
    double P[9], Q[9];      // test / source vertices, canonical order
    double nt[3];           // unit outward normal of the test triangle
    double At, As;          // areas
    int rel, order;         // relation and Gauss order per dimension
    int pi[3], qi[3];       // canonical local index -> caller's local index
};

void launch_patterns(int N, int K, int nph, const double *ct, double k, const int *rtri, const double *rcoef,
                     const int *rloc, const double *tri_v, const double *tri_n, const double *tri_a,
                     const double *centre, cpx<double> *R, cpx<double> *Q, hipStream_t s);
void launch_touch(int npairs, const TouchPair *pairs, double k, const double *gnodes, const int *goff,
                  cpx<double> *out, hipStream_t s);
void launch_slots(int nbox, const int *box_start, const int *near_start, const int *near_box, const long long *val_off,
                  const int *rtri, const int *rloc, const double *rcoef, const double *tri_v, const double *tri_n,
                  const double *tri_a, const int *tp_start, const int *tp_s, const cpx<double> *touch, double k,
                  cpx<double> *em64, cpx<double> *c64, cpx<float> *em32, cpx<float> *c32, hipStream_t s);
void launch_to_float(const cpx<double> *a, cpx<float> *b, long long n, hipStream_t s);
// right-hand sides of eqs. 49-50 for plane waves, written in user RWG order
// (dirs: nrhs x (khat, pol)); single = complex64 output, else complex128
void launch_plane_wave(bool single, int N, int nrhs, double k, const int *perm, const int *rtri, const int *rloc,
                       const double *rcoef, const double *tri_v, const double *tri_n, const double *tri_a,
                       const double *dirs, void *b, long long ldb, hipStream_t s);

// far field F . theta_hat, F . phi_hat of the currents x (user RWG order,
// 2N x nrhs) in ndir directions (dirs: device, ndir x 3): F is ndir x 2 x
// nrhs; single = complex64 input/output, else complex128
void launch_far_field(bool single, int N, double k, const int *perm, const int *rtri, const int *rloc,
                      const double *rcoef, const double *tri_v, const double *tri_a, const double *dirs, int ndir,
                      const void *x, long long ldx, void *F, int nrhs, hipStream_t s);

}  // namespace mlfma
