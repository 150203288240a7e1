// Launchers of the Krylov-side kernels (krylov.hip).
#pragma once

#include "ovs_common.h"

namespace ovs {

constexpr int kHessMaxK = 1536;   // largest Arnoldi size of the Hessenberg inner sign

int defl_nchunk(long N);
void launch_defl(const double2* R, const double2* L, const double2* B, const double* sgn, int m,
                 int nrhs, long N, double* partials, double* CD, double2* bR, double2* bL,
                 double2* yex, hipStream_t s);
// Projections of X (nrhs fields) against the deflation space: outQ = X - R
// (L^dag X) and outQd = X - L (R^dag X) + L kappa (kappa [nrhs][m] or null);
// either output may be null.  CD [m][nrhs][4] receives the dots.
void launch_defl_proj(const double2* R, const double2* L, const double2* X, int m, int nrhs, long N,
                      double* partials, double* CD, const double2* kappa, double2* outQ,
                      double2* outQd, hipStream_t s);
// CD[j][r] = (L_j^dag B_r, R_j^dag B_r) only (used to check L^dag R = I)
void launch_defl_cd(const double2* R, const double2* L, const double2* B, int m, int nrhs, long N,
                    double* partials, double* CD, hipStream_t s);
void launch_start(const double2* bR, const double2* bL, int nrhs, long N, double* partials,
                  double* sums, void* V0, void* W0, bool f32, hipStream_t s);

int update_nwg(long N);
void launch_alpha(const double* partials, int nparts, const CoefArrays& co, const int* it,
                  const int* rhs_map, const int* n_active, int nslots, hipStream_t s);
// apart != nullptr: alpha is formed from the dual stencil's anparts partials
// inside the update (k_alpha is then not launched).  nt: streaming stores of
// the new vectors.
void launch_update(bool f32, const void* T, const void* S, void* basis, long basis_stride,
                   void* wbuf, long N, const CoefArrays& co, const int* it, const int* rhs_map,
                   const int* n_active, int nslots, double* partials, bool ring,
                   const double* apart, int anparts, int nt, hipStream_t s);
// beta, the probe gather (probes != nullptr) and the iteration advance in one
// launch; *ticket must be zero before the first launch and stays zero after each.
void launch_beta_tail(bool f32, const double* partials, int nparts, const CoefArrays& co, int* it,
                      const int* rhs_map, const int* n_active, int nslots, int* ticket,
                      const void* basis, long basis_stride, long N, bool ring, const int* idx,
                      int P, double2* probes, hipStream_t s);
void launch_advance(int* it, hipStream_t s);
void launch_probe_gather(bool f32, const void* basis, long basis_stride, long N, bool ring,
                         const int* it, bool first, const int* idx, int P, int kmax,
                         const int* rhs_map, const int* n_active, int nslots, double2* probes,
                         hipStream_t s);
void launch_probe_y(const double2* probes, const double2* coef, const int* kvec, int kmax,
                    const double2* yex, long N, const int* idx, int P, double2* yp, int nrhs,
                    hipStream_t s);

void launch_make_coef(const double2* x, const double* sv, const double* nb, int kmax, int nrhs,
                      double2* coef, hipStream_t s);
void launch_combine(bool f32, const void* basis, long basis_stride, long N, const double2* coef,
                    int kmax, const int* kused, const double2* yex, double2* y, int nrhs,
                    hipStream_t s);
void launch_replay(bool f32, const void* T, void* ring, long ring_stride, long N,
                   const CoefArrays& co, int i, const double2* coef, const int* kused, double2* y,
                   int nrhs, hipStream_t s);
void launch_overlap(const double2* b, double2* y, long N, int V, hipStream_t s);

int arn_nchunk(long N);
void launch_arn_dots(bool f32, const void* basis, long basis_stride, const void* T, long N,
                     int nvec, int nrhs, double* partials, double* red, hipStream_t s);
// G = X^H Y (nx x ny, column-major) for column-major FP64 blocks with
// leading dimension N: one dot launch per column of Y (tall-skinny products
// that library GEMMs tile poorly); partials hold nx * arn_nchunk(N) * 2.
void launch_gram(const double2* X, int nx, const double2* Y, int ny, long N, double* partials,
                 double2* G, hipStream_t s);
void launch_arn_accum(const double* red, int nvec, int kmax, int j, bool first, double2* H,
                      double2* hcur, int nrhs, hipStream_t s);
void launch_arn_axpy(bool f32, const void* basis, long basis_stride, void* T, long N, int nvec,
                     const double2* hcur, int kmax, int nrhs, double* partials, double* red,
                     hipStream_t s);
void launch_norm2(bool f32, const void* T, long N, int nrhs, double* partials, double* red,
                  hipStream_t s);
void launch_arn_sub(const double* red_n, const double* red_tn, double2* H, int kmax, int j,
                    double* scl, int* kstop, int* status, int nrhs, hipStream_t s);
void launch_scale_copy(bool f32, const void* T, void* out, long N, const double* scl, int nrhs,
                       hipStream_t s);

// Inner sign by the tau = e^u trapezoid rule.  The tridiagonal form runs its
// shifted solves in launches of at most kIsignWaveChunk waves of 64 solves
// per source (mult, swp: [nrhs][kIsignWaveChunk][kmax][64]; part: [nrhs][all
// waves][2][kmax]); the Hessenberg form kIsignHessChunk solves per source
// (ys: [nrhs][kIsignHessChunk][kmax]; acc: [nrhs][2][kmax]).  A launch takes
// about k sequential elimination steps whatever its number of waves, so the
// chunk holds every solve of the rules down to step 1/16 (43 waves): one
// launch for those, two at 1/32 and four at 1/64.
constexpr int kIsignWaveChunk = 48;
constexpr int kIsignHessChunk = 1024;
// A trapezoid rule in u: nodes u = n h for n0 <= n < n0 + nnode.
struct QuadNodes {
  double h;   // step in u
  int n0;     // first node index (u = n h)
  int nnode;  // number of nodes
};
int isign_tri_nwave(int nnode);
// rules: device array [nrhs], the rule of each source; nwave: the largest
// isign_tri_nwave over the sources with kvec[r] > 0 (the part stride).
void launch_isign_tri(const double2* alpha, const double* beta, const double2* gamma, int kmax,
                      const int* kvec, int nrhs, const QuadNodes* rules, int nwave, double2* mult,
                      unsigned char* swp, double2* part, double2* x, double* err, hipStream_t s);
void launch_isign_hess(const double2* H, int kmax, const int* kvec, int nrhs, double h, int n0,
                       int nnode, double2* ys, double2* acc, double2* x, double* err,
                       hipStream_t s);

}  // namespace ovs
