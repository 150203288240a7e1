// Deflation eigensolver: kernels (eig.hip) and driver (eigsolve.cpp).
#pragma once

#include "ovs_common.h"

namespace ovs {

void launch_fill_random(double2* X, long nfields, const Geometry& g, unsigned long long seed,
                        hipStream_t s);
// Ynew = alpha (MY - c Y) + beta Yold (Yold may be null), n entries
void launch_cheb(double2* Ynew, const double2* MY, const double2* Y, const double2* Yold,
                 double alpha, double c, double beta, long n, hipStream_t s);
void launch_resid(double2* D, const double2* AR, const double2* R, const double2* theta, int nb,
                  long Np, hipStream_t s);
// One step of block CG on the normal equations (eig.hip): part holds
// n * cg_nchunk(Np) doubles.
int cg_nchunk(long Np);
void launch_cg_xr(double2* X, double2* R, const double2* P, const double2* W, const double* rr,
                  const double* tt, int n, long Np, double* part, hipStream_t s);
void launch_cg_p(double2* P, const double2* R, const double* rr, double* rr_next,
                 const double* part, int n, long Np, hipStream_t s);

// Critical eigentriples of A = gamma5 Dw(mu): the m eigenvalues of smallest
// magnitude with right and left eigenvectors, biorthonormalised.  Writes the
// FP64 device fields R, L ([m][12][Vs], allocated by the caller) and the host
// eigenvalues lam[m]; info[0] = max relative residual, info[1] =
// max |L^dagger R - I|, info[2] = Krylov-Schur restarts (both sides).
ovs_status compute_eigentriples(ovs_lattice_s* l, int m, double tol, int max_iter, double2* R,
                                double2* L, double* lam, double* info);

}  // namespace ovs
