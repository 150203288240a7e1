// Deflation eigensolver: kernels (eig.hip) and driver (eigsolve.cpp).
#pragma once

#include "ovs_common.h"

namespace ovs {

void launch_fill_random(double2* X, long nfields, const Geometry& g, unsigned long long seed,
                        hipStream_t s);
void launch_cheb(double2* Ynew, const double2* MY, const double2* Y, const double2* Yold,
                 double alpha, double c, double beta, long n, hipStream_t s);
void launch_resid(double2* D, const double2* AR, const double2* R, const double2* theta, int nb,
                  long Np, hipStream_t s);

// Critical eigentriples of A = gamma5 Dw(mu): the m eigenvalues of smallest
// magnitude with right and left eigenvectors, biorthonormalised.  Writes the
// FP64 device fields R, L ([m][12][Vs], allocated by the caller) and the host
// eigenvalues lam[m]; info[0] = max relative residual, info[1] =
// max |L^dagger R - I|, info[2] = filter passes used (both sides).
ovs_status compute_eigentriples(ovs_lattice_s* l, int m, double tol, int max_iter, double2* R,
                                double2* L, double* lam, double* info);

}  // namespace ovs
