// Small dense complex linear algebra on the host (column-major).
#pragma once

#include <complex>

namespace ovs {
namespace dense {

// Eigenvalues lam[n] and unit-norm right eigenvectors V (n x n, column k for
// lam[k]) of a general complex matrix A (n x n).  Returns 0, or < 0 if the QR
// iteration did not converge.
int eig(int n, const std::complex<double>* A, std::complex<double>* lam, std::complex<double>* V);
// In-place Cholesky A = R^H R (R upper).  Returns -1 if A is not positive definite.
int cholesky(int n, std::complex<double>* A);
// In-place inverse with partial pivoting.  Returns -1 if singular.
int inverse(int n, std::complex<double>* A);

}  // namespace dense
}  // namespace ovs
