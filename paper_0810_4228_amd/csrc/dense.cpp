// Small dense complex linear algebra on the host, for the Rayleigh-Ritz and
// biorthonormalisation steps of the deflation eigensolver (matrices of order
// <= a few hundred).  Column-major storage: A[i + n*j] is row i, column j.
//
//   eig:      Householder reduction to Hessenberg form, then single-shift QR
//             iterations with Wilkinson shifts (complex Schur form A = Z T Z^H),
//             eigenvectors of T by back substitution, mapped back with Z.
//   cholesky: A = R^H R for Hermitian positive definite A (upper R).
//   inverse:  Gauss-Jordan with partial pivoting.
#include "dense.h"

#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

namespace ovs {
namespace dense {

using cd = std::complex<double>;

static inline cd& at(std::vector<cd>& a, int n, int i, int j) { return a[i + (size_t)n * j]; }

// Givens rotation G = [[c, s], [-conj(s), c]] with G [a; b] = [r; 0], c real.
static void givens(cd a, cd b, double& c, cd& s) {
  const double aa = std::abs(a), bb = std::abs(b);
  if (bb == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  if (aa == 0.0) {
    c = 0.0;
    s = std::conj(b) / bb;
    return;
  }
  const double nrm = std::hypot(aa, bb);
  c = aa / nrm;
  s = (a / aa) * std::conj(b) / nrm;
}

int eig(int n, const cd* A, cd* lam, cd* V) {
  if (n <= 0) return -1;
  std::vector<cd> H(A, A + (size_t)n * n);
  std::vector<cd> Z((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) at(Z, n, i, i) = 1.0;
  // ---- Householder reduction to upper Hessenberg form ----
  std::vector<cd> v(n);
  for (int k = 0; k + 2 < n; ++k) {
    double xn = 0.0;
    for (int i = k + 1; i < n; ++i) xn += std::norm(at(H, n, i, k));
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const cd x0 = at(H, n, k + 1, k);
    const cd ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cd(1.0);
    for (int i = 0; i < n; ++i) v[i] = 0.0;
    for (int i = k + 1; i < n; ++i) v[i] = at(H, n, i, k);
    v[k + 1] += ph * xn;
    double vn = 0.0;
    for (int i = k + 1; i < n; ++i) vn += std::norm(v[i]);
    vn = std::sqrt(vn);
    for (int i = k + 1; i < n; ++i) v[i] /= vn;
    // H <- (I - 2 v v^H) H
    for (int j = 0; j < n; ++j) {
      cd d = 0.0;
      for (int i = k + 1; i < n; ++i) d += std::conj(v[i]) * at(H, n, i, j);
      for (int i = k + 1; i < n; ++i) at(H, n, i, j) -= 2.0 * v[i] * d;
    }
    // H <- H (I - 2 v v^H), Z <- Z (I - 2 v v^H)
    for (int i = 0; i < n; ++i) {
      cd d = 0.0, e = 0.0;
      for (int j = k + 1; j < n; ++j) {
        d += at(H, n, i, j) * v[j];
        e += at(Z, n, i, j) * v[j];
      }
      for (int j = k + 1; j < n; ++j) {
        at(H, n, i, j) -= 2.0 * d * std::conj(v[j]);
        at(Z, n, i, j) -= 2.0 * e * std::conj(v[j]);
      }
    }
    for (int i = k + 2; i < n; ++i) at(H, n, i, k) = 0.0;
  }
  // ---- shifted QR iterations to the complex Schur form ----
  const double eps = std::numeric_limits<double>::epsilon();
  double hnorm = 0.0;
  for (auto& x : H) hnorm = std::max(hnorm, std::abs(x));
  if (hnorm == 0.0) hnorm = 1.0;
  int hi = n - 1, iter = 0, total = 0;
  std::vector<double> cs(n);
  std::vector<cd> ss(n);
  while (hi > 0) {
    int l = hi;
    for (; l > 0; --l) {
      const double sub = std::abs(at(H, n, l, l - 1));
      double scale_ = std::abs(at(H, n, l - 1, l - 1)) + std::abs(at(H, n, l, l));
      if (scale_ == 0.0) scale_ = hnorm;
      if (sub <= eps * scale_ || sub <= 1e-300) {
        at(H, n, l, l - 1) = 0.0;
        break;
      }
    }
    if (l == hi) {
      --hi;
      iter = 0;
      continue;
    }
    if (++total > 100 * n) return -2;  // no convergence
    ++iter;
    // Wilkinson shift: eigenvalue of the trailing 2x2 block closer to H[hi][hi]
    cd sigma;
    if (iter % 11 == 10) {
      sigma = at(H, n, hi, hi) + cd(std::abs(at(H, n, hi, hi - 1)), 0.0);  // exceptional shift
    } else {
      const cd a = at(H, n, hi - 1, hi - 1), b = at(H, n, hi - 1, hi);
      const cd c = at(H, n, hi, hi - 1), d = at(H, n, hi, hi);
      const cd tr = a + d, det = a * d - b * c;
      const cd disc = std::sqrt(tr * tr * 0.25 - det);
      const cd e1 = tr * 0.5 + disc, e2 = tr * 0.5 - disc;
      sigma = (std::abs(e1 - d) < std::abs(e2 - d)) ? e1 : e2;
    }
    for (int i = l; i <= hi; ++i) at(H, n, i, i) -= sigma;
    for (int k = l; k < hi; ++k) {
      double c;
      cd s;
      givens(at(H, n, k, k), at(H, n, k + 1, k), c, s);
      cs[k] = c;
      ss[k] = s;
      for (int j = k; j < n; ++j) {
        const cd x = at(H, n, k, j), y = at(H, n, k + 1, j);
        at(H, n, k, j) = c * x + s * y;
        at(H, n, k + 1, j) = -std::conj(s) * x + c * y;
      }
    }
    for (int k = l; k < hi; ++k) {
      const double c = cs[k];
      const cd s = ss[k];
      const int imax = std::min(k + 2, hi);
      for (int i = 0; i <= imax; ++i) {
        const cd x = at(H, n, i, k), y = at(H, n, i, k + 1);
        at(H, n, i, k) = c * x + std::conj(s) * y;
        at(H, n, i, k + 1) = -s * x + c * y;
      }
      for (int i = 0; i < n; ++i) {
        const cd x = at(Z, n, i, k), y = at(Z, n, i, k + 1);
        at(Z, n, i, k) = c * x + std::conj(s) * y;
        at(Z, n, i, k + 1) = -s * x + c * y;
      }
    }
    for (int i = l; i <= hi; ++i) at(H, n, i, i) += sigma;
  }
  for (int i = 0; i < n; ++i) lam[i] = at(H, n, i, i);
  // ---- eigenvectors of the triangular T, mapped back with Z ----
  std::vector<cd> x(n);
  const double small = eps * hnorm;
  for (int k = 0; k < n; ++k) {
    for (int i = 0; i < n; ++i) x[i] = 0.0;
    x[k] = 1.0;
    for (int j = k - 1; j >= 0; --j) {
      cd sum = 0.0;
      for (int i = j + 1; i <= k; ++i) sum += at(H, n, j, i) * x[i];
      cd den = at(H, n, j, j) - lam[k];
      if (std::abs(den) < small) den = small;
      x[j] = -sum / den;
    }
    double nrm = 0.0;
    for (int i = 0; i < n; ++i) {
      cd acc = 0.0;
      for (int j = 0; j <= k; ++j) acc += at(Z, n, i, j) * x[j];
      V[i + (size_t)n * k] = acc;
      nrm += std::norm(acc);
    }
    nrm = std::sqrt(nrm);
    for (int i = 0; i < n; ++i) V[i + (size_t)n * k] /= nrm;
  }
  return 0;
}

int cholesky(int n, cd* A) {
  // in place: upper triangle of A becomes R with A = R^H R; lower part zeroed
  std::vector<cd> a(A, A + (size_t)n * n);
  for (int j = 0; j < n; ++j) {
    double d = std::real(at(a, n, j, j));
    for (int k = 0; k < j; ++k) d -= std::norm(at(a, n, k, j));
    if (!(d > 0.0)) return -1;
    const double rjj = std::sqrt(d);
    at(a, n, j, j) = rjj;
    for (int i = j + 1; i < n; ++i) {
      cd s = at(a, n, j, i);
      for (int k = 0; k < j; ++k) s -= std::conj(at(a, n, k, j)) * at(a, n, k, i);
      at(a, n, j, i) = s / rjj;
    }
  }
  for (int j = 0; j < n; ++j)
    for (int i = j + 1; i < n; ++i) at(a, n, i, j) = 0.0;
  std::copy(a.begin(), a.end(), A);
  return 0;
}

int inverse(int n, cd* A) {
  std::vector<cd> a(A, A + (size_t)n * n), inv((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) at(inv, n, i, i) = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    double best = std::abs(at(a, n, c, c));
    for (int r = c + 1; r < n; ++r)
      if (std::abs(at(a, n, r, c)) > best) {
        best = std::abs(at(a, n, r, c));
        p = r;
      }
    if (best == 0.0) return -1;
    if (p != c)
      for (int j = 0; j < n; ++j) {
        std::swap(at(a, n, p, j), at(a, n, c, j));
        std::swap(at(inv, n, p, j), at(inv, n, c, j));
      }
    const cd piv = at(a, n, c, c);
    for (int j = 0; j < n; ++j) {
      at(a, n, c, j) /= piv;
      at(inv, n, c, j) /= piv;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const cd f = at(a, n, r, c);
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        at(a, n, r, j) -= f * at(a, n, c, j);
        at(inv, n, r, j) -= f * at(inv, n, c, j);
      }
    }
  }
  std::copy(inv.begin(), inv.end(), A);
  return 0;
}

}  // namespace dense
}  // namespace ovs
