// Eigenvalues of the overlap operator D_ov(mu) = 1 + gamma5 sgn(A) (Section 1)
// with the sign function applied by the two-sided Lanczos driver: the use the
// closing outlook of Section 5 names for these methods.
//
// Outer method: Arnoldi with thick restarts in Krylov-Schur form.  The
// factorisation D V_m = V_m H_m + h v_{m+1} e_m^T is built with one sign
// solve per step (ovs_sign_apply with OVS_FLAG_OVERLAP, one source, writing
// straight into the next basis column) and classical Gram-Schmidt applied
// twice (rocBLAS zgemv on the lattice stream).  At a restart the Ritz pairs of
// H_m are ordered by |theta|; the Ritz vectors of the `keep` smallest span an
// H_m-invariant subspace, so with Q an orthonormal basis of it (host, modified
// Gram-Schmidt twice) D (V_m Q) = (V_m Q)(Q^H H_m Q) + h v_{m+1} (e_m^T Q), and
// the factorisation continues from keep + 1 vectors.  A Ritz pair's residual
// is |h| |e_m^T y| (unit y); the iteration stops when the nev wanted ones are
// all below tol.  The inner solves' own error (tol_inner) bounds what tol can
// reach.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <numeric>
#include <vector>

#include "../../include/ovsign.h"
#include "dense.h"
#include "ovs_common.h"
#include "ovs_host.h"

using namespace ovs;

namespace {

using cd = std::complex<double>;

struct Blas {
  rocblas_handle h = nullptr;
  ~Blas() {
    if (h) (void)rocblas_destroy_handle(h);
  }
};

struct Buffers {
  std::vector<void*> p;
  ~Buffers() {
    for (void* q : p) (void)hipFree(q);
  }
  template <class T>
  T* alloc(size_t n) {
    void* q = nullptr;
    if (hipMalloc(&q, n * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    p.push_back(q);
    return (T*)q;
  }
};

// splitmix64: the fixed start vector (entries uniform in [-1, 1) + i [-1, 1))
uint64_t mix(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// Columns of Y (m x k, column-major) replaced by an orthonormal basis of their
// span: modified Gram-Schmidt, twice.  False if a column is (numerically)
// dependent on the previous ones.
bool mgs2(int m, int k, std::vector<cd>& Y) {
  for (int j = 0; j < k; ++j) {
    cd* yj = &Y[(size_t)j * m];
    double n0 = 0;
    for (int r = 0; r < m; ++r) n0 += std::norm(yj[r]);
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < j; ++i) {
        const cd* yi = &Y[(size_t)i * m];
        cd d = 0;
        for (int r = 0; r < m; ++r) d += std::conj(yi[r]) * yj[r];
        for (int r = 0; r < m; ++r) yj[r] -= d * yi[r];
      }
    double n = 0;
    for (int r = 0; r < m; ++r) n += std::norm(yj[r]);
    if (!(n > 1e-24 * n0) || n == 0) return false;
    const double s = 1.0 / std::sqrt(n);
    for (int r = 0; r < m; ++r) yj[r] *= s;
  }
  return true;
}

}  // namespace

extern "C" ovs_status ovs_overlap_eigs(ovs_lattice l, ovs_deflation defl, int32_t n_defl,
                                       int32_t nev, int32_t ncv, int32_t k_inner,
                                       double tol_inner, int32_t inner_flags, double tol,
                                       int32_t max_restarts, double* lambda, void* vecs,
                                       double* info) {
  if (!l || !lambda || nev < 1 || ncv < nev + 2 || ncv > 256 || k_inner < 1 ||
      !(tol_inner > 0) || !(tol > 0) || max_restarts < 0 ||
      (inner_flags & ~(OVS_FLAG_TWO_PASS | OVS_FLAG_GRAPH | OVS_FLAG_PERSISTENT)))
    return OVS_ERR_ARG;
  if (!ready(l)) return OVS_ERR_STATE;
  const long N = 12L * l->g.V;
  if (ncv >= N || k_inner > N) return OVS_ERR_ARG;
  const int m = ncv;
  StreamScope sc(l);
  hipStream_t s = l->stream;
  Blas bl;
  if (rocblas_create_handle(&bl.h) != rocblas_status_success ||
      rocblas_set_stream(bl.h, s) != rocblas_status_success ||
      rocblas_set_pointer_mode(bl.h, rocblas_pointer_mode_host) != rocblas_status_success)
    return OVS_ERR_HIP;
  Buffers mem;
  auto* V = mem.alloc<rocblas_double_complex>((size_t)(m + 1) * N);
  auto* W = mem.alloc<rocblas_double_complex>((size_t)m * N);  // V_m Q at a restart
  auto* hd = mem.alloc<rocblas_double_complex>(m + 1);
  auto* Qd = mem.alloc<rocblas_double_complex>((size_t)m * m);
  if (!V || !W || !hd || !Qd) return OVS_ERR_ALLOC;
  const rocblas_double_complex one{1.0, 0.0}, zero{0.0, 0.0}, mone{-1.0, 0.0};
  auto col = [&](int j) { return V + (size_t)j * N; };
  auto blas_ok = [](rocblas_status st) { return st == rocblas_status_success; };

  {  // start vector
    std::vector<cd> v0(N);
    for (long i = 0; i < N; ++i) {
      const uint64_t a = mix(2 * (uint64_t)i), b = mix(2 * (uint64_t)i + 1);
      v0[i] = cd((double)(a >> 11) * 0x1.0p-52 - 1.0, (double)(b >> 11) * 0x1.0p-52 - 1.0);
    }
    OVS_HIP(hipMemcpyAsync(col(0), v0.data(), N * sizeof(cd), hipMemcpyHostToDevice, s));
    double nrm = 0;
    if (!blas_ok(rocblas_dznrm2(bl.h, (rocblas_int)N, col(0), 1, &nrm))) return OVS_ERR_HIP;
    const double inv = 1.0 / nrm;
    if (!blas_ok(rocblas_zdscal(bl.h, (rocblas_int)N, &inv, col(0), 1))) return OVS_ERR_HIP;
    OVS_HIP(hipStreamSynchronize(s));  // v0 leaves host memory
  }

  std::vector<cd> H((size_t)(m + 1) * m, cd(0));  // column-major, leading dimension m + 1
  auto Hat = [&](int r, int c) -> cd& { return H[(size_t)c * (m + 1) + r]; };
  std::vector<cd> hh(m + 1), h2(m + 1), theta(m), Y((size_t)m * m), Hm((size_t)m * m);
  std::vector<int> order(m);
  std::vector<double> res(m);
  int k = 0, restarts = 0, matvecs = 0, inner_warn = 0;
  bool converged = false;
  ovs_status st = OVS_OK;
  for (;;) {
    // extend the factorisation from k to m columns
    for (int j = k; j < m; ++j) {
      const double ti = tol_inner;
      ovs_rhs_info ri;
      st = ovs_sign_apply(l, defl, n_defl, col(j), col(j + 1), 1, k_inner, &ti, OVS_2SL,
                          OVS_FLAG_OVERLAP | inner_flags, &ri);
      ++matvecs;
      if (st < 0) return st;
      if (st > 0) ++inner_warn;
      // classical Gram-Schmidt against v_0 .. v_j, twice
      for (int pass = 0; pass < 2; ++pass) {
        if (!blas_ok(rocblas_zgemv(bl.h, rocblas_operation_conjugate_transpose, (rocblas_int)N,
                                   j + 1, &one, V, (rocblas_int)N, col(j + 1), 1, &zero, hd, 1)) ||
            !blas_ok(rocblas_zgemv(bl.h, rocblas_operation_none, (rocblas_int)N, j + 1, &mone, V,
                                   (rocblas_int)N, hd, 1, &one, col(j + 1), 1)))
          return OVS_ERR_HIP;
        OVS_HIP(hipMemcpyAsync(pass ? h2.data() : hh.data(), hd, (j + 1) * sizeof(cd),
                               hipMemcpyDeviceToHost, s));
      }
      double beta = 0;
      if (!blas_ok(rocblas_dznrm2(bl.h, (rocblas_int)N, col(j + 1), 1, &beta))) return OVS_ERR_HIP;
      OVS_HIP(hipStreamSynchronize(s));
      for (int i = 0; i <= j; ++i) Hat(i, j) = hh[i] + h2[i];
      Hat(j + 1, j) = beta;
      if (!(beta > 0) || !std::isfinite(beta)) return OVS_WARN_BREAKDOWN;
      const double inv = 1.0 / beta;
      if (!blas_ok(rocblas_zdscal(bl.h, (rocblas_int)N, &inv, col(j + 1), 1))) return OVS_ERR_HIP;
    }
    // Ritz pairs of H_m, ordered by |theta|
    for (int c = 0; c < m; ++c)
      for (int r = 0; r < m; ++r) Hm[(size_t)c * m + r] = Hat(r, c);
    if (dense::eig(m, Hm.data(), theta.data(), Y.data()) != 0) return OVS_WARN_BREAKDOWN;
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return std::abs(theta[a]) < std::abs(theta[b]); });
    const double hlast = std::abs(Hat(m, m - 1));
    double worst = 0;
    for (int i = 0; i < m; ++i) res[i] = hlast * std::abs(Y[(size_t)order[i] * m + (m - 1)]);
    for (int i = 0; i < nev; ++i) worst = std::max(worst, res[i]);
    if (info) info[0] = worst;
    if (worst <= tol) {
      converged = true;
      break;
    }
    if (restarts == max_restarts) break;
    // thick restart: keep the Ritz vectors of the `keep` smallest |theta|
    int keep = std::min(nev + (m - nev) / 2, m - 1);
    std::vector<cd> Q((size_t)m * keep);
    for (int i = 0; i < keep; ++i)
      std::copy_n(&Y[(size_t)order[i] * m], m, &Q[(size_t)i * m]);
    if (!mgs2(m, keep, Q)) return OVS_WARN_BREAKDOWN;
    OVS_HIP(hipMemcpyAsync(Qd, Q.data(), Q.size() * sizeof(cd), hipMemcpyHostToDevice, s));
    if (!blas_ok(rocblas_zgemm(bl.h, rocblas_operation_none, rocblas_operation_none,
                               (rocblas_int)N, keep, m, &one, V, (rocblas_int)N, Qd, m, &zero, W,
                               (rocblas_int)N)))
      return OVS_ERR_HIP;
    OVS_HIP(hipMemcpyAsync(col(0), W, (size_t)keep * N * sizeof(cd), hipMemcpyDeviceToDevice, s));
    OVS_HIP(hipMemcpyAsync(col(keep), col(m), N * sizeof(cd), hipMemcpyDeviceToDevice, s));
    // T = Q^H H_m Q and the new residual row h e_m^T Q
    std::vector<cd> HQ((size_t)m * keep, cd(0)), T((size_t)keep * keep, cd(0));
    for (int c = 0; c < keep; ++c)
      for (int r = 0; r < m; ++r) {
        cd a = 0;
        for (int q = 0; q < m; ++q) a += Hm[(size_t)q * m + r] * Q[(size_t)c * m + q];
        HQ[(size_t)c * m + r] = a;
      }
    for (int c = 0; c < keep; ++c)
      for (int r = 0; r < keep; ++r) {
        cd a = 0;
        for (int q = 0; q < m; ++q) a += std::conj(Q[(size_t)r * m + q]) * HQ[(size_t)c * m + q];
        T[(size_t)c * keep + r] = a;
      }
    const cd hm = Hat(m, m - 1);
    std::fill(H.begin(), H.end(), cd(0));
    for (int c = 0; c < keep; ++c) {
      for (int r = 0; r < keep; ++r) Hat(r, c) = T[(size_t)c * keep + r];
      Hat(keep, c) = hm * Q[(size_t)c * m + (m - 1)];
    }
    k = keep;
    ++restarts;
    OVS_HIP(hipStreamSynchronize(s));  // Q and the host matrices are reused
  }
  for (int i = 0; i < nev; ++i) {
    lambda[2 * i] = theta[order[i]].real();
    lambda[2 * i + 1] = theta[order[i]].imag();
  }
  if (vecs) {  // x_i = V_m y_i: unit norm (V_m orthonormal, y_i unit)
    std::vector<cd> Ys((size_t)m * nev);
    for (int i = 0; i < nev; ++i) std::copy_n(&Y[(size_t)order[i] * m], m, &Ys[(size_t)i * m]);
    OVS_HIP(hipMemcpyAsync(Qd, Ys.data(), Ys.size() * sizeof(cd), hipMemcpyHostToDevice, s));
    if (!blas_ok(rocblas_zgemm(bl.h, rocblas_operation_none, rocblas_operation_none,
                               (rocblas_int)N, nev, m, &one, V, (rocblas_int)N, Qd, m, &zero,
                               (rocblas_double_complex*)vecs, (rocblas_int)N)))
      return OVS_ERR_HIP;
    OVS_HIP(hipStreamSynchronize(s));
  }
  if (info) {
    info[1] = restarts;
    info[2] = matvecs;
    info[3] = inner_warn;
  }
  return converged && inner_warn == 0 ? OVS_OK : OVS_WARN_NOT_CONVERGED;
}
