// Eigenvalues of the overlap operator D_ov(mu) = 1 + gamma5 sgn(A) (Section 1)
// with the sign function applied by the two-sided Lanczos driver: the use the
// closing outlook of Section 5 names for these methods.
//
// Outer method: block Arnoldi with thick restarts in Krylov-Schur form, block
// size b (b = 1: plain Arnoldi).  The factorisation D V_m = V_m H_m + V' R E^T
// (V' the next block, E the last b columns) grows by one block per step: one
// batched sign solve of b sources (ovs_sign_apply with OVS_FLAG_OVERLAP,
// writing straight into the next block of the basis), classical Gram-Schmidt
// against the basis applied twice, then Cholesky QR applied twice to the new
// block (rocBLAS zgemm on the lattice stream, the b x b factors on the host).
// At a restart the Ritz pairs of H_m are ordered by |theta|; the Ritz vectors
// of the `keep` smallest span an H_m-invariant subspace, so with Q an
// orthonormal basis of it (host, modified Gram-Schmidt twice)
// D (V_m Q) = (V_m Q)(Q^H H_m Q) + V' (R E^T Q), and the factorisation
// continues from keep + b vectors.  A Ritz pair's residual is |R E^T y| (unit
// y); the iteration stops when the nev wanted ones are all below tol.  The
// inner solves' own error (tol_inner) bounds what tol can reach.
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
#include "ovs_krylov.h"

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

namespace ovs {

// The block Krylov-Schur driver for any operator given as op(in, out, n, warn):
// n canonical complex128 fields in, n out (device), *warn += sources whose
// application returned a warning.  Arguments are checked by the callers.
ovs_status block_krylov_eigs(ovs_lattice_s* l, const BlockOp& op, int nev, int ncv, int block,
                             double tol, int max_restarts, double* lambda, void* vecs,
                             double* info, const KrylovOptions& opt) {
  const int bs = block;
  const long N = opt.field_len > 0 ? opt.field_len : 12L * l->g.V;
  const int nconv = opt.nconv > 0 ? std::min(opt.nconv, nev) : nev;
  const int m = ncv;
  StreamScope sc(l);
  hipStream_t s = l->stream;
  Blas bl;
  if (rocblas_create_handle(&bl.h) != rocblas_status_success ||
      rocblas_set_stream(bl.h, s) != rocblas_status_success ||
      rocblas_set_pointer_mode(bl.h, rocblas_pointer_mode_host) != rocblas_status_success)
    return OVS_ERR_HIP;
  Buffers mem;
  auto* V = mem.alloc<rocblas_double_complex>((size_t)(m + bs) * N);
  auto* Wt = mem.alloc<rocblas_double_complex>((size_t)m * N);  // zgemm outputs
  auto* Hd = mem.alloc<rocblas_double_complex>((size_t)(m + bs) * bs);
  auto* Rd = mem.alloc<rocblas_double_complex>((size_t)bs * bs);
  auto* Qd = mem.alloc<rocblas_double_complex>((size_t)(m + bs) * (m + bs));
  double* gpart = mem.alloc<double>((size_t)2 * (m + bs) * arn_nchunk(N));  // dot partials
  if (!V || !Wt || !Hd || !Rd || !Qd || !gpart) return OVS_ERR_ALLOC;
  const rocblas_double_complex one{1.0, 0.0}, zero{0.0, 0.0}, mone{-1.0, 0.0};
  const auto opN = rocblas_operation_none;
  const rocblas_int n32 = (rocblas_int)N;
  auto col = [&](int j) { return V + (size_t)j * N; };
  auto blas_ok = [](rocblas_status st) { return st == rocblas_status_success; };

  // Orthonormalises the block at columns c .. c + bs - 1 against columns
  // 0 .. c - 1 (classical Gram-Schmidt, twice) and within itself (Cholesky QR,
  // twice).  Returns the coefficients: hc (c x bs) and the upper triangular
  // r (bs x bs) with block_in = V[:, 0:c] hc + block_out r.
  std::vector<cd> hc, hp, g(bs * bs), r(bs * bs), rp(bs * bs);
  auto orth_block = [&](int c) -> ovs_status {
    rocblas_double_complex* W = col(c);
    hc.assign((size_t)c * bs, cd(0));
    hp.resize((size_t)c * bs);
    for (int pass = 0; pass < 2 && c > 0; ++pass) {
      // V^H W by the dot kernel (tall-skinny: K = N), W -= V (V^H W) by zgemm
      launch_gram((const double2*)V, c, (const double2*)W, bs, N, gpart, (double2*)Hd, s);
      OVS_HIP(hipGetLastError());
      if (!blas_ok(rocblas_zgemm(bl.h, opN, opN, n32, bs, c, &mone, V, n32, Hd, c, &one, W, n32)))
        return OVS_ERR_HIP;
      OVS_HIP(hipMemcpyAsync(hp.data(), Hd, hp.size() * sizeof(cd), hipMemcpyDeviceToHost, s));
      OVS_HIP(hipStreamSynchronize(s));
      for (size_t i = 0; i < hc.size(); ++i) hc[i] += hp[i];
    }
    std::fill(r.begin(), r.end(), cd(0));
    for (int i = 0; i < bs; ++i) r[(size_t)i * bs + i] = 1.0;
    for (int pass = 0; pass < 2; ++pass) {
      launch_gram((const double2*)W, bs, (const double2*)W, bs, N, gpart, (double2*)Rd, s);
      OVS_HIP(hipGetLastError());
      OVS_HIP(hipMemcpyAsync(g.data(), Rd, g.size() * sizeof(cd), hipMemcpyDeviceToHost, s));
      OVS_HIP(hipStreamSynchronize(s));
      if (dense::cholesky(bs, g.data()) != 0) return OVS_WARN_BREAKDOWN;
      // r <- g r (both upper triangular)
      for (int j = 0; j < bs; ++j)
        for (int i = 0; i <= j; ++i) {
          cd a = 0;
          for (int q = i; q <= j; ++q) a += g[(size_t)q * bs + i] * r[(size_t)j * bs + q];
          rp[(size_t)j * bs + i] = a;
        }
      for (int j = 0; j < bs; ++j)
        for (int i = 0; i < bs; ++i) r[(size_t)j * bs + i] = i <= j ? rp[(size_t)j * bs + i] : 0.0;
      if (dense::inverse(bs, g.data()) != 0) return OVS_WARN_BREAKDOWN;
      OVS_HIP(hipMemcpyAsync(Rd, g.data(), g.size() * sizeof(cd), hipMemcpyHostToDevice, s));
      if (!blas_ok(rocblas_zgemm(bl.h, opN, opN, n32, bs, bs, &one, W, n32, Rd, bs, &zero, Wt, n32)))
        return OVS_ERR_HIP;
      OVS_HIP(hipMemcpyAsync(W, Wt, (size_t)bs * N * sizeof(cd), hipMemcpyDeviceToDevice, s));
      OVS_HIP(hipStreamSynchronize(s));  // g is reused
    }
    return OVS_OK;
  };

  if (opt.start) {
    opt.start(col(0), bs);
    const ovs_status so = orth_block(0);
    if (so != OVS_OK) return so;
  } else {  // start block
    std::vector<cd> v0(N);
    for (int c = 0; c < bs; ++c) {
      for (long i = 0; i < N; ++i) {
        const uint64_t e = 2 * ((uint64_t)c * (uint64_t)N + (uint64_t)i);
        const uint64_t a = mix(e), b = mix(e + 1);
        v0[i] = cd((double)(a >> 11) * 0x1.0p-52 - 1.0, (double)(b >> 11) * 0x1.0p-52 - 1.0);
      }
      OVS_HIP(hipMemcpyAsync(col(c), v0.data(), N * sizeof(cd), hipMemcpyHostToDevice, s));
      OVS_HIP(hipStreamSynchronize(s));  // v0 is refilled
    }
    const ovs_status so = orth_block(0);
    if (so != OVS_OK) return so;
  }

  const int ld = m + bs;
  std::vector<cd> H((size_t)ld * m, cd(0));  // column-major, leading dimension m + bs
  auto Hat = [&](int i, int j) -> cd& { return H[(size_t)j * ld + i]; };
  std::vector<cd> theta(m), Y((size_t)m * m), Hm((size_t)m * m);
  std::vector<int> order(m);
  std::vector<double> res(m);
  std::vector<cd> rq(nev);
  int k = 0, restarts = 0, matvecs = 0, inner_warn = 0;
  bool converged = false;
  for (;;) {
    // extend the factorisation from k to m columns, one block at a time
    for (int p = k; p < m; p += bs) {
      const ovs_status st = op(col(p), col(p + bs), bs, &inner_warn);
      matvecs += bs;
      if (st < 0) return st;
      const ovs_status so = orth_block(p + bs);
      if (so != OVS_OK) return so;
      for (int j = 0; j < bs; ++j) {
        for (int i = 0; i < p + bs; ++i) Hat(i, p + j) = hc[(size_t)j * (p + bs) + i];
        for (int i = 0; i < bs; ++i) Hat(p + bs + i, p + j) = r[(size_t)j * bs + i];
      }
    }
    // Harmonic Ritz pairs for the target 0 (the wanted eigenvalues lie inside
    // the spectrum, where Ritz values are unreliable): with H_m and the last
    // block row R, M = H_m + H_m^{-H} E R^H R E^T; (theta, y) eigenpairs of M,
    // ordered by |theta|.  Each y (unit) is reported with its Rayleigh
    // quotient rho = y^H H_m y and the residual |H_bar y - rho [y; 0]| of
    // D (V_m y) - rho V_m y.  If H_m is singular (a zero mode already in the
    // basis) the cycle takes ordinary Ritz pairs (eigenpairs of H_m), and so
    // does the largest-magnitude mode, ordered by decreasing |theta|.
    for (int c = 0; c < m; ++c)
      for (int i = 0; i < m; ++i) Hm[(size_t)c * m + i] = Hat(i, c);
    std::vector<cd> Hinv((size_t)m * m), M(Hm), RR((size_t)bs * bs);
    for (int c = 0; c < m; ++c)
      for (int i = 0; i < m; ++i) Hinv[(size_t)c * m + i] = std::conj(Hm[(size_t)i * m + c]);
    const bool harmonic = !opt.largest && dense::inverse(m, Hinv.data()) == 0;  // H_m^{-H}
    if (harmonic) {
      for (int j = 0; j < bs; ++j)  // R^H R
        for (int i = 0; i < bs; ++i) {
          cd a = 0;
          for (int q = 0; q < bs; ++q) a += std::conj(Hat(m + q, m - bs + i)) * Hat(m + q, m - bs + j);
          RR[(size_t)j * bs + i] = a;
        }
      for (int j = 0; j < bs; ++j)
        for (int i = 0; i < m; ++i) {
          cd a = 0;
          for (int q = 0; q < bs; ++q) a += Hinv[(size_t)(m - bs + q) * m + i] * RR[(size_t)j * bs + q];
          M[(size_t)(m - bs + j) * m + i] += a;
        }
    }
    if (dense::eig(m, M.data(), theta.data(), Y.data()) != 0) return OVS_WARN_BREAKDOWN;
    std::iota(order.begin(), order.end(), 0);
    if (opt.largest)
      std::stable_sort(order.begin(), order.end(),
                       [&](int a, int b) { return std::abs(theta[a]) > std::abs(theta[b]); });
    else
      std::stable_sort(order.begin(), order.end(),
                       [&](int a, int b) { return std::abs(theta[a]) < std::abs(theta[b]); });
    double worst = 0;
    for (int q = 0; q < nev; ++q) {
      const cd* y = &Y[(size_t)order[q] * m];
      std::vector<cd> hy(m, cd(0));
      for (int c = 0; c < m; ++c)
        for (int i = 0; i < m; ++i) hy[i] += Hm[(size_t)c * m + i] * y[c];
      cd rho = 0;
      for (int i = 0; i < m; ++i) rho += std::conj(y[i]) * hy[i];
      double n2 = 0;
      for (int i = 0; i < m; ++i) n2 += std::norm(hy[i] - rho * y[i]);
      for (int i = 0; i < bs; ++i) {
        cd a = 0;
        for (int j = 0; j < bs; ++j) a += Hat(m + i, m - bs + j) * y[m - bs + j];
        n2 += std::norm(a);
      }
      rq[q] = rho;
      res[q] = std::sqrt(n2);
      if (q < nconv) worst = std::max(worst, res[q]);
    }
    if (info) info[0] = worst;
    if (opt.progress) opt.progress(restarts, worst, matvecs);
    if (worst <= tol) {
      converged = true;
      break;
    }
    if (restarts == max_restarts) break;
    // thick restart: keep the vectors of the `keep` smallest |theta| (rounded so
    // that whole blocks are added; ncv >= nev + 2 bs keeps keep >= nev) and the
    // block G = [-H_m^{-H} E R^H; I] that the residuals of harmonic pairs lie in
    // (G = [0; I] for ordinary Ritz pairs).  With Qt an orthonormal basis of
    // [[Q; 0], G] ((m + bs) x (keep + bs)), D (V_m Q) = (V_bar Qt)(Qt^H H_bar Q).
    const int add = std::max(1, ((m - nev) - (m - nev) / 2) / bs) * bs;
    const int keep = m - add;
    const int kt = keep + bs;
    std::vector<cd> Qt((size_t)ld * kt, cd(0));
    for (int i = 0; i < keep; ++i)
      std::copy_n(&Y[(size_t)order[i] * m], m, &Qt[(size_t)i * ld]);
    for (int j = 0; j < bs; ++j) {
      cd* gj = &Qt[(size_t)(keep + j) * ld];
      if (harmonic)
        for (int i = 0; i < m; ++i) {
          cd a = 0;
          for (int q = 0; q < bs; ++q)
            a -= Hinv[(size_t)(m - bs + q) * m + i] * std::conj(Hat(m + j, m - bs + q));
          gj[i] = a;
        }
      gj[m + j] = 1.0;
    }
    if (!mgs2(ld, kt, Qt)) return OVS_WARN_BREAKDOWN;
    OVS_HIP(hipMemcpyAsync(Qd, Qt.data(), Qt.size() * sizeof(cd), hipMemcpyHostToDevice, s));
    if (!blas_ok(rocblas_zgemm(bl.h, opN, opN, n32, kt, ld, &one, V, n32, Qd, ld, &zero, Wt, n32)))
      return OVS_ERR_HIP;
    OVS_HIP(hipMemcpyAsync(col(0), Wt, (size_t)kt * N * sizeof(cd), hipMemcpyDeviceToDevice, s));
    // new projected matrix Qt^H H_bar Q, (keep + bs) x keep
    std::vector<cd> HQ((size_t)ld * keep, cd(0));
    for (int c = 0; c < keep; ++c)
      for (int i = 0; i < ld; ++i) {
        cd a = 0;
        for (int q = 0; q < m; ++q) a += Hat(i, q) * Qt[(size_t)c * ld + q];
        HQ[(size_t)c * ld + i] = a;
      }
    std::vector<cd> Hn((size_t)kt * keep, cd(0));
    for (int c = 0; c < keep; ++c)
      for (int i = 0; i < kt; ++i) {
        cd a = 0;
        for (int q = 0; q < ld; ++q) a += std::conj(Qt[(size_t)i * ld + q]) * HQ[(size_t)c * ld + q];
        Hn[(size_t)c * kt + i] = a;
      }
    std::fill(H.begin(), H.end(), cd(0));
    for (int c = 0; c < keep; ++c)
      for (int i = 0; i < kt; ++i) Hat(i, c) = Hn[(size_t)c * kt + i];
    k = keep;
    ++restarts;
    OVS_HIP(hipStreamSynchronize(s));  // Q and the host matrices are reused
  }
  for (int i = 0; i < nev; ++i) {
    lambda[2 * i] = rq[i].real();
    lambda[2 * i + 1] = rq[i].imag();
  }
  if (vecs) {  // x_i = V_m y_i: unit norm (V_m orthonormal, y_i unit)
    std::vector<cd> Ys((size_t)m * nev);
    for (int i = 0; i < nev; ++i) std::copy_n(&Y[(size_t)order[i] * m], m, &Ys[(size_t)i * m]);
    OVS_HIP(hipMemcpyAsync(Qd, Ys.data(), Ys.size() * sizeof(cd), hipMemcpyHostToDevice, s));
    if (!blas_ok(rocblas_zgemm(bl.h, opN, opN, n32, nev, m, &one, V, n32, Qd, m, &zero,
                               (rocblas_double_complex*)vecs, n32)))
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

}  // namespace ovs

extern "C" ovs_status ovs_overlap_eigs(ovs_lattice l, ovs_deflation defl, int32_t n_defl,
                                       int32_t nev, int32_t ncv, int32_t block, int32_t k_inner,
                                       double tol_inner, int32_t inner_flags, double tol,
                                       int32_t max_restarts, double* lambda, void* vecs,
                                       double* info) {
  const int bs = block;
  if (!l || !lambda || nev < 1 || bs < 1 || bs > 16 || ncv % bs != 0 || ncv < nev + 2 * bs ||
      ncv > 256 || k_inner < 1 || !(tol_inner > 0) || !(tol > 0) || max_restarts < 0 ||
      (inner_flags & ~(OVS_FLAG_TWO_PASS | OVS_FLAG_GRAPH | OVS_FLAG_PERSISTENT)))
    return OVS_ERR_ARG;
  if (!ready(l)) return OVS_ERR_STATE;
  const long N = 12L * l->g.V;
  if (ncv + bs >= N || k_inner > N) return OVS_ERR_ARG;
  std::vector<double> tols(bs, tol_inner);
  std::vector<ovs_rhs_info> ri(bs);
  // one application of D_ov to a block: a batched sign solve
  const BlockOp op = [&](const void* in, void* out, int n, int* warn) -> ovs_status {
    const ovs_status st = ovs_sign_apply(l, defl, n_defl, in, out, n, k_inner, tols.data(),
                                         OVS_2SL, OVS_FLAG_OVERLAP | inner_flags, nullptr, 0,
                                         ri.data());
    if (st >= 0)
      for (int i = 0; i < n; ++i) *warn += ri[i].status != OVS_OK;
    return st;
  };
  return block_krylov_eigs(l, op, nev, ncv, bs, tol, max_restarts, lambda, vecs, info);
}

