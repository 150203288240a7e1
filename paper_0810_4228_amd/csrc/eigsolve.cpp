// Critical eigentriples of A = gamma5 Dw(mu) on the GPU for LR deflation
// (Section 3: right/left eigenvectors of the m eigenvalues of smallest
// magnitude, L^dagger R = I; Section 5 computes them once per configuration).
//
// Method (the paper uses ARPACK on a CPU): Chebyshev-filtered subspace
// iteration.  The eigenvalues of smallest |lambda| of A are those of smallest
// modulus of M = A^2, which lie near the origin while the rest of spec(M)
// stays near the positive real interval [a, b].  A degree-d Chebyshev
// polynomial of M, scaled to 1 at z = 0, damps [a, b] and keeps the wanted
// part; the filtered block is orthonormalised (Cholesky QR, twice) and a
// Rayleigh-Ritz step on A gives Ritz pairs and the next cut a.  The same is
// done with A^dagger = A(-mu) for the left vectors, which are then paired by
// lambda_L = conj(lambda_R) and biorthonormalised (blockwise for clusters).
// Block applications of A use the multi-source stencil in FP64; the tall
// skinny products X^H Y and X C are rocBLAS zgemm calls; the small dense
// problems run on the host.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>
#include <vector>

#include "dense.h"
#include "ovs_common.h"
#include "ovs_eig.h"
#include "ovs_krylov.h"

namespace ovs {
namespace {

using cd = std::complex<double>;
constexpr int kFilterDegree = 60;

struct Handle {
  rocblas_handle h = nullptr;
  ~Handle() {
    if (h) (void)rocblas_destroy_handle(h);
  }
};

struct DevMem {
  std::vector<void*> ptrs;
  ~DevMem() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <class T>
  T* alloc(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    ptrs.push_back(p);
    return (T*)p;
  }
};

Hop hop_of(double m_w, double mu) {
  Hop h;
  const double k = 1.0 / (8.0 + 2.0 * m_w);
  for (int nu = 0; nu < 4; ++nu) {
    h.fwd[nu] = (nu == 3) ? k * std::exp(mu) : k;
    h.bwd[nu] = (nu == 3) ? k * std::exp(-mu) : k;
    h.f32_fwd[nu] = (float)h.fwd[nu];
    h.f32_bwd[nu] = (float)h.bwd[nu];
  }
  return h;
}

bool zgemm_ch(rocblas_handle h, const double2* X, int nx, const double2* Y, int ny, long Np,
              double2* G) {  // G = X^H Y   (nx x ny)
  const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
  return rocblas_zgemm(h, rocblas_operation_conjugate_transpose, rocblas_operation_none, nx, ny,
                       (rocblas_int)Np, &one, (const rocblas_double_complex*)X, (rocblas_int)Np,
                       (const rocblas_double_complex*)Y, (rocblas_int)Np, &zero,
                       (rocblas_double_complex*)G, nx) == rocblas_status_success;
}

bool zgemm_nn(rocblas_handle h, const double2* X, int nx, const double2* C, int ny, long Np,
              double2* Z) {  // Z = X C   (Np x ny)
  const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
  return rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, (rocblas_int)Np, ny, nx,
                       &one, (const rocblas_double_complex*)X, (rocblas_int)Np,
                       (const rocblas_double_complex*)C, nx, &zero, (rocblas_double_complex*)Z,
                       (rocblas_int)Np) == rocblas_status_success;
}

}  // namespace

ovs_status compute_eigentriples(ovs_lattice_s* l, int m, double tol, int max_iter, double2* Rout,
                                double2* Lout, double* lam_out, double* info) {
  const Geometry& g = l->g;
  const long Np = 12L * g.Vs;
  const hipStream_t s = l->stream;
  int nb = std::max(2 * m, m + 16);  // guard vectors beyond the m wanted ones
  nb = (nb + 3) & ~3;
  if (nb > 12L * g.V) return OVS_ERR_ARG;
  if (Np > 0x7fffffffL) return OVS_ERR_ARG;
  const void* links64 = (l->prec == OVS_F64) ? l->links : l->links64;
  if (!links64) return OVS_ERR_STATE;
  Tuning t64;  // FP64 stencil, one source per thread
  const Hop hA = hop_of(l->m_w, l->mu), hAd = hop_of(l->m_w, -l->mu);

  DevMem mem;
  double2* blk[5];
  for (auto& b : blk) {
    b = mem.alloc<double2>((size_t)nb * Np);
    if (!b) return OVS_ERR_ALLOC;
  }
  double2* Gd = mem.alloc<double2>((size_t)nb * nb);
  double2* Cd = mem.alloc<double2>((size_t)nb * nb);
  double2* thd = mem.alloc<double2>(nb);
  double* part = mem.alloc<double>((size_t)nb * 256);
  double* red = mem.alloc<double>(nb);
  // left Ritz vectors kept for the pairing: the m wanted ones and the guard
  // ones after them (a near-degenerate boundary pair can order differently on
  // the two sides)
  const int mkeep = std::min(nb, m + 4);
  double2* Lkeep = mem.alloc<double2>((size_t)mkeep * Np);
  if (!Gd || !Cd || !thd || !part || !red || !Lkeep) return OVS_ERR_ALLOC;

  Handle bh;
  if (rocblas_create_handle(&bh.h) != rocblas_status_success) {
    record_error("rocblas_create_handle", __LINE__, hipErrorUnknown);
    return OVS_ERR_HIP;
  }
  if (rocblas_set_stream(bh.h, s) != rocblas_status_success) return OVS_ERR_HIP;

  auto applyA = [&](const double2* X, double2* Y, int n, bool dag) -> bool {
    return launch_wilson(false, links64, X, Y, n, g, dag ? hAd : hA, false, true, t64, s) == hipSuccess;
  };
  auto norms2 = [&](const double2* X, int n, std::vector<double>& out) -> bool {
    launch_norm2(false, X, Np, n, part, red, s);
    out.resize(n);
    if (hipMemcpyAsync(out.data(), red, sizeof(double) * n, hipMemcpyDeviceToHost, s) != hipSuccess)
      return false;
    return hipStreamSynchronize(s) == hipSuccess;
  };
  auto to_host = [&](const double2* d, int n, std::vector<cd>& h) -> bool {
    h.resize(n);
    if (hipMemcpyAsync(h.data(), d, sizeof(double2) * n, hipMemcpyDeviceToHost, s) != hipSuccess)
      return false;
    return hipStreamSynchronize(s) == hipSuccess;
  };
  auto to_dev = [&](const std::vector<cd>& h, double2* d) -> bool {
    if (hipMemcpyAsync(d, h.data(), sizeof(double2) * h.size(), hipMemcpyHostToDevice, s) != hipSuccess)
      return false;
    return hipStreamSynchronize(s) == hipSuccess;
  };

  // ---- spectral bound b of M = A^2 by power iteration on one field ----
  double b_est = 0.0;
  {
    double2 *x = blk[0], *t = blk[1], *y = blk[2];
    launch_fill_random(x, 1, g, 977, s);
    std::vector<double> nn;
    for (int it = 0; it < 30; ++it) {
      if (!applyA(x, t, 1, false) || !applyA(t, y, 1, false)) return OVS_ERR_HIP;
      if (!norms2(y, 1, nn)) return OVS_ERR_HIP;
      const double ny = std::sqrt(nn[0]);
      if (!(ny > 0)) return OVS_ERR_HIP;
      if (it > 0) b_est = ny;  // x has unit norm from the second iteration on
      launch_cheb(x, y, y, nullptr, 1.0 / ny, 0.0, 0.0, Np, s);
    }
  }
  const double bnd = 1.3 * b_est;

  int passes_total = 0;
  double maxres_all = 0.0;
  std::vector<cd> theta_side[2];
  std::vector<double> nn;
  std::vector<cd> Gh, Ch;

  for (int side = 0; side < 2; ++side) {
    const bool dag = side == 1;
    // pointers into the 5 blocks
    double2* Q = blk[0];
    double2* F[2] = {blk[1], blk[2]};   // free blocks for the filter recurrence
    double2* T1 = blk[3];
    double2* MY = blk[4];
    launch_fill_random(Q, nb, g, 1234567ull + 7919ull * side, s);

    // Cholesky QR, applied twice, of the first n fields of X
    auto orthonormalize = [&](double2*& X, double2*& spare, int n) -> ovs_status {
      for (int rep = 0; rep < 2; ++rep) {
        if (!zgemm_ch(bh.h, X, n, X, n, Np, Gd)) return OVS_ERR_HIP;
        if (!to_host(Gd, n * n, Gh)) return OVS_ERR_HIP;
        if (dense::cholesky(n, Gh.data()) != 0) return OVS_ERR_HIP;
        if (dense::inverse(n, Gh.data()) != 0) return OVS_ERR_HIP;
        if (!to_dev(Gh, Cd)) return OVS_ERR_HIP;
        if (!zgemm_nn(bh.h, X, n, Cd, n, Np, spare)) return OVS_ERR_HIP;
        std::swap(X, spare);
      }
      return OVS_OK;
    };
    // eigen-decomposition of an n x n device matrix, columns sorted by |ev|
    // (ties by Re, Im); writes the sorted eigenvector matrix to Cd
    auto small_ritz = [&](int n, std::vector<cd>& ev) -> ovs_status {
      if (!to_host(Gd, n * n, Gh)) return OVS_ERR_HIP;
      std::vector<cd> lam(n), Y((size_t)n * n);
      if (dense::eig(n, Gh.data(), lam.data(), Y.data()) != 0) return OVS_ERR_HIP;
      std::vector<int> order(n);
      std::iota(order.begin(), order.end(), 0);
      std::sort(order.begin(), order.end(), [&](int i, int j) {
        const double ai = std::abs(lam[i]), aj = std::abs(lam[j]);
        if (ai != aj) return ai < aj;
        if (lam[i].real() != lam[j].real()) return lam[i].real() < lam[j].real();
        return lam[i].imag() < lam[j].imag();
      });
      Ch.assign((size_t)n * n, 0.0);
      ev.resize(n);
      for (int j = 0; j < n; ++j) {
        ev[j] = lam[order[j]];
        for (int i = 0; i < n; ++i) Ch[i + (size_t)n * j] = Y[i + (size_t)n * order[j]];
      }
      return to_dev(Ch, Cd) ? OVS_OK : OVS_ERR_HIP;
    };
    ovs_status st = orthonormalize(Q, F[0], nb);
    if (st != OVS_OK) return st;

    const int mp = std::min(nb, m + 4);  // vectors kept for the final step on A
    double a_cut = bnd / 40.0;
    std::vector<cd> eta, theta;
    double maxres = 1e300;
    const int degree = kFilterDegree;
    for (int pass = 0; pass < max_iter; ++pass) {
      ++passes_total;
      // ---- Chebyshev filter p(M) Q with p(0) = 1 ----
      const double e = 0.5 * (bnd - a_cut), c = 0.5 * (bnd + a_cut);
      const double t0 = -c / e;
      double2* prev = Q;
      double2* cur = F[0];
      double2* next = F[1];
      if (!applyA(prev, T1, nb, dag) || !applyA(T1, MY, nb, dag)) return OVS_ERR_HIP;
      launch_cheb(cur, MY, prev, nullptr, 1.0 / (e * t0), c, 0.0, (long)nb * Np, s);
      double rho = 1.0 / t0;
      for (int k = 1; k < degree; ++k) {
        const double rn = 1.0 / (2.0 * t0 - rho);
        if (!applyA(cur, T1, nb, dag) || !applyA(T1, MY, nb, dag)) return OVS_ERR_HIP;
        launch_cheb(next, MY, cur, prev, 2.0 * rn / e, c, -rho * rn, (long)nb * Np, s);
        rho = rn;
        double2* tmp = prev;
        prev = cur;
        cur = next;
        next = tmp;
      }
      Q = cur;
      F[0] = prev;
      F[1] = next;
      if ((st = orthonormalize(Q, F[0], nb)) != OVS_OK) return st;
      // ---- Rayleigh-Ritz on M = A^2: the wanted values are the extremal ones near 0 ----
      if (!applyA(Q, T1, nb, dag) || !applyA(T1, MY, nb, dag)) return OVS_ERR_HIP;
      if (!zgemm_ch(bh.h, Q, nb, MY, nb, Np, Gd)) return OVS_ERR_HIP;
      if ((st = small_ritz(nb, eta)) != OVS_OK) return st;
      if (!zgemm_nn(bh.h, Q, nb, Cd, nb, Np, F[0])) return OVS_ERR_HIP;
      std::swap(Q, F[0]);
      a_cut = std::min(0.5 * bnd, 1.02 * std::abs(eta[nb - 1]));
      // ---- Rayleigh-Ritz on A in the span of the first mp Ritz vectors of M ----
      double2* S = F[0];
      double2* spare = F[1];
      if (hipMemcpyAsync(S, Q, sizeof(double2) * (size_t)mp * Np, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return OVS_ERR_HIP;
      if ((st = orthonormalize(S, spare, mp)) != OVS_OK) return st;
      double2* W = MY;
      if (!applyA(S, W, mp, dag)) return OVS_ERR_HIP;
      if (!zgemm_ch(bh.h, S, mp, W, mp, Np, Gd)) return OVS_ERR_HIP;
      if ((st = small_ritz(mp, theta)) != OVS_OK) return st;
      double2* Rv = T1;      // Ritz vectors of A
      double2* ARv = spare;  // A times them
      if (!zgemm_nn(bh.h, S, mp, Cd, mp, Np, Rv)) return OVS_ERR_HIP;
      if (!zgemm_nn(bh.h, W, mp, Cd, mp, Np, ARv)) return OVS_ERR_HIP;
      if (!to_dev(theta, thd)) return OVS_ERR_HIP;
      launch_resid(W, ARv, Rv, thd, mp, Np, s);
      if (!norms2(W, mp, nn)) return OVS_ERR_HIP;
      maxres = 0.0;
      for (int j = 0; j < m; ++j)
        maxres = std::max(maxres, std::sqrt(nn[j]) / std::max(std::abs(theta[j]), 1e-12));
      // keep the current best m Ritz vectors of this side
      double2* dst = dag ? Lkeep : Rout;
      if (hipMemcpyAsync(dst, Rv, sizeof(double2) * (size_t)(dag ? mkeep : m) * Np,
                         hipMemcpyDeviceToDevice, s) != hipSuccess)
        return OVS_ERR_HIP;
      if (maxres <= tol) break;
    }
    if (hipStreamSynchronize(s) != hipSuccess) return OVS_ERR_HIP;
    maxres_all = std::max(maxres_all, maxres);
    theta_side[side] = theta;
  }

  // ---- pair left with right (lambda_L = conj(lambda_R)), the left partner
  // of each of the m right Ritz values searched among mkeep left ones ----
  std::vector<int> perm(m, -1);
  std::vector<char> used(mkeep, 0);
  for (int j = 0; j < m; ++j) {
    double best = 1e300;
    int bk = -1;
    for (int k = 0; k < mkeep && k < (int)theta_side[1].size(); ++k) {
      if (used[k]) continue;
      const double d = std::abs(std::conj(theta_side[1][k]) - theta_side[0][j]);
      if (d < best) { best = d; bk = k; }
    }
    perm[j] = bk;
    used[bk] = 1;
  }
  for (int j = 0; j < m; ++j)
    if (hipMemcpyAsync(Lout + (size_t)j * Np, Lkeep + (size_t)perm[j] * Np, sizeof(double2) * Np,
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
      return OVS_ERR_HIP;
  // ---- biorthonormalise: L_b <- L_b (G_bb^H)^{-1}, G = L^H R, clusters b ----
  if (!zgemm_ch(bh.h, Lout, m, Rout, m, Np, Gd)) return OVS_ERR_HIP;
  if (!to_host(Gd, m * m, Gh)) return OVS_ERR_HIP;
  std::vector<cd> X((size_t)m * m, 0.0);
  int i0 = 0;
  while (i0 < m) {
    int i1 = i0 + 1;
    const cd l0 = theta_side[0][i0];
    while (i1 < m && std::abs(theta_side[0][i1] - l0) <= 1e-6 * std::max(1.0, std::abs(l0))) ++i1;
    const int nbk = i1 - i0;
    std::vector<cd> Mb((size_t)nbk * nbk);
    for (int a = 0; a < nbk; ++a)
      for (int bb = 0; bb < nbk; ++bb)  // (G_bb)^H
        Mb[a + (size_t)nbk * bb] = std::conj(Gh[(i0 + bb) + (size_t)m * (i0 + a)]);
    if (dense::inverse(nbk, Mb.data()) != 0) return OVS_ERR_HIP;
    for (int a = 0; a < nbk; ++a)
      for (int bb = 0; bb < nbk; ++bb) X[(i0 + a) + (size_t)m * (i0 + bb)] = Mb[a + (size_t)nbk * bb];
    i0 = i1;
  }
  if (!to_dev(X, Cd)) return OVS_ERR_HIP;
  if (!zgemm_nn(bh.h, Lout, m, Cd, m, Np, blk[0])) return OVS_ERR_HIP;
  if (hipMemcpyAsync(Lout, blk[0], sizeof(double2) * (size_t)m * Np, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return OVS_ERR_HIP;
  if (!zgemm_ch(bh.h, Lout, m, Rout, m, Np, Gd)) return OVS_ERR_HIP;
  if (!to_host(Gd, m * m, Gh)) return OVS_ERR_HIP;
  double dev = 0.0;
  for (int a = 0; a < m; ++a)
    for (int bb = 0; bb < m; ++bb)
      dev = std::max(dev, std::abs(Gh[a + (size_t)m * bb] - (a == bb ? cd(1.0) : cd(0.0))));
  for (int j = 0; j < m; ++j) {
    lam_out[2 * j] = theta_side[0][j].real();
    lam_out[2 * j + 1] = theta_side[0][j].imag();
  }
  info[0] = maxres_all;
  info[1] = dev;
  info[2] = passes_total;
  (void)hipGetLastError();  // rocBLAS may leave a non-fatal status behind
  return OVS_OK;
}

}  // namespace ovs
