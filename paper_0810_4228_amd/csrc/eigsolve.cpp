// Critical eigentriples of A = gamma5 Dw(mu) on the GPU for LR deflation
// (Section 3: right/left eigenvectors of the m eigenvalues of smallest
// magnitude, L^dagger R = I; Section 5 computes them once per configuration).
//
// Method (the paper uses ARPACK on a CPU): shift-and-invert.  The eigenvalues
// of smallest |lambda| of A are those of largest magnitude of A^{-1}, well
// separated from the rest whatever their phase (for mu > 0 they spread into
// the complex plane, where polynomial filters in A or A^2 cannot single them
// out).  Block Krylov-Schur (thick restarts, ordinary Ritz extraction) runs
// on A^{-1}; each application solves A x = y for a block of sources by
// conjugate gradients on the normal equations A^dagger A x = A^dagger y, with
// the multi-source FP64 stencil and per-source coefficients on the device.
// A Rayleigh-Ritz step on A itself in the span of the converged vectors gives
// the eigenvalues and the true residuals.  The same is done with A^dagger =
// A(-mu) for the left vectors, which are then paired by lambda_L =
// conj(lambda_R) and biorthonormalised (blockwise for clusters).  The tall
// skinny products X^H Y and X C are rocBLAS zgemm calls; the small dense
// problems run on the host.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <complex>
#include <numeric>
#include <vector>

#include "dense.h"
#include "ovs_common.h"
#include "ovs_eig.h"
#include "ovs_host.h"
#include "ovs_krylov.h"

namespace ovs {
namespace {

using cd = std::complex<double>;

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
  // m wanted pairs and 4 guard pairs on each side: a near-degenerate pair at
  // the boundary can order differently on the two sides
  // Single-vector Krylov-Schur: blocks would cut the polynomial degree per
  // solve, and with one or two sources the CG step already streams its
  // fields at close to the rate of larger blocks
  const int nev = m + 4;
  const int bs = 1;
  const int ncv = std::max(3 * nev, nev + 8);
  if ((long)ncv + bs >= 12L * g.V) return OVS_ERR_ARG;
  if (Np > 0x7fffffffL) return OVS_ERR_ARG;
  const void* links64 = (l->prec == OVS_F64) ? l->links : l->links64;
  if (!links64) return OVS_ERR_STATE;
  Tuning t64;  // FP64 stencil, one source per thread
  const Hop hA = hop_of(l->m_w, l->mu), hAd = hop_of(l->m_w, -l->mu);
  const bool progress = (l->debug_flags & OVS_DEBUG_PROGRESS) != 0;
  Ranges rg(l, "ovs_deflation_compute");

  DevMem mem;
  // CG work blocks (bs fields each) and the per-side results (nev fields each)
  double2 *cR = mem.alloc<double2>((size_t)bs * Np), *cP = mem.alloc<double2>((size_t)bs * Np);
  double2 *cT = mem.alloc<double2>((size_t)bs * Np), *cW = mem.alloc<double2>((size_t)bs * Np);
  double2 *cX = mem.alloc<double2>((size_t)bs * Np), *cY = mem.alloc<double2>((size_t)bs * Np);
  double2 *vecs = mem.alloc<double2>((size_t)nev * Np), *AS = mem.alloc<double2>((size_t)nev * Np);
  double2 *spare = mem.alloc<double2>((size_t)nev * Np), *Lkeep = mem.alloc<double2>((size_t)nev * Np);
  double2* Gd = mem.alloc<double2>((size_t)nev * nev);
  double2* Cd = mem.alloc<double2>((size_t)nev * nev);
  double2* thd = mem.alloc<double2>(nev);
  // deflation space of the inner solves (below): ns vectors, filtered in a
  // block of nbA
  const int ns = (int)std::min<long>(m + 24, 12L * g.V / 4);
  const int nbA = ns + 16;
  if (nbA >= 12L * g.V) return OVS_ERR_ARG;
  // dot partials for up to max(nev, nbA) vectors
  double* part = mem.alloc<double>((size_t)2 * std::max(nev, nbA) * std::max(cg_nchunk(Np), arn_nchunk(Np)));
  double* red = mem.alloc<double>(nev);
  double* rrd = mem.alloc<double>(2 * bs);
  double* ttd = mem.alloc<double>(bs);
  if (!cR || !cP || !cT || !cW || !cX || !cY || !vecs || !AS || !spare || !Lkeep || !Gd || !Cd || !thd ||
      !part || !red || !rrd || !ttd)
    return OVS_ERR_ALLOC;
  // the stencil writes only lattice sites: pad entries stay zero from here on
  for (double2* b : {cR, cP, cT, cW, cX, cY})
    if (hipMemsetAsync(b, 0, sizeof(double2) * bs * Np, s) != hipSuccess) return OVS_ERR_HIP;
  for (double2* b : {vecs, AS, spare, Lkeep})
    if (hipMemsetAsync(b, 0, sizeof(double2) * nev * Np, s) != hipSuccess) return OVS_ERR_HIP;

  Handle bh;
  if (rocblas_create_handle(&bh.h) != rocblas_status_success) {
    record_error("rocblas_create_handle", __LINE__, hipErrorUnknown);
    return OVS_ERR_HIP;
  }
  if (rocblas_set_stream(bh.h, s) != rocblas_status_success) return OVS_ERR_HIP;

  auto zgemm_ch = [&](const double2* X, int nx, const double2* Y, int ny, double2* G) -> bool {
    launch_gram(X, nx, Y, ny, Np, part, G, s);  // G = X^H Y
    return hipGetLastError() == hipSuccess;
  };
  auto apply = [&](const double2* X, double2* Y, int n, const Hop& h) -> bool {
    return launch_wilson(false, links64, X, Y, n, g, h, false, true, t64, s) == hipSuccess;
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

  // Cholesky QR, applied twice, of the first n fields of X (result in X; tmp
  // holds n fields, Gd and Cd n x n)
  auto orthonormalize = [&](double2* X, int n, double2* tmp, double2* G, double2* C) -> ovs_status {
    std::vector<cd> Gh;
    for (int rep = 0; rep < 2; ++rep) {
      if (!zgemm_ch(X, n, X, n, G)) return OVS_ERR_HIP;
      if (!to_host(G, n * n, Gh)) return OVS_ERR_HIP;
      if (dense::cholesky(n, Gh.data()) != 0) return OVS_ERR_HIP;
      if (dense::inverse(n, Gh.data()) != 0) return OVS_ERR_HIP;
      if (!to_dev(Gh, C)) return OVS_ERR_HIP;
      if (!zgemm_nn(bh.h, X, n, C, n, Np, tmp)) return OVS_ERR_HIP;
      if (hipMemcpyAsync(X, tmp, sizeof(double2) * n * Np, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return OVS_ERR_HIP;
    }
    return OVS_OK;
  };

  // ---- |A| by power iteration on A^dagger A ----
  double anorm = 0.0;
  {
    double2 *x = cR, *t = cT, *y = cW;
    launch_fill_random(x, 1, g, 977, s);
    std::vector<double> nn;
    for (int it = 0; it < 30; ++it) {
      if (!apply(x, t, 1, hA) || !apply(t, y, 1, hAd)) return OVS_ERR_HIP;
      if (!norms2(y, 1, nn)) return OVS_ERR_HIP;
      const double ny = std::sqrt(nn[0]);
      if (!(ny > 0)) return OVS_ERR_HIP;
      if (it > 0) anorm = std::sqrt(ny);  // x has unit norm from the second iteration on
      launch_cheb(x, y, y, nullptr, 1.0 / ny, 0.0, 0.0, Np, s);
    }
  }
  // ---- deflation space of the inner solves: the ns smallest singular
  // triples of A.  Chebyshev-filtered subspace iteration on the Hermitian
  // A^dagger A (spectrum [sigma_min^2, |A|^2] on the real axis, where the
  // filter is sharp) gives the right singular vectors S and sigma^2; the left
  // ones are U = A S / sigma.  CG on A^dagger A x = A^dagger y starts from the
  // part of the solution in span S (and CG on A A^dagger from span U), so its
  // rate is set by sigma_{ns+1} rather than sigma_min.
  std::vector<double> eta(ns);
  double2* Sd = mem.alloc<double2>((size_t)ns * Np);
  double2* Ud = mem.alloc<double2>((size_t)ns * Np);
  double2* cproj = mem.alloc<double2>(ns);
  if (!Sd || !Ud || !cproj) return OVS_ERR_ALLOC;
  int filter_passes = 0;
  rg.phase("singular_subspace");
  {
    DevMem ma;
    double2* blkA[5];
    for (auto& b : blkA) {
      b = ma.alloc<double2>((size_t)nbA * Np);
      if (!b) return OVS_ERR_ALLOC;
      if (hipMemsetAsync(b, 0, sizeof(double2) * nbA * Np, s) != hipSuccess) return OVS_ERR_HIP;
    }
    double2* GA = ma.alloc<double2>((size_t)nbA * nbA);
    double2* CA = ma.alloc<double2>((size_t)nbA * nbA);
    double* partA = ma.alloc<double>((size_t)2 * nbA * std::max(cg_nchunk(Np), arn_nchunk(Np)));
    double* redA = ma.alloc<double>(nbA);
    double2* thA = ma.alloc<double2>(nbA);
    if (!GA || !CA || !partA || !redA || !thA) return OVS_ERR_ALLOC;
    double2 *Q = blkA[0], *F0 = blkA[1], *F1 = blkA[2], *T1 = blkA[3], *MY = blkA[4];
    auto normal = [&](const double2* X, double2* Y) -> bool {  // Y = A^dagger A X
      return apply(X, T1, nbA, hA) && apply(T1, Y, nbA, hAd);
    };
    launch_fill_random(Q, nbA, g, 4242ull, s);
    ovs_status st = orthonormalize(Q, nbA, F0, GA, CA);
    if (st != OVS_OK) return st;
    const double bnd = 1.05 * anorm * anorm;
    double a_cut = bnd / 40.0;
    constexpr int kDegree = 40, kMaxPasses = 60;
    std::vector<cd> Gh, ev(nbA), Y((size_t)nbA * nbA), Ch((size_t)nbA * nbA);
    std::vector<double> nn;
    for (int pass = 0; pass < kMaxPasses; ++pass) {
      ++filter_passes;
      // p(A^dagger A) Q, p the degree-kDegree Chebyshev polynomial of
      // [a_cut, bnd] scaled to p(0) = 1
      const double e = 0.5 * (bnd - a_cut), c = 0.5 * (bnd + a_cut), t0 = -c / e;
      double2 *prev = Q, *cur = F0, *next = F1;
      if (!normal(prev, MY)) return OVS_ERR_HIP;
      launch_cheb(cur, MY, prev, nullptr, 1.0 / (e * t0), c, 0.0, (long)nbA * Np, s);
      double rho = 1.0 / t0;
      for (int k = 1; k < kDegree; ++k) {
        const double rn = 1.0 / (2.0 * t0 - rho);
        if (!normal(cur, MY)) return OVS_ERR_HIP;
        launch_cheb(next, MY, cur, prev, 2.0 * rn / e, c, -rho * rn, (long)nbA * Np, s);
        rho = rn;
        double2* tmp = prev;
        prev = cur;
        cur = next;
        next = tmp;
      }
      Q = cur;
      F0 = prev;
      F1 = next;
      if ((st = orthonormalize(Q, nbA, F0, GA, CA)) != OVS_OK) return st;
      // Rayleigh-Ritz: ascending Ritz values of A^dagger A
      if (!normal(Q, MY)) return OVS_ERR_HIP;
      launch_gram(Q, nbA, MY, nbA, Np, partA, GA, s);
      if (!to_host(GA, nbA * nbA, Gh)) return OVS_ERR_HIP;
      if (dense::eig(nbA, Gh.data(), ev.data(), Y.data()) != 0) return OVS_ERR_HIP;
      std::vector<int> order(nbA);
      std::iota(order.begin(), order.end(), 0);
      std::sort(order.begin(), order.end(), [&](int i, int j) { return ev[i].real() < ev[j].real(); });
      std::vector<cd> th(nbA);
      for (int j = 0; j < nbA; ++j) {
        th[j] = cd(ev[order[j]].real(), 0.0);
        double n2 = 0.0;
        for (int i = 0; i < nbA; ++i) n2 += std::norm(Y[i + (size_t)nbA * order[j]]);
        const double sc = n2 > 0 ? 1.0 / std::sqrt(n2) : 0.0;
        for (int i = 0; i < nbA; ++i) Ch[i + (size_t)nbA * j] = sc * Y[i + (size_t)nbA * order[j]];
      }
      if (!to_dev(Ch, CA)) return OVS_ERR_HIP;
      if (!zgemm_nn(bh.h, Q, nbA, CA, nbA, Np, F0)) return OVS_ERR_HIP;
      if (!zgemm_nn(bh.h, MY, nbA, CA, nbA, Np, F1)) return OVS_ERR_HIP;
      std::swap(Q, F0);
      if (!to_dev(th, thA)) return OVS_ERR_HIP;
      launch_resid(MY, F1, Q, thA, nbA, Np, s);
      launch_norm2(false, MY, Np, ns, partA, redA, s);
      nn.resize(ns);
      if (hipMemcpyAsync(nn.data(), redA, sizeof(double) * ns, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return OVS_ERR_HIP;
      double worst = 0.0;
      for (int j = 0; j < ns; ++j) {
        eta[j] = std::max(th[j].real(), 1e-300);
        worst = std::max(worst, std::sqrt(nn[j]) / eta[j]);
      }
      a_cut = std::min(0.5 * bnd, 1.02 * th[nbA - 1].real());
      if (progress) {
        fprintf(stderr, "ovs eigentriples: singular subspace pass %d: sigma_min %.3e sigma_%d %.3e residual %.2e\n",
                pass + 1, std::sqrt(eta[0]), ns, std::sqrt(eta[ns - 1]), worst);
        fflush(stderr);
      }
      if (worst <= 1e-6) break;
    }
    if (hipMemcpyAsync(Sd, Q, sizeof(double2) * (size_t)ns * Np, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return OVS_ERR_HIP;
    // U = A S diag(1 / sigma)
    if (!apply(Sd, T1, ns, hA)) return OVS_ERR_HIP;
    std::vector<cd> D((size_t)ns * ns, 0.0);
    for (int j = 0; j < ns; ++j) D[j + (size_t)ns * j] = 1.0 / std::sqrt(eta[j]);
    if (!to_dev(D, CA)) return OVS_ERR_HIP;
    if (!zgemm_nn(bh.h, T1, ns, CA, ns, Np, Ud)) return OVS_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return OVS_ERR_HIP;
  }

  // |A x - lambda x| / |lambda| <= |A| |A^{-1} x - x / lambda| for unit x: the
  // outer tolerance on A^{-1}; the inner solves run below it
  const double tol_outer = 0.5 * tol / anorm;
  const double tol_inner = std::max(0.1 * tol, 1e-14);
  constexpr int kCgMax = 100000, kCgCheck = 24, kCgStall = 2000;  // even: graphs of two steps
  long cg_total = 0;
  int cg_fail = 0;
  // x += D diag(1 / eta) D^H r for one field (D = S or U)
  auto project_add = [&](const double2* D, const double2* r, double2* x) -> bool {
    launch_gram(D, ns, r, 1, Np, part, cproj, s);
    std::vector<cd> c;
    if (!to_host(cproj, ns, c)) return false;
    for (int j = 0; j < ns; ++j) c[j] /= eta[j];
    if (!to_dev(c, cproj)) return false;
    const rocblas_double_complex one(1.0, 0.0);
    return rocblas_zgemm(bh.h, rocblas_operation_none, rocblas_operation_none, (rocblas_int)Np, 1, ns,
                         &one, (const rocblas_double_complex*)D, (rocblas_int)Np,
                         (const rocblas_double_complex*)cproj, ns, &one, (rocblas_double_complex*)x,
                         (rocblas_int)Np) == rocblas_status_success;
  };

  // x = M^{-1} y for one source, M = A (hf = hA, deflation space S) or
  // A^dagger (hf = hAd, space U): CG on M^H M x = M^H y from the deflated
  // start, restarted from the true residual with a second projection once it
  // is 1e-5 of the start (rounding brings back the components along D).
  // Two CG steps (parity back to rr[0]) on the fixed work fields, captured
  // once per operator as a HIP graph: at 8^4 a step is a few microseconds of
  // work per launch, so launch overhead would dominate the solve.
  struct CgGraph {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    ~CgGraph() {
      if (x) (void)hipGraphExecDestroy(x);
      if (g) (void)hipGraphDestroy(g);
    }
  } cg_graph[2];
  auto enqueue_two_steps = [&](const Hop& hf, const Hop& hb) -> bool {
    for (int c = 0; c < 2; ++c) {
      if (!apply(cP, cT, 1, hf)) return false;  // t = M p
      launch_norm2(false, cT, Np, 1, part, ttd, s);
      if (!apply(cT, cW, 1, hb)) return false;  // w = M^H t
      launch_cg_xr(cX, cR, cP, cW, rrd + c * bs, ttd, 1, Np, part, s);
      launch_cg_p(cP, cR, rrd + c * bs, rrd + (1 - c) * bs, part, 1, Np, s);
    }
    return true;
  };
  // x = M^{-1} y for one source, M = A (hf = hA, deflation space S) or
  // A^dagger (hf = hAd, space U): CG on M^H M x = M^H y from the deflated
  // start, restarted from the true residual with a second projection once it
  // is 1e-5 of the start (rounding brings back the components along D).
  // y is copied to cY and the iterate lives in cX (the graph's fields).
  auto solve = [&](const double2* Y, double2* X, int n, const Hop& hf, const Hop& hb,
                   const double2* D, CgGraph& cg) -> ovs_status {
    if (n != 1) return OVS_ERR_ARG;
    std::vector<double> yy, res;
    if (hipMemcpyAsync(cY, Y, sizeof(double2) * Np, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return OVS_ERR_HIP;
    if (!norms2(cY, 1, yy)) return OVS_ERR_HIP;
    if (hipMemsetAsync(cX, 0, sizeof(double2) * Np, s) != hipSuccess) return OVS_ERR_HIP;
    if (!to_dev(std::vector<cd>(1, cd(1.0)), thd)) return OVS_ERR_HIP;  // theta = 1: resid = a - b
    if (!apply(cY, cW, 1, hb)) return OVS_ERR_HIP;  // b = M^H y (kept in cW until the first step)
    if (!project_add(D, cW, cX)) return OVS_ERR_HIP;
    // r = b - M^H M x, p = r
    auto restart = [&]() -> bool {
      if (!apply(cX, cT, 1, hf)) return false;
      launch_resid(cP, cY, cT, thd, 1, Np, s);  // y - M x
      if (!apply(cP, cR, 1, hb)) return false;  // r = M^H (y - M x)
      if (hipMemcpyAsync(cP, cR, sizeof(double2) * Np, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return false;
      launch_norm2(false, cR, Np, 1, part, rrd, s);
      return true;
    };
    if (!restart()) return OVS_ERR_HIP;
    if (!cg.x) {
      if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return OVS_ERR_HIP;
      const bool ok = enqueue_two_steps(hf, hb);
      const hipError_t ce = hipStreamEndCapture(s, &cg.g);
      if (!ok || ce != hipSuccess) return OVS_ERR_HIP;
      if (hipGraphInstantiate(&cg.x, cg.g, nullptr, nullptr, 0) != hipSuccess) return OVS_ERR_HIP;
    }
    int nproj = 1;
    double best = 1e300;
    int best_it = 0;
    for (int it = 2; it <= kCgMax; it += 2) {
      if (hipGraphLaunch(cg.x, s) != hipSuccess) return OVS_ERR_HIP;
      if (it % kCgCheck == 0 || it == kCgMax) {  // true residual y - M x
        if (!apply(cX, cT, 1, hf)) return OVS_ERR_HIP;
        launch_resid(cW, cT, cY, thd, 1, Np, s);
        if (!norms2(cW, 1, res)) return OVS_ERR_HIP;
        const double rel = std::sqrt(res[0] / yy[0]);
        const bool done = rel <= tol_inner;
        if (rel < 0.5 * best) {
          best = rel;
          best_it = it;
        }
        const bool stalled = it - best_it >= kCgStall;
        if (done || stalled || it == kCgMax) {
          cg_total += it;
          if (!done && rel > 10.0 * tol_inner) ++cg_fail;
          if (progress) {
            fprintf(stderr, "ovs eigentriples: solve: %d CG iterations, residual %.2e\n", it, rel);
            fflush(stderr);
          }
          if (hipMemcpyAsync(X, cX, sizeof(double2) * Np, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return OVS_ERR_HIP;
          return OVS_OK;
        }
        if (nproj == 1 && rel <= 1e-5) {  // second projection from the current residual
          if (!project_add(D, cR, cX) || !restart()) return OVS_ERR_HIP;
          nproj = 2;
        }
      }
    }
    return OVS_OK;
  };

  int restarts_total = 0;
  double maxres_all = 0.0;
  bool unconverged = false;
  std::vector<cd> theta_side[2];
  std::vector<double> res_side[2];
  for (int side = 0; side < 2; ++side) {
    rg.phase(side ? "krylov_schur_left" : "krylov_schur_right");
    const Hop& hf = side ? hAd : hA;
    const Hop& hb = side ? hA : hAd;
    KrylovOptions ko;
    ko.field_len = Np;
    ko.largest = true;
    ko.nconv = m;  // a left partner among the guards (ties in |lambda|) is checked below
    ko.start = [&](void* b, int n) { launch_fill_random((double2*)b, n, g, 1234567ull + 7919ull * side, s); };
    if (progress)
      ko.progress = [&](int rs, double worst, int nmv) {
        fprintf(stderr, "ovs eigentriples: side %d cycle %d residual(A^-1) %.3e solves %d CG iterations %ld\n",
                side, rs + 1, worst, nmv, cg_total);
        fflush(stderr);
      };
    const BlockOp op = [&](const void* in, void* out, int n, int*) -> ovs_status {
      return solve((const double2*)in, (double2*)out, n, hf, hb, side ? Ud : Sd, cg_graph[side]);
    };
    std::vector<double> lam_inv(2 * nev);
    double kinfo[4] = {0, 0, 0, 0};
    ovs_status st = block_krylov_eigs(l, op, nev, ncv, bs, tol_outer, max_iter, lam_inv.data(),
                                      vecs, kinfo, ko);
    if (st != OVS_OK && st != OVS_WARN_NOT_CONVERGED) return st;  // no vectors
    restarts_total += (int)kinfo[1];
    // ---- Rayleigh-Ritz on M in the span of the nev vectors ----
    if ((st = orthonormalize(vecs, nev, spare, Gd, Cd)) != OVS_OK) return st;
    if (!apply(vecs, AS, nev, hf)) return OVS_ERR_HIP;
    if (!zgemm_ch(vecs, nev, AS, nev, Gd)) return OVS_ERR_HIP;
    std::vector<cd> Gh, lam(nev), Y((size_t)nev * nev), Ch((size_t)nev * nev);
    if (!to_host(Gd, nev * nev, Gh)) return OVS_ERR_HIP;
    if (dense::eig(nev, Gh.data(), lam.data(), Y.data()) != 0) return OVS_ERR_HIP;
    std::vector<int> order(nev);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int i, int j) {
      const double ai = std::abs(lam[i]), aj = std::abs(lam[j]);
      if (ai != aj) return ai < aj;
      if (lam[i].real() != lam[j].real()) return lam[i].real() < lam[j].real();
      return lam[i].imag() < lam[j].imag();
    });
    std::vector<cd> theta(nev);
    for (int j = 0; j < nev; ++j) {
      theta[j] = lam[order[j]];
      double n2 = 0.0;
      for (int i = 0; i < nev; ++i) n2 += std::norm(Y[i + (size_t)nev * order[j]]);
      const double sc = n2 > 0 ? 1.0 / std::sqrt(n2) : 0.0;  // unit Ritz vectors
      for (int i = 0; i < nev; ++i) Ch[i + (size_t)nev * j] = sc * Y[i + (size_t)nev * order[j]];
    }
    if (!to_dev(Ch, Cd)) return OVS_ERR_HIP;
    double2* Rv = side ? Lkeep : spare;
    if (!zgemm_nn(bh.h, vecs, nev, Cd, nev, Np, Rv)) return OVS_ERR_HIP;
    if (!zgemm_nn(bh.h, AS, nev, Cd, nev, Np, vecs)) return OVS_ERR_HIP;  // M Rv
    if (!to_dev(theta, thd)) return OVS_ERR_HIP;
    launch_resid(AS, vecs, Rv, thd, nev, Np, s);
    std::vector<double> nn;
    if (!norms2(AS, nev, nn)) return OVS_ERR_HIP;
    std::vector<double>& rs = res_side[side];
    rs.resize(nev);
    for (int j = 0; j < nev; ++j) rs[j] = std::sqrt(nn[j]) / std::max(std::abs(theta[j]), 1e-300);
    double maxres = 0.0;
    for (int j = 0; j < m; ++j) maxres = std::max(maxres, rs[j]);
    if (progress) {
      fprintf(stderr, "ovs eigentriples: side %d done, Krylov-Schur status %d, residual(A) %.3e, CG iterations %ld\n",
              side, (int)st, maxres, cg_total);
      fflush(stderr);
    }
    if (side == 0 &&
        hipMemcpyAsync(Rout, Rv, sizeof(double2) * (size_t)m * Np, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return OVS_ERR_HIP;
    if (side == 0) maxres_all = maxres;
    if (st != OVS_OK || cg_fail) unconverged = true;
    theta_side[side] = theta;
  }
  if (hipStreamSynchronize(s) != hipSuccess) return OVS_ERR_HIP;
  rg.phase("pairing");
  const int mkeep = nev;
  std::vector<cd> Gh;

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
    maxres_all = std::max(maxres_all, res_side[1][bk]);
  }
  if (unconverged) maxres_all = std::max(maxres_all, 2.0 * tol);  // flags the result
  for (int j = 0; j < m; ++j)
    if (hipMemcpyAsync(Lout + (size_t)j * Np, Lkeep + (size_t)perm[j] * Np, sizeof(double2) * Np,
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
      return OVS_ERR_HIP;
  // ---- biorthonormalise: L <- L (G^H)^{-1}, G = L^H R, so that L^H R = I to
  // rounding (the deflation projector 1 - R L^H is then exactly idempotent);
  // the left residuals are measured again afterwards ----
  if (!zgemm_ch(Lout, m, Rout, m, Gd)) return OVS_ERR_HIP;
  if (!to_host(Gd, m * m, Gh)) return OVS_ERR_HIP;
  std::vector<cd> X((size_t)m * m);
  for (int a = 0; a < m; ++a)
    for (int bb = 0; bb < m; ++bb) X[a + (size_t)m * bb] = std::conj(Gh[bb + (size_t)m * a]);
  if (dense::inverse(m, X.data()) != 0) return OVS_ERR_HIP;
  if (!to_dev(X, Cd)) return OVS_ERR_HIP;
  if (!zgemm_nn(bh.h, Lout, m, Cd, m, Np, spare)) return OVS_ERR_HIP;
  if (hipMemcpyAsync(Lout, spare, sizeof(double2) * (size_t)m * Np, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return OVS_ERR_HIP;
  if (!zgemm_ch(Lout, m, Rout, m, Gd)) return OVS_ERR_HIP;
  if (!to_host(Gd, m * m, Gh)) return OVS_ERR_HIP;
  double dev = 0.0;
  for (int a = 0; a < m; ++a)
    for (int bb = 0; bb < m; ++bb)
      dev = std::max(dev, std::abs(Gh[a + (size_t)m * bb] - (a == bb ? cd(1.0) : cd(0.0))));
  {  // |A^dagger l_j - conj(lambda_j) l_j| / (|lambda_j| |l_j|) of the final L
    if (!apply(Lout, AS, m, hAd)) return OVS_ERR_HIP;
    std::vector<cd> th(m);
    for (int j = 0; j < m; ++j) th[j] = std::conj(theta_side[0][j]);
    if (!to_dev(th, thd)) return OVS_ERR_HIP;
    launch_resid(vecs, AS, Lout, thd, m, Np, s);
    std::vector<double> nr, nl;
    if (!norms2(vecs, m, nr) || !norms2(Lout, m, nl)) return OVS_ERR_HIP;
    for (int j = 0; j < m; ++j)
      maxres_all = std::max(maxres_all, std::sqrt(nr[j] / nl[j]) / std::abs(theta_side[0][j]));
  }
  for (int j = 0; j < m; ++j) {
    lam_out[2 * j] = theta_side[0][j].real();
    lam_out[2 * j + 1] = theta_side[0][j].imag();
  }
  info[0] = maxres_all;
  info[1] = dev;
  info[2] = restarts_total;
  (void)filter_passes;
  (void)hipGetLastError();  // rocBLAS may leave a non-fatal status behind
  return OVS_OK;
}

}  // namespace ovs
