// Krylov-side kernels: LR deflation (Section 3), the two-sided Lanczos update
// and coefficient steps (Section 4), the Arnoldi Gram-Schmidt steps
// (Section 2), the combination |b_R| V_k x (eq. 2sLapp / Arnapp) and the
// inner sign sgn(T) e_1 of the small projected matrix.
//
// All inner products and norms accumulate in FP64 and are reduced in a fixed
// order (per-workgroup partials, then one pass over the partials), so results
// are bitwise repeatable from run to run.
#include <algorithm>

#include "ovs_common.h"
#include "ovs_device.h"
#include "ovs_krylov.h"
#include "ovs_lanczos.h"

namespace ovs {

static inline int cdiv_i(long a, long b) { return (int)((a + b - 1) / b); }

// ===========================================================================
// Generic fixed-order reduction of per-workgroup partials.
// partials: [nslots][nparts][nv]; out: [nslots][nv].  One workgroup per slot.
// ===========================================================================
template <int NV>
__global__ void __launch_bounds__(256) k_reduce_partials(const double* __restrict__ partials,
                                                         int nparts, double* __restrict__ out) {
  __shared__ double lds[4 * NV];
  const long slot = blockIdx.x;
  double v[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) v[j] = 0.0;
  for (int p = threadIdx.x; p < nparts; p += blockDim.x) {
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] += partials[(slot * nparts + p) * NV + j];
  }
  block_sum<NV>(v, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) out[slot * NV + j] = v[j];
  }
}

// ===========================================================================
// LR deflation (Section 3 and eq. 2sLapp):
//   C = L^dag b, D = R^dag b, b_R = b - R C, b_L = b - L D, y_ex = R sgn(Lam) C
// ===========================================================================
constexpr int kDeflRhs = 8;  // sources per thread in the dot kernel

// partials [m][nrhs][nchunk][4] = (C.re, C.im, D.re, D.im)
__global__ void __launch_bounds__(256) k_defl_dots(const double2* __restrict__ R,
                                                   const double2* __restrict__ L,
                                                   const double2* __restrict__ B, int nrhs, long N,
                                                   int nchunk, double* __restrict__ partials) {
  __shared__ double lds[4 * 4 * kDeflRhs];
  const int j = blockIdx.y;
  const int r0 = blockIdx.z * kDeflRhs;
  const int nr = min(kDeflRhs, nrhs - r0);
  double v[4 * kDeflRhs];
#pragma unroll
  for (int q = 0; q < 4 * kDeflRhs; ++q) v[q] = 0.0;
  const double2* Rj = R + (long)j * N;
  const double2* Lj = L + (long)j * N;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N; e += (long)gridDim.x * blockDim.x) {
    const Cx<double> rr = c64(Rj[e]), ll = c64(Lj[e]);
#pragma unroll
    for (int q = 0; q < kDeflRhs; ++q) {
      if (q < nr) {
        const Cx<double> bb = c64(B[(long)(r0 + q) * N + e]);
        const Cx<double> c = cmulc(ll, bb), d = cmulc(rr, bb);
        v[4 * q + 0] += c.re;
        v[4 * q + 1] += c.im;
        v[4 * q + 2] += d.re;
        v[4 * q + 3] += d.im;
      }
    }
  }
  block_sum<4 * kDeflRhs>(v, lds);
  if (threadIdx.x == 0) {
    // compile-time bounds keep v[] in registers (a runtime bound indexes it
    // dynamically, which puts it in scratch memory)
#pragma unroll
    for (int q = 0; q < kDeflRhs; ++q)
      if (q < nr)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          partials[(((long)j * nrhs + r0 + q) * nchunk + blockIdx.x) * 4 + t] = v[4 * q + t];
  }
}

// CD: [m][nrhs][4] reduced (C, D); sgn: [m] sign of Re lambda.
__global__ void __launch_bounds__(256) k_defl_axpy(const double2* __restrict__ R,
                                                   const double2* __restrict__ L,
                                                   const double2* __restrict__ B,
                                                   const double* __restrict__ CD,
                                                   const double* __restrict__ sgn, int m, int nrhs,
                                                   long N, double2* __restrict__ bR,
                                                   double2* __restrict__ bL,
                                                   double2* __restrict__ yex) {
  const int r = blockIdx.y;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N; e += (long)gridDim.x * blockDim.x) {
    const Cx<double> b = c64(B[(long)r * N + e]);
    Cx<double> pr = {0, 0}, pl = {0, 0}, py = {0, 0};
    for (int j = 0; j < m; ++j) {
      const double* cd = CD + ((long)j * nrhs + r) * 4;
      const Cx<double> c = {cd[0], cd[1]}, d = {cd[2], cd[3]};
      const Cx<double> rr = c64(R[(long)j * N + e]), ll = c64(L[(long)j * N + e]);
      pr = cfma(rr, c, pr);
      pl = cfma(ll, d, pl);
      if (yex) py = cfma(rr, scale(sgn[j], c), py);
    }
    if (bR) bR[(long)r * N + e] = d2(b - pr);
    if (bL) bL[(long)r * N + e] = d2(b - pl);
    if (yex) yex[(long)r * N + e] = d2(py);
  }
}

// D[j][r] -= kappa[r][j] (the bL output of k_defl_axpy then gains + L kappa)
__global__ void k_cd_shift(double* __restrict__ CD, const double2* __restrict__ kappa, int m,
                           int nrhs) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * nrhs) return;
  const int j = e / nrhs, r = e % nrhs;
  const double2 k = kappa[(long)r * m + j];
  CD[(long)e * 4 + 2] -= k.x;
  CD[(long)e * 4 + 3] -= k.y;
}

// per-source partials of |b_R|^2 and b_L^dag b_R: [nrhs][nchunk][3]
__global__ void __launch_bounds__(256) k_start_dots(const double2* __restrict__ bR,
                                                    const double2* __restrict__ bL, long N,
                                                    int nchunk, double* __restrict__ partials) {
  __shared__ double lds[4 * 3];
  const int r = blockIdx.y;
  double v[3] = {0, 0, 0};
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N; e += (long)gridDim.x * blockDim.x) {
    const Cx<double> a = c64(bR[(long)r * N + e]), l = c64(bL[(long)r * N + e]);
    v[0] += cnorm2(a);
    const Cx<double> s = cmulc(l, a);
    v[1] += s.re;
    v[2] += s.im;
  }
  block_sum<3>(v, lds);
  if (threadIdx.x == 0)
    for (int t = 0; t < 3; ++t) partials[((long)r * nchunk + blockIdx.x) * 3 + t] = v[t];
}

// Start vectors v_1 = b_R / n_b, w_1 = b_L n_b / conj(sigma) (stored in
// storage precision) from sums[r] = (|b_R|^2, sigma.re, sigma.im).
template <typename T2>
__global__ void k_start_vectors(const double2* __restrict__ bR, const double2* __restrict__ bL,
                                const double* __restrict__ sums, long N, T2* __restrict__ V0,
                                T2* __restrict__ W0) {
  const int r = blockIdx.y;
  const double nb = sqrt(sums[r * 3 + 0]);
  const Cx<double> sig = {sums[r * 3 + 1], sums[r * 3 + 2]};
  const double inv = nb > 0 ? 1.0 / nb : 0.0;
  Cx<double> fw = {0, 0};
  if (nb > 0 && (sig.re != 0 || sig.im != 0)) fw = cdiv(Cx<double>{nb, 0}, Cx<double>{sig.re, -sig.im});
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N; e += (long)gridDim.x * blockDim.x) {
    if (V0) st64(V0 + (long)r * N + e, scale(inv, c64(bR[(long)r * N + e])));
    if (W0) st64(W0 + (long)r * N + e, cmul(fw, c64(bL[(long)r * N + e])));
  }
}

// ===========================================================================
// Two-sided Lanczos coefficient steps (Section 4).  The iteration index lives
// in device memory (*it) so a captured chunk of iterations can be replayed.
// ===========================================================================

// ---- per-step kernels (bodies in ovs_lanczos.h) ----------------------------

__global__ void __launch_bounds__(256) k_alpha(const double* __restrict__ partials, int nparts,
                                               CoefArrays co, const int* __restrict__ it,
                                               const int* __restrict__ rhs_map,
                                               const int* __restrict__ n_active) {
  alpha_body(blockIdx.x, *it, partials, nparts, co, rhs_map, *n_active);
}

template <typename T2>
__global__ void __launch_bounds__(256) k_update(const T2* __restrict__ T, const T2* __restrict__ S,
                                                T2* __restrict__ basis, long basis_stride,
                                                T2* __restrict__ wbuf, long slot_stride, long N,
                                                CoefArrays co, const int* __restrict__ it,
                                                const int* __restrict__ rhs_map,
                                                const int* __restrict__ n_active,
                                                double* __restrict__ partials, int two_pass_ring,
                                                const double* __restrict__ apart, int anparts,
                                                int nt) {
  update_body<T2>(blockIdx.x, blockIdx.y, gridDim.x, *it, T, S, basis, basis_stride, wbuf,
                  slot_stride, N, co, rhs_map, *n_active, partials, two_pass_ring, apart, anparts,
                  nt);
}

// beta_body for one source slot per workgroup, then the iteration advance:
// the last workgroup to finish (a ticket counter, reset by that workgroup, so
// it is zero between launches) increments *it, after every workgroup has read it.
template <typename T2>
__global__ void __launch_bounds__(256) k_beta_tail(const double* __restrict__ partials, int nparts,
                                                   CoefArrays co, int* __restrict__ it,
                                                   const int* __restrict__ rhs_map,
                                                   const int* __restrict__ n_active,
                                                   int* __restrict__ ticket,
                                                   const T2* __restrict__ basis, long basis_stride,
                                                   long N, int ring, const int* __restrict__ idx,
                                                   int P, double2* __restrict__ probes) {
  const int i = *it;
  beta_body<T2>(blockIdx.x, i, partials, nparts, co, rhs_map, *n_active, basis, basis_stride, N,
                ring, idx, P, probes);
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(ticket, 1) == (int)gridDim.x - 1) {
      *ticket = 0;
      *it = i + 1;
    }
  }
}

// Probe sketch for the convergence estimate: the entries idx[0..P) of the
// stored Lanczos vector V~_j (j = *it + 1, or j = 0 before the first step) of
// every active source are copied to probes[slot][j][P] in FP64.
template <typename T2>
__global__ void __launch_bounds__(256) k_probe_gather(const T2* __restrict__ basis, long basis_stride,
                                                      long N, int ring, const int* __restrict__ it,
                                                      int first, const int* __restrict__ idx, int P,
                                                      int kmax, const int* __restrict__ rhs_map,
                                                      const int* __restrict__ n_active,
                                                      double2* __restrict__ probes) {
  const int jj = blockIdx.y;
  if (jj >= *n_active) return;
  const int slot = rhs_map[jj];
  const int j = first ? 0 : *it + 1;
  if (j >= kmax) return;
  const long sl = ring ? (j % 3) : j;
  const T2* v = basis + sl * basis_stride + (long)slot * N;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x)
    probes[((long)slot * kmax + j) * P + p] = d2(ld64(v + idx[p]));
}

// yp[r][p] = yex[r][idx[p]] + sum_{i < k_r} coef[r][i] probes[r][i][p]
__global__ void __launch_bounds__(256) k_probe_y(const double2* __restrict__ probes,
                                                 const double2* __restrict__ coef,
                                                 const int* __restrict__ kvec, int kmax,
                                                 const double2* __restrict__ yex, long N,
                                                 const int* __restrict__ idx, int P,
                                                 double2* __restrict__ yp) {
  const int r = blockIdx.y;
  const int k = kvec[r];
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
    Cx<double> acc = yex ? c64(yex[(long)r * N + idx[p]]) : Cx<double>{0, 0};
    const double2* cr = coef + (long)r * kmax;
    const double2* pr = probes + (long)r * kmax * P + p;
    // the same sequential sum as one term per step, with the loads of eight
    // terms issued before their multiply-adds (one thread's loop is otherwise
    // a chain of dependent memory latencies)
    int i = 0;
    for (; i + 8 <= k; i += 8) {
      Cx<double> c[8], q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        c[u] = c64(cr[i + u]);
        q[u] = c64(pr[(long)(i + u) * P]);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = cfma(c[u], q[u], acc);
    }
    for (; i < k; ++i) acc = cfma(c64(cr[i]), c64(pr[(long)i * P]), acc);
    yp[(long)r * P + p] = d2(acc);
  }
}

__global__ void k_advance(int* it) { *it += 1; }

// ===========================================================================
// Combination y = y_ex + sum_i coef_i V~_i   (coef_i = n_b x_i sv_i)
// ===========================================================================
template <typename T2>
__global__ void __launch_bounds__(256) k_combine(const T2* __restrict__ basis, long basis_stride,
                                                 long N, const double2* __restrict__ coef, int kmax,
                                                 const int* __restrict__ kused,
                                                 const double2* __restrict__ yex,
                                                 double2* __restrict__ y) {
  const int r = blockIdx.y;
  const int kr = kused[r];
  const double2* cr = coef + (long)r * kmax;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N; e += (long)gridDim.x * blockDim.x) {
    Cx<double> acc = yex ? c64(yex[(long)r * N + e]) : Cx<double>{0, 0};
    const T2* br = basis + (long)r * N + e;
    // the same sequential sum as one term per step, with the loads of eight
    // basis vectors issued before their multiply-adds: one load in flight per
    // wave would leave the sweep over the k_used stored vectors latency-bound
    int i = 0;
    for (; i + 8 <= kr; i += 8) {
      Cx<double> q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) q[u] = ld64(br + (long)(i + u) * basis_stride);
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = cfma(c64(cr[i + u]), q[u], acc);
    }
    for (; i < kr; ++i) acc = cfma(c64(cr[i]), ld64(br + (long)i * basis_stride), acc);
    y[(long)r * N + e] = d2(acc);
  }
}

// coef[r][i] = n_b x[r][i] sv[r][i] for i < kused[r], else 0
__global__ void k_make_coef(const double2* __restrict__ x, const double* __restrict__ sv,
                            const double* __restrict__ nb, int kmax, int nrhs,
                            double2* __restrict__ coef) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)nrhs * kmax) return;
  const long r = e / kmax, i = e % kmax;
  coef[e] = d2(scale(nb[r] * (sv ? sv[r * (kmax + 1) + i] : 1.0), c64(x[e])));
}

// Second pass of the small-memory evaluation: replay v_{i+1} from the stored
// coefficients (identical arithmetic to k_update) and accumulate y.
template <typename T2>
__global__ void __launch_bounds__(256) k_replay(const T2* __restrict__ T, T2* __restrict__ ring,
                                                long ring_stride, long N, CoefArrays co, int i,
                                                const double2* __restrict__ coef,
                                                const int* __restrict__ kused,
                                                double2* __restrict__ y) {
  const int r = blockIdx.y;
  const int kr = kused[r];
  if (i >= kr) return;
  const long ks = co.kmax;
  const bool prev = i > 0;
  const bool next = i + 1 < kr;
  const Cx<double> a = c64(co.alpha[r * ks + i]);
  const double svi = co.sv[r * (ks + 1) + i];
  const double svm = prev ? co.sv[r * (ks + 1) + i - 1] : 0.0;
  const Cx<double> gm = prev ? c64(co.gamma[r * ks + i - 1]) : Cx<double>{0, 0};
  const Cx<double> c1 = {svi, 0.0};
  const Cx<double> c2 = scale(-svi, a);
  const Cx<double> c3 = scale(-svm, gm);
  const Cx<double> ci = c64(coef[r * ks + i]);
  const T2* Vi = ring + (long)(i % 3) * ring_stride + (long)r * N;
  const T2* Vm = ring + (long)((i + 2) % 3) * ring_stride + (long)r * N;
  T2* Vn = ring + (long)((i + 1) % 3) * ring_stride + (long)r * N;
  const T2* Ts = T + (long)r * N;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N; e += (long)gridDim.x * blockDim.x) {
    const Cx<double> vi = ld64(Vi + e);
    y[(long)r * N + e] = d2(cfma(ci, vi, c64(y[(long)r * N + e])));
    if (next) {
      Cx<double> vt = cmul(c1, ld64(Ts + e));
      vt = cfma(c2, vi, vt);
      if (prev) vt = cfma(c3, ld64(Vm + e), vt);
      st64(Vn + e, vt);
    }
  }
}

// y <- b + gamma5 y  (D_ov b, eq. (1.1)); fields [nrhs][12][V] FP64
__global__ void k_overlap(const double2* __restrict__ b, double2* __restrict__ y, long N, int V) {
  // V: the padded plane stride Vs; component c of offset e (layout of fidx)
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N; e += (long)gridDim.x * blockDim.x) {
    const long loc = e % (12L * V);
    const int c = (int)(2 * ((loc >> 1) / V) + (loc & 1));
    Cx<double> v = c64(y[e]);
    if (c >= 6) v = -v;
    y[e] = d2(c64(b[e]) + v);
  }
}

// ===========================================================================
// Arnoldi (Section 2): classical Gram-Schmidt applied twice.
// ===========================================================================
constexpr int kArnVec = 8;  // basis vectors per workgroup in the dot kernel

// partials [nrhs][nvec][nchunk][2] of v_i^dag t, i < nvec
template <typename T2>
__global__ void __launch_bounds__(256) k_block_dots(const T2* __restrict__ basis, long basis_stride,
                                                    const T2* __restrict__ T, long N, int nvec,
                                                    int nchunk, double* __restrict__ partials) {
  __shared__ double lds[4 * 2 * kArnVec];
  const int r = blockIdx.y;
  const int i0 = blockIdx.z * kArnVec;
  const int ni = min(kArnVec, nvec - i0);
  double v[2 * kArnVec];
#pragma unroll
  for (int q = 0; q < 2 * kArnVec; ++q) v[q] = 0.0;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N; e += (long)gridDim.x * blockDim.x) {
    const Cx<double> t = ld64(T + (long)r * N + e);
#pragma unroll
    for (int q = 0; q < kArnVec; ++q) {
      if (q < ni) {
        const Cx<double> p = cmulc(ld64(basis + (i0 + q) * basis_stride + (long)r * N + e), t);
        v[2 * q] += p.re;
        v[2 * q + 1] += p.im;
      }
    }
  }
  block_sum<2 * kArnVec>(v, lds);
  if (threadIdx.x == 0)
    for (int q = 0; q < ni; ++q)
      for (int t = 0; t < 2; ++t)
        partials[(((long)r * nvec + i0 + q) * nchunk + blockIdx.x) * 2 + t] = v[2 * q + t];
}

// H[r][j][i] += h_i (column-major: column j of H_r), hcur[r][i] = h_i
__global__ void k_arn_accum(const double* __restrict__ red, int nvec, int kmax, int j, int first,
                            double2* __restrict__ H, double2* __restrict__ hcur, int nrhs) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nrhs * nvec) return;
  const int r = e / nvec, i = e % nvec;
  const Cx<double> h = {red[(long)e * 2], red[(long)e * 2 + 1]};
  double2* hij = H + ((long)r * kmax + j) * kmax + i;
  *hij = first ? d2(h) : d2(c64(*hij) + h);
  hcur[(long)r * kmax + i] = d2(h);
}

// T -= sum_i hcur_i V_i ; partials of |T|^2 [nrhs][nchunk]
template <typename T2>
__global__ void __launch_bounds__(256) k_block_axpy(const T2* __restrict__ basis, long basis_stride,
                                                    T2* __restrict__ T, long N, int nvec,
                                                    const double2* __restrict__ hcur, int kmax,
                                                    double* __restrict__ partials) {
  __shared__ double lds[4];
  const int r = blockIdx.y;
  double v[1] = {0.0};
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N; e += (long)gridDim.x * blockDim.x) {
    Cx<double> t = ld64(T + (long)r * N + e);
    for (int i = 0; i < nvec; ++i)
      t = t - cmul(c64(hcur[(long)r * kmax + i]), ld64(basis + i * basis_stride + (long)r * N + e));
    st64(T + (long)r * N + e, t);
    v[0] += cnorm2(round_to(T, t));
  }
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) partials[(long)r * gridDim.x + blockIdx.x] = v[0];
}

// H[j+1][j] = |t| and scl = 1/|t|; lucky breakdown |t| <= 1e-14 |A v_j| stops
// the source at k = j+1 (scl = 0 from then on).
__global__ void k_arn_sub(const double* __restrict__ red_n, const double* __restrict__ red_tn,
                          double2* __restrict__ H, int kmax, int j, double* __restrict__ scl,
                          int* __restrict__ kstop, int* __restrict__ status, int nrhs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  double2* hsub = H + ((long)r * kmax + j) * kmax + (j + 1);
  if (status[r] != 0) {
    scl[r] = 0.0;
    *hsub = make_double2(0.0, 0.0);
    return;
  }
  const double h = sqrt(red_n[r]), tn = sqrt(red_tn[r]);
  if (!(h > 1e-14 * tn)) {
    status[r] = 1;
    kstop[r] = j + 1;
    scl[r] = 0.0;
    *hsub = make_double2(0.0, 0.0);
  } else {
    scl[r] = 1.0 / h;
    *hsub = make_double2(h, 0.0);
  }
}

// partials of |T|^2 [nrhs][nchunk]
template <typename T2>
__global__ void __launch_bounds__(256) k_norm2(const T2* __restrict__ T, long N,
                                               double* __restrict__ partials) {
  __shared__ double lds[4];
  const int r = blockIdx.y;
  double v[1] = {0.0};
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N; e += (long)gridDim.x * blockDim.x)
    v[0] += cnorm2(ld64(T + (long)r * N + e));
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) partials[(long)r * gridDim.x + blockIdx.x] = v[0];
}

// V_{j+1} = T / h, h = |T| (scale[r] = 1/h or 0 after breakdown)
template <typename T2>
__global__ void k_scale_copy(const T2* __restrict__ T, T2* __restrict__ out, long N,
                             const double* __restrict__ scl) {
  const int r = blockIdx.y;
  const double s = scl[r];
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N; e += (long)gridDim.x * blockDim.x)
    st64(out + (long)r * N + e, scale(s, ld64(T + (long)r * N + e)));
}

// ===========================================================================
// Inner sign: x = sgn(T) e_1 for a small non-Hermitian T with no eigenvalue
// on the imaginary axis, from sgn(z) = (1/pi) int_0^inf [1/(z+i tau) +
// 1/(z-i tau)] d tau, tau = e^u, trapezoidal rule in u:
//   x ~= (h/pi) sum_n e^{u_n} [ (T + i e^{u_n})^{-1} e_1 + (T - i e^{u_n})^{-1} e_1 ].
// The nodes with even n form the rule with step 2h; their difference gives
// the error estimate.  Each shifted solve (T + i sigma) y = e_1 eliminates the
// subdiagonal from the bottom up by column operations with column pivoting:
// M P E = R upper triangular, so y = P E e_1 / R_00 with P E stored as one
// multiplier and one swap bit per column.
// ===========================================================================

// One thread per (source r, shifted solve q): q = 2*node + (0: +tau, 1: -tau).
// Tridiagonal T_r = tridiag(beta, alpha, gamma) of size k_r, with the rule of
// source r (rules[r]: each source may be at its own step).  Wave results are
// reduced over lanes: part[r][wave][2][kmax] complex (fine rule, coarse rule),
// wave = wave0 + blockIdx.x of nwave in all; waves beyond a source's nodes
// write zero rows.  A launch covers one chunk of waves; the multipliers of a
// chunk live in mult/swp [r][blockIdx.x][kmax][64], which the next chunk
// (ordered on the stream) reuses.
__global__ void __launch_bounds__(64) k_isign_tri(const double2* __restrict__ alpha,
                                                  const double* __restrict__ beta,
                                                  const double2* __restrict__ gamma, int kmax,
                                                  const int* __restrict__ kvec,
                                                  const QuadNodes* __restrict__ rules,
                                                  int wave0, int nwave,
                                                  double2* __restrict__ mult,
                                                  unsigned char* __restrict__ swp,
                                                  double2* __restrict__ part) {
  const int r = blockIdx.y;
  const QuadNodes qn = rules[r];
  const int wave = wave0 + blockIdx.x;
  const int lane = threadIdx.x;
  const int q = wave * 64 + lane;
  const int nq = 2 * qn.nnode;
  const int k = kvec[r];
  const bool live = q < nq;
  const int node = qn.n0 + (live ? q / 2 : 0);
  const double tau = exp(node * qn.h);
  const double sig = live ? ((q & 1) ? -tau : tau) : 1.0;
  const double wfine = live ? qn.h / M_PI * tau : 0.0;
  const double wcoarse = (live && ((node & 1) == 0)) ? 2.0 * qn.h / M_PI * tau : 0.0;
  const double2* al = alpha + (long)r * kmax;
  const double* be = beta + (long)r * kmax;
  const double2* ga = gamma + (long)r * kmax;
  const long mbase = ((long)(r * gridDim.x + blockIdx.x) * kmax) * 64 + lane;
  double2* part_r = part + ((long)r * nwave + wave) * 2 * kmax;
  if (k <= 0) return;
  if (wave * 64 >= nq) {
    // beyond this source's nodes (its rule is coarser than another
    // source's in the launch): zero rows, no solves (uniform over the wave)
    for (int j = lane; j < k; j += 64) {
      part_r[j] = make_double2(0.0, 0.0);
      part_r[kmax + j] = make_double2(0.0, 0.0);
    }
    return;
  }
  // elimination from the bottom: current column j holds (cu: row j-1, cd: row j)
  Cx<double> cu = (k >= 2) ? c64(ga[k - 2]) : Cx<double>{0, 0};
  Cx<double> cd = c64(al[k - 1]) + Cx<double>{0.0, sig};
  for (int j = k - 1; j >= 1; --j) {
    const Cx<double> du = (j >= 2) ? c64(ga[j - 2]) : Cx<double>{0, 0};
    const Cx<double> dm = c64(al[j - 1]) + Cx<double>{0.0, sig};
    const Cx<double> dd = {be[j - 1], 0.0};
    const bool sw = cabs1(dd) > cabs1(cd);
    Cx<double> m;
    if (sw) {
      m = cdiv(cd, dd);
      const Cx<double> nu_ = -cmul(m, du);
      const Cx<double> nd = cu - cmul(m, dm);
      cu = nu_;
      cd = nd;
    } else {
      m = cdiv(dd, cd);
      const Cx<double> nd = dm - cmul(m, cu);
      cu = du;
      cd = nd;
    }
    mult[mbase + (long)j * 64] = d2(m);
    swp[mbase + (long)j * 64] = sw ? 1 : 0;
  }
  const Cx<double> inv_r00 = cdiv(Cx<double>{1.0, 0.0}, cd);
  // z = P E e_1 streamed out top-down; row j-1 is final after column j.  The
  // weighted rows of the 64 lanes are buffered in LDS for kRows rows at a time
  // and summed over the lanes in a fixed order, one (row, part) per lane.
  constexpr int kRows = 16;
  __shared__ double rows[kRows][4][65];  // [row][fine re, fine im, coarse re, coarse im][lane]
  Cx<double> cur = inv_r00;
  for (int j0 = 1; j0 <= k; j0 += kRows) {
    const int nrow = min(kRows, k - j0 + 1);
    // the block's multipliers and swaps, loaded together rather than one row
    // per dependent step (rows from k on clamped to row k-1, never used)
    double2 mb[kRows];
    unsigned char sb[kRows];
#pragma unroll
    for (int t = 0; t < kRows; ++t) {
      const long jc = min(j0 + t, k - 1);
      mb[t] = mult[mbase + jc * 64];
      sb[t] = swp[mbase + jc * 64];
    }
#pragma unroll
    for (int t = 0; t < kRows; ++t) {
      if (t < nrow) {
        const int j = j0 + t;
        Cx<double> fin;
        if (j < k) {
          const Cx<double> m = c64(mb[t]);
          const Cx<double> nw = -cmul(m, cur);
          if (sb[t]) {
            fin = nw;
          } else {
            fin = cur;
            cur = nw;
          }
        } else {
          fin = cur;
        }
        rows[t][0][lane] = wfine * fin.re;
        rows[t][1][lane] = wfine * fin.im;
        rows[t][2][lane] = wcoarse * fin.re;
        rows[t][3][lane] = wcoarse * fin.im;
      }
    }
    __syncthreads();
    {
      const int t = lane & (kRows - 1), c = lane / kRows;  // 16 rows x 4 parts = 64 lanes
      if (t < nrow) {
        double acc = 0.0;
        for (int l = 0; l < 64; ++l) acc += rows[t][c][l];
        double* out = reinterpret_cast<double*>(part_r + (c < 2 ? 0 : kmax) + (j0 - 1 + t));
        out[c & 1] = acc;
      }
    }
    __syncthreads();
  }
}

// x[r][j] = sum over waves (fixed order); err[r] = |x_fine - x_coarse| / |x_fine|
__global__ void __launch_bounds__(256) k_isign_final(const double2* __restrict__ part, int nwave,
                                                     int kmax, const int* __restrict__ kvec,
                                                     double2* __restrict__ x,
                                                     double* __restrict__ err) {
  __shared__ double lds[4 * 2];
  const int r = blockIdx.x;
  const int k = kvec[r];
  double v[2] = {0, 0};
  for (int j = threadIdx.x; j < kmax; j += blockDim.x) {
    Cx<double> f = {0, 0}, c = {0, 0};
    if (j < k) {
      for (int w = 0; w < nwave; ++w) {
        const double2* p = part + ((long)r * nwave + w) * 2 * kmax;
        f = f + c64(p[j]);
        c = c + c64(p[kmax + j]);
      }
    }
    x[(long)r * kmax + j] = d2(f);
    v[0] += cnorm2(f - c);
    v[1] += cnorm2(f);
  }
  block_sum<2>(v, lds);
  if (threadIdx.x == 0) err[r] = v[1] > 0 ? sqrt(v[0] / v[1]) : 0.0;
}

// Hessenberg variant: one workgroup per (source r, shifted solve q), q = q0 +
// blockIdx.x for a chunk of gridDim.x solves.  The current column lives in
// LDS; H is column-major [r][kmax][kmax].
// Output ys[r][blockIdx.x][kmax] = (H + i sigma)^{-1} e_1 (unweighted).
constexpr int kHessMax = 1536;

__global__ void __launch_bounds__(256) k_isign_hess(const double2* __restrict__ H, int kmax,
                                                    const int* __restrict__ kvec, QuadNodes qn,
                                                    int q0, double2* __restrict__ ys) {
  __shared__ double2 c[kHessMax];
  __shared__ double2 mlt[kHessMax];
  __shared__ unsigned char swv[kHessMax];
  __shared__ double2 bc_m;
  __shared__ int bc_sw;
  const int q = q0 + blockIdx.x;
  const int r = blockIdx.y;
  const int k = kvec[r];
  const int node = qn.n0 + q / 2;
  const double tau = exp(node * qn.h);
  const double sig = (q & 1) ? -tau : tau;
  const double2* Hr = H + (long)r * kmax * kmax;
  double2* y = ys + ((long)r * gridDim.x + blockIdx.x) * kmax;
  if (k <= 0) return;
  // current column k-1 (rows 0..k-1)
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    Cx<double> v = c64(Hr[(long)(k - 1) * kmax + i]);
    if (i == k - 1) v.im += sig;
    c[i] = d2(v);
  }
  __syncthreads();
  for (int j = k - 1; j >= 1; --j) {
    const double2* dcol = Hr + (long)(j - 1) * kmax;
    if (threadIdx.x == 0) {
      const Cx<double> cd = c64(c[j]);
      const Cx<double> dd = c64(dcol[j]);  // subdiagonal entry H[j][j-1]
      const bool sw = cabs1(dd) > cabs1(cd);
      const Cx<double> m = sw ? cdiv(cd, dd) : cdiv(dd, cd);
      bc_m = d2(m);
      bc_sw = sw;
      mlt[j] = d2(m);
      swv[j] = sw;
    }
    __syncthreads();
    const Cx<double> m = c64(bc_m);
    const bool sw = bc_sw;
    for (int i = threadIdx.x; i < j; i += blockDim.x) {
      Cx<double> d = c64(dcol[i]);
      if (i == j - 1) d.im += sig;
      const Cx<double> ci = c64(c[i]);
      c[i] = d2(sw ? ci - cmul(m, d) : d - cmul(m, ci));
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    Cx<double> cur = cdiv(Cx<double>{1.0, 0.0}, c64(c[0]));
    for (int j = 1; j < k; ++j) {
      const Cx<double> nw = -cmul(c64(mlt[j]), cur);
      if (swv[j]) {
        y[j - 1] = d2(nw);
      } else {
        y[j - 1] = d2(cur);
        cur = nw;
      }
    }
    y[k - 1] = d2(cur);
  }
}

// acc[r][0][j] += sum over the chunk's solves of w_q ys (fine rule),
// acc[r][1][j] the same over the coarse rule's nodes; solves in order, so the
// sums are the same for every run.  first: the chunk starts the sums.
__global__ void __launch_bounds__(256) k_isign_hess_accum(const double2* __restrict__ ys, int q0,
                                                          int nq_chunk, int kmax,
                                                          const int* __restrict__ kvec,
                                                          QuadNodes qn, int first,
                                                          double2* __restrict__ acc) {
  const int r = blockIdx.y;
  const int k = kvec[r];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kmax) return;
  double2* a = acc + (long)r * 2 * kmax;
  Cx<double> f = first ? Cx<double>{0, 0} : c64(a[j]);
  Cx<double> c = first ? Cx<double>{0, 0} : c64(a[kmax + j]);
  if (j < k) {
    for (int qq = 0; qq < nq_chunk; ++qq) {
      const int node = qn.n0 + (q0 + qq) / 2;
      const double tau = exp(node * qn.h);
      const Cx<double> yv = c64(ys[((long)r * nq_chunk + qq) * kmax + j]);
      f = f + scale(qn.h / M_PI * tau, yv);
      if ((node & 1) == 0) c = c + scale(2.0 * qn.h / M_PI * tau, yv);
    }
  }
  a[j] = d2(f);
  a[kmax + j] = d2(c);
}

// x[r] = fine sums; err[r] = |x_fine - x_coarse| / |x_fine|
__global__ void __launch_bounds__(256) k_isign_hess_final(const double2* __restrict__ acc, int kmax,
                                                          const int* __restrict__ kvec,
                                                          double2* __restrict__ x,
                                                          double* __restrict__ err) {
  __shared__ double lds[4 * 2];
  const int r = blockIdx.x;
  const int k = kvec[r];
  double v[2] = {0, 0};
  for (int j = threadIdx.x; j < kmax; j += blockDim.x) {
    Cx<double> f = {0, 0}, c = {0, 0};
    if (j < k) {
      f = c64(acc[(long)r * 2 * kmax + j]);
      c = c64(acc[(long)r * 2 * kmax + kmax + j]);
    }
    x[(long)r * kmax + j] = d2(f);
    v[0] += cnorm2(f - c);
    v[1] += cnorm2(f);
  }
  block_sum<2>(v, lds);
  if (threadIdx.x == 0) err[r] = v[1] > 0 ? sqrt(v[0] / v[1]) : 0.0;
}

// ===========================================================================
// Host-side launchers
// ===========================================================================

static int chunks_for(long N, int cap = 1024) {
  long b = (N + 255) / 256;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (int)b;
}

// chunks of the deflation dots: at least 16 entries per thread, so that the
// per-workgroup reduction of 4 kDeflRhs values does not dominate (one entry
// per thread made the dots latency-bound: 107 us for m = 30 at 8^4)
int defl_nchunk(long N) {
  long c = (N + 256L * 16 - 1) / (256L * 16);
  if (c > 512) c = 512;
  if (c < 1) c = 1;
  return (int)c;
}

void launch_defl(const double2* R, const double2* L, const double2* B, const double* sgn, int m,
                 int nrhs, long N, double* partials, double* CD, double2* bR, double2* bL,
                 double2* yex, hipStream_t s) {
  const int nch = defl_nchunk(N);
  hipLaunchKernelGGL(k_defl_dots, dim3(nch, m, cdiv_i(nrhs, kDeflRhs)), dim3(256), 0, s, R, L, B,
                     nrhs, N, nch, partials);
  hipLaunchKernelGGL(k_reduce_partials<4>, dim3(m * nrhs), dim3(256), 0, s, partials, nch, CD);
  hipLaunchKernelGGL(k_defl_axpy, dim3(chunks_for(N, 4096), nrhs), dim3(256), 0, s, R, L, B, CD,
                     sgn, m, nrhs, N, bR, bL, yex);
}

void launch_defl_proj(const double2* R, const double2* L, const double2* X, int m, int nrhs, long N,
                      double* partials, double* CD, const double2* kappa, double2* outQ,
                      double2* outQd, hipStream_t s) {
  const int nch = defl_nchunk(N);
  hipLaunchKernelGGL(k_defl_dots, dim3(nch, m, cdiv_i(nrhs, kDeflRhs)), dim3(256), 0, s, R, L, X,
                     nrhs, N, nch, partials);
  hipLaunchKernelGGL(k_reduce_partials<4>, dim3(m * nrhs), dim3(256), 0, s, partials, nch, CD);
  if (kappa)
    hipLaunchKernelGGL(k_cd_shift, dim3(cdiv_i(m * nrhs, 256)), dim3(256), 0, s, CD, kappa, m, nrhs);
  hipLaunchKernelGGL(k_defl_axpy, dim3(chunks_for(N, 4096), nrhs), dim3(256), 0, s, R, L, X, CD,
                     (const double*)nullptr, m, nrhs, N, outQ, outQd, (double2*)nullptr);
}

void launch_defl_cd(const double2* R, const double2* L, const double2* B, int m, int nrhs, long N,
                    double* partials, double* CD, hipStream_t s) {
  const int nch = defl_nchunk(N);
  hipLaunchKernelGGL(k_defl_dots, dim3(nch, m, cdiv_i(nrhs, kDeflRhs)), dim3(256), 0, s, R, L, B,
                     nrhs, N, nch, partials);
  hipLaunchKernelGGL(k_reduce_partials<4>, dim3(m * nrhs), dim3(256), 0, s, partials, nch, CD);
}

void launch_start(const double2* bR, const double2* bL, int nrhs, long N, double* partials,
                  double* sums, void* V0, void* W0, bool f32, hipStream_t s) {
  const int nch = chunks_for(N, 512);
  hipLaunchKernelGGL(k_start_dots, dim3(nch, nrhs), dim3(256), 0, s, bR, bL, N, nch, partials);
  hipLaunchKernelGGL(k_reduce_partials<3>, dim3(nrhs), dim3(256), 0, s, partials, nch, sums);
  if (!V0 && !W0) return;  // norms only
  if (f32)
    hipLaunchKernelGGL(k_start_vectors<float2>, dim3(chunks_for(N, 4096), nrhs), dim3(256), 0, s,
                       bR, bL, sums, N, (float2*)V0, (float2*)W0);
  else
    hipLaunchKernelGGL(k_start_vectors<double2>, dim3(chunks_for(N, 4096), nrhs), dim3(256), 0, s,
                       bR, bL, sums, N, (double2*)V0, (double2*)W0);
}

// 256 workgroups per source: each reduces the dual stencil's partials for alpha
// first, so fewer and longer-running workgroups keep that head cheap.
int update_nwg(long N) { return chunks_for(N, 256); }

void launch_alpha(const double* partials, int nparts, const CoefArrays& co, const int* it,
                  const int* rhs_map, const int* n_active, int nslots, hipStream_t s) {
  hipLaunchKernelGGL(k_alpha, dim3(nslots), dim3(256), 0, s, partials, nparts, co, it, rhs_map,
                     n_active);
}

void launch_update(bool f32, const void* T, const void* S, void* basis, long basis_stride,
                   void* wbuf, long N, const CoefArrays& co, const int* it, const int* rhs_map,
                   const int* n_active, int nslots, double* partials, bool ring,
                   const double* apart, int anparts, int nt, hipStream_t s) {
  dim3 grid(update_nwg(N), nslots);
  if (f32)
    hipLaunchKernelGGL(k_update<float2>, grid, dim3(256), 0, s, (const float2*)T, (const float2*)S,
                       (float2*)basis, basis_stride, (float2*)wbuf, N, N, co, it, rhs_map, n_active,
                       partials, (int)ring, apart, anparts, nt);
  else
    hipLaunchKernelGGL(k_update<double2>, grid, dim3(256), 0, s, (const double2*)T,
                       (const double2*)S, (double2*)basis, basis_stride, (double2*)wbuf, N, N, co,
                       it, rhs_map, n_active, partials, (int)ring, apart, anparts, nt);
}

void launch_beta_tail(bool f32, const double* partials, int nparts, const CoefArrays& co, int* it,
                      const int* rhs_map, const int* n_active, int nslots, int* ticket,
                      const void* basis, long basis_stride, long N, bool ring, const int* idx,
                      int P, double2* probes, hipStream_t s) {
  if (f32)
    hipLaunchKernelGGL(k_beta_tail<float2>, dim3(nslots), dim3(256), 0, s, partials, nparts, co, it,
                       rhs_map, n_active, ticket, (const float2*)basis, basis_stride, N, (int)ring,
                       idx, P, probes);
  else
    hipLaunchKernelGGL(k_beta_tail<double2>, dim3(nslots), dim3(256), 0, s, partials, nparts, co, it,
                       rhs_map, n_active, ticket, (const double2*)basis, basis_stride, N, (int)ring,
                       idx, P, probes);
}

void launch_probe_gather(bool f32, const void* basis, long basis_stride, long N, bool ring,
                         const int* it, bool first, const int* idx, int P, int kmax,
                         const int* rhs_map, const int* n_active, int nslots, double2* probes,
                         hipStream_t s) {
  dim3 grid(cdiv_i(P, 256), nslots);
  if (f32)
    hipLaunchKernelGGL(k_probe_gather<float2>, grid, dim3(256), 0, s, (const float2*)basis,
                       basis_stride, N, (int)ring, it, (int)first, idx, P, kmax, rhs_map, n_active,
                       probes);
  else
    hipLaunchKernelGGL(k_probe_gather<double2>, grid, dim3(256), 0, s, (const double2*)basis,
                       basis_stride, N, (int)ring, it, (int)first, idx, P, kmax, rhs_map, n_active,
                       probes);
}

void launch_probe_y(const double2* probes, const double2* coef, const int* kvec, int kmax,
                    const double2* yex, long N, const int* idx, int P, double2* yp, int nrhs,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_probe_y, dim3(cdiv_i(P, 64), nrhs), dim3(64), 0, s, probes, coef, kvec,
                     kmax, yex, N, idx, P, yp);
}

void launch_advance(int* it, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, s, it);
}

void launch_make_coef(const double2* x, const double* sv, const double* nb, int kmax, int nrhs,
                      double2* coef, hipStream_t s) {
  long n = (long)nrhs * kmax;
  hipLaunchKernelGGL(k_make_coef, dim3(cdiv_i(n, 256)), dim3(256), 0, s, x, sv, nb, kmax, nrhs, coef);
}

void launch_combine(bool f32, const void* basis, long basis_stride, long N, const double2* coef,
                    int kmax, const int* kused, const double2* yex, double2* y, int nrhs,
                    hipStream_t s) {
  dim3 grid(chunks_for(N, 4096), nrhs);
  if (f32)
    hipLaunchKernelGGL(k_combine<float2>, grid, dim3(256), 0, s, (const float2*)basis, basis_stride,
                       N, coef, kmax, kused, yex, y);
  else
    hipLaunchKernelGGL(k_combine<double2>, grid, dim3(256), 0, s, (const double2*)basis,
                       basis_stride, N, coef, kmax, kused, yex, y);
}

void launch_replay(bool f32, const void* T, void* ring, long ring_stride, long N,
                   const CoefArrays& co, int i, const double2* coef, const int* kused, double2* y,
                   int nrhs, hipStream_t s) {
  dim3 grid(chunks_for(N, 4096), nrhs);
  if (f32)
    hipLaunchKernelGGL(k_replay<float2>, grid, dim3(256), 0, s, (const float2*)T, (float2*)ring,
                       ring_stride, N, co, i, coef, kused, y);
  else
    hipLaunchKernelGGL(k_replay<double2>, grid, dim3(256), 0, s, (const double2*)T, (double2*)ring,
                       ring_stride, N, co, i, coef, kused, y);
}

void launch_overlap(const double2* b, double2* y, long N, int V, hipStream_t s) {
  hipLaunchKernelGGL(k_overlap, dim3(chunks_for(N, 8192)), dim3(256), 0, s, b, y, N, V);
}

int arn_nchunk(long N) { return chunks_for(N, 256); }

void launch_arn_dots(bool f32, const void* basis, long basis_stride, const void* T, long N,
                     int nvec, int nrhs, double* partials, double* red, hipStream_t s) {
  const int nch = arn_nchunk(N);
  dim3 grid(nch, nrhs, cdiv_i(nvec, kArnVec));
  if (f32)
    hipLaunchKernelGGL(k_block_dots<float2>, grid, dim3(256), 0, s, (const float2*)basis,
                       basis_stride, (const float2*)T, N, nvec, nch, partials);
  else
    hipLaunchKernelGGL(k_block_dots<double2>, grid, dim3(256), 0, s, (const double2*)basis,
                       basis_stride, (const double2*)T, N, nvec, nch, partials);
  hipLaunchKernelGGL(k_reduce_partials<2>, dim3(nrhs * nvec), dim3(256), 0, s, partials, nch, red);
}

void launch_gram(const double2* X, int nx, const double2* Y, int ny, long N, double* partials,
                 double2* G, hipStream_t s) {
  for (int j = 0; j < ny; ++j)
    launch_arn_dots(false, X, N, Y + (long)j * N, N, nx, 1, partials, (double*)(G + (long)j * nx), s);
}

void launch_arn_accum(const double* red, int nvec, int kmax, int j, bool first, double2* H,
                      double2* hcur, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_arn_accum, dim3(cdiv_i((long)nrhs * nvec, 256)), dim3(256), 0, s, red, nvec,
                     kmax, j, (int)first, H, hcur, nrhs);
}

void launch_arn_axpy(bool f32, const void* basis, long basis_stride, void* T, long N, int nvec,
                     const double2* hcur, int kmax, int nrhs, double* partials, double* red,
                     hipStream_t s) {
  const int nch = arn_nchunk(N);
  dim3 grid(nch, nrhs);
  if (f32)
    hipLaunchKernelGGL(k_block_axpy<float2>, grid, dim3(256), 0, s, (const float2*)basis,
                       basis_stride, (float2*)T, N, nvec, hcur, kmax, partials);
  else
    hipLaunchKernelGGL(k_block_axpy<double2>, grid, dim3(256), 0, s, (const double2*)basis,
                       basis_stride, (double2*)T, N, nvec, hcur, kmax, partials);
  hipLaunchKernelGGL(k_reduce_partials<1>, dim3(nrhs), dim3(256), 0, s, partials, nch, red);
}

void launch_norm2(bool f32, const void* T, long N, int nrhs, double* partials, double* red,
                  hipStream_t s) {
  const int nch = arn_nchunk(N);
  dim3 grid(nch, nrhs);
  if (f32)
    hipLaunchKernelGGL(k_norm2<float2>, grid, dim3(256), 0, s, (const float2*)T, N, partials);
  else
    hipLaunchKernelGGL(k_norm2<double2>, grid, dim3(256), 0, s, (const double2*)T, N, partials);
  hipLaunchKernelGGL(k_reduce_partials<1>, dim3(nrhs), dim3(256), 0, s, partials, nch, red);
}

void launch_arn_sub(const double* red_n, const double* red_tn, double2* H, int kmax, int j,
                    double* scl, int* kstop, int* status, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_arn_sub, dim3(cdiv_i(nrhs, 64)), dim3(64), 0, s, red_n, red_tn, H, kmax, j,
                     scl, kstop, status, nrhs);
}

void launch_scale_copy(bool f32, const void* T, void* out, long N, const double* scl, int nrhs,
                       hipStream_t s) {
  dim3 grid(chunks_for(N, 4096), nrhs);
  if (f32)
    hipLaunchKernelGGL(k_scale_copy<float2>, grid, dim3(256), 0, s, (const float2*)T, (float2*)out,
                       N, scl);
  else
    hipLaunchKernelGGL(k_scale_copy<double2>, grid, dim3(256), 0, s, (const double2*)T,
                       (double2*)out, N, scl);
}

int isign_tri_nwave(int nnode) { return cdiv_i(2L * nnode, 64); }

void launch_isign_tri(const double2* alpha, const double* beta, const double2* gamma, int kmax,
                      const int* kvec, int nrhs, const QuadNodes* rules, int nwave, double2* mult,
                      unsigned char* swp, double2* part, double2* x, double* err, hipStream_t s) {
  const int nw = std::max(nwave, 1);
  for (int w0 = 0; w0 < nw; w0 += kIsignWaveChunk)
    hipLaunchKernelGGL(k_isign_tri, dim3(std::min(kIsignWaveChunk, nw - w0), nrhs), dim3(64), 0,
                       s, alpha, beta, gamma, kmax, kvec, rules, w0, nw, mult, swp, part);
  hipLaunchKernelGGL(k_isign_final, dim3(nrhs), dim3(256), 0, s, part, nw, kmax, kvec, x, err);
}

void launch_isign_hess(const double2* H, int kmax, const int* kvec, int nrhs, double h, int n0,
                       int nnode, double2* ys, double2* acc, double2* x, double* err,
                       hipStream_t s) {
  QuadNodes qn{h, n0, nnode};
  const int nq = 2 * nnode;
  for (int q0 = 0; q0 < nq; q0 += kIsignHessChunk) {
    const int nc = std::min(kIsignHessChunk, nq - q0);
    hipLaunchKernelGGL(k_isign_hess, dim3(nc, nrhs), dim3(256), 0, s, H, kmax, kvec, qn, q0, ys);
    hipLaunchKernelGGL(k_isign_hess_accum, dim3(cdiv_i(kmax, 256), nrhs), dim3(256), 0, s, ys, q0,
                       nc, kmax, kvec, qn, (int)(q0 == 0), acc);
  }
  hipLaunchKernelGGL(k_isign_hess_final, dim3(nrhs), dim3(256), 0, s, acc, kmax, kvec, x, err);
}

}  // namespace ovs
