// Kernels of the gradient of L = Re <chi, y_k> with respect to b, mu and the
// links, for the two-sided Lanczos approximation of Section 4 without
// deflation, y_k = |b| V_k sgn(G_k) e_1 (eq. 2sLapp with m = 0).
//
// The driver (gradient.cpp) runs the Lanczos recurrences forward storing the
// FP64 bases V, W (or checkpoints), then walks them backwards.  Every vector
// step is a short linear combination of stored fields with fused dot
// products (k_lin, k_lin_multi); the per-source scalar steps mostly run at
// the start of the combination launch that uses their coefficient rows
// (k_lin_step, k_lin_multi_step); the pairs of A and A^dagger applications
// are the dual stencil; the link and mu derivatives are accumulated by
// k_gforce (one step) and k_gforce_group (a group of steps).  Reductions
// are fixed-order.
#include <cmath>

#include "ovs_common.h"
#include "ovs_device.h"
#include "ovs_grad.h"
#include "ovs_spin.h"

namespace ovs {

// ---- linear combinations with fused dots -------------------------------------

// Workgroups per source of the linear combinations: up to 1024 (four per CU),
// so that one source's pass keeps enough waves in flight to stream from HBM.
int lin_nchunk(long stride) {
  long c = (stride + kWG - 1) / kWG;
  if (c > 1024) c = 1024;
  if (c < 1) c = 1;
  return (int)c;
}

// TAB: the launch ran a scalar step whose coefficient rows are in `tab`
// (LDS); a combination with a.tab >= 0 takes them from there instead of the
// global table a.coef.
template <bool TAB>
__device__ __forceinline__ void lin_body(const LinArgs& a, long stride, int nrhs, double* lds,
                                         const double2 (*tab)[kLinTerms]) {
  const int r = blockIdx.y;
  const long off = (long)r * stride;
  Cx<double> c[kLinTerms];
  if (TAB && a.tab >= 0) {
#pragma unroll
    for (int j = 0; j < kLinTerms; ++j)
      c[j] = (j < a.nterm) ? c64(tab[a.tab][j]) : Cx<double>{0.0, 0.0};
  } else {
#pragma unroll
    for (int j = 0; j < kLinTerms; ++j)
      c[j] = (j < a.nterm) ? c64(a.coef[(long)j * nrhs + r]) : Cx<double>{0.0, 0.0};
  }
  double part[2 * kLinDots];
#pragma unroll
  for (int q = 0; q < 2 * kLinDots; ++q) part[q] = 0.0;
  for (long e = (long)blockIdx.x * kWG + threadIdx.x; e < stride; e += (long)gridDim.x * kWG) {
    Cx<double> v = {0.0, 0.0};
    if (a.accumulate) v = c64(a.out[off + e]);
#pragma unroll
    for (int j = 0; j < kLinTerms; ++j)
      if (j < a.nterm) v = cfma(c[j], c64(a.x[j][off + e]), v);
    if (a.out) a.out[off + e] = d2(v);
#pragma unroll
    for (int q = 0; q < kLinDots; ++q) {
      if (q < a.ndot) {
        const Cx<double> y = a.y[q] ? c64(a.y[q][off + e]) : v;
        const Cx<double> p = cmulc(y, v);
        part[2 * q] += p.re;
        part[2 * q + 1] += p.im;
      }
    }
  }
  if (a.ndot == 0) return;  // uniform over the workgroup
  block_sum<2 * kLinDots>(part, lds);
  if (threadIdx.x == 0) {
    double* dst = a.partials + ((long)r * gridDim.x + blockIdx.x) * 2 * kLinDots;
#pragma unroll
    for (int q = 0; q < 2 * kLinDots; ++q) dst[q] = part[q];
  }
}

__global__ void __launch_bounds__(kWG) k_lin(LinArgs a, long stride, int nrhs) {
  __shared__ double lds[(kWG / 64) * 2 * kLinDots];
  lin_body<false>(a, stride, nrhs, lds, nullptr);
}

// Several linear combinations in one launch: each is computed as k_lin
// computes it (same grid, same per-element arithmetic, its own partial sums),
// so the results equal those of separate launches bit for bit.  A thread
// visits the same elements in every combination, so a combination may read
// an earlier one's output at the element it is computing (written by the same
// thread); no other element of another's output.
__global__ void __launch_bounds__(kWG) k_lin_multi(LinMulti m, long stride, int nrhs) {
  __shared__ double lds[(kWG / 64) * 2 * kLinDots];
  for (int j = 0; j < m.n; ++j) {
    __syncthreads();  // lds of the previous combination
    lin_body<false>(m.a[j], stride, nrhs, lds, nullptr);
  }
}

void launch_lin(const LinArgs& a, long stride, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_lin, dim3(lin_nchunk(stride), nrhs), dim3(kWG), 0, s, a, stride, nrhs);
}

void launch_lin_multi(const LinMulti& m, long stride, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_lin_multi, dim3(lin_nchunk(stride), nrhs), dim3(kWG), 0, s, m, stride,
                     nrhs);
}

// Workgroup of the per-source scalar kernels: one per source, the dot sums
// over the chunks reduced by all its threads.
constexpr int kScalarWG = 256;

// Fixed-order sums over the chunks of ND dots of source r (dot q[d] of the
// partials parts[d]): strided over the chunks by the workgroup, then a
// fixed-order workgroup sum; every thread receives the results.
template <int ND>
__device__ void wg_dot_sums(const double* const (&parts)[ND], const int (&q)[ND], int r,
                            int nchunk, Cx<double> (&out)[ND]) {
  __shared__ double lds[(kScalarWG / 64) * 2 * ND];
  __shared__ double res[2 * ND];
  double v[2 * ND];
#pragma unroll
  for (int j = 0; j < 2 * ND; ++j) v[j] = 0.0;
  for (int c = threadIdx.x; c < nchunk; c += blockDim.x) {
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const double* pp = parts[d] + ((long)r * nchunk + c) * 2 * kLinDots + 2 * q[d];
      v[2 * d] += pp[0];
      v[2 * d + 1] += pp[1];
    }
  }
  block_sum<2 * ND>(v, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < 2 * ND; ++j) res[j] = v[j];
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < ND; ++d) out[d] = {res[2 * d], res[2 * d + 1]};
}

__device__ __forceinline__ Cx<double> cconj(Cx<double> a) { return {a.re, -a.im}; }
__device__ __forceinline__ void set_coef(const GradScalars& s, int t, int j, int r, Cx<double> v) {
  s.coef[((long)t * kLinTerms + j) * s.nrhs + r] = d2(v);
}

// Where a scalar step puts the coefficient rows it forms for source r: the
// LDS table of the linear combination that follows it in the same launch
// (`lds`, read by all of that launch's threads), and/or the global tables
// (`coef`) for later launches.  `wr`: the step also writes its scalars
// (alpha, beta, ...) to global memory; in a combination launch only its
// first workgroup of each source does.
struct TabOut {
  double2 (*lds)[kLinTerms];
  double2* coef;
  int nrhs;
  int r;
  bool wr;
  __device__ void put(int t, int j, Cx<double> v) const {
    if (lds) lds[t][j] = d2(v);
    if (coef) coef[((long)t * kLinTerms + j) * nrhs + r] = d2(v);
  }
};

// ---- forward scalar steps ------------------------------------------------------

__global__ void __launch_bounds__(kScalarWG) k_gf_norm(GradScalars s, const double* part, int nchunk) {
  const int r = blockIdx.x;
  Cx<double> d[1];
  wg_dot_sums<1>({part}, {0}, r, nchunk, d);
  if (threadIdx.x != 0) return;
  const double nb = sqrt(d[0].re);
  s.nb[r] = nb;
  s.status[r] = 0;
  set_coef(s, kTabNorm, 0, r, {nb > 0.0 ? 1.0 / nb : 0.0, 0.0});
}

__global__ void __launch_bounds__(kScalarWG) k_gf_start(GradScalars s, const double* part,
                                                         const double* part_b, int nchunk) {
  const int r = blockIdx.x;
  Cx<double> d[3];
  wg_dot_sums<3>({part, part, part_b}, {0, 1, 0}, r, nchunk, d);
  if (threadIdx.x != 0) return;
  const double nb = sqrt(d[0].re);
  const Cx<double> sig = d[1];
  s.nb[r] = nb;
  s.sigma[r] = d2(sig);
  s.status[r] = 0;
  set_coef(s, kTabNorm, 0, r, {nb > 0.0 ? 1.0 / nb : 0.0, 0.0});
  // |b_R| <= 1e-12 |b|: the source lies in span R (the solve drops the Krylov
  // part there); like a start with no biorthogonal partner, it has no gradient
  const bool ok = nb > 1e-12 * sqrt(d[2].re) && (sig.re != 0.0 || sig.im != 0.0);
  set_coef(s, kTabStartW, 0, r, ok ? cdiv(Cx<double>{nb, 0.0}, cconj(sig)) : Cx<double>{0.0, 0.0});
  if (!ok) s.status[r] = 2;
}

// alpha_i = w_i^dagger t_i (dot 0), |t_i|^2 (dot 1); coefficient rows of the
// update.  All threads of the workgroup take part (the dot sums); thread 0
// forms the rows.
__device__ void step_gf_alpha(const GradScalars& s, int i, const double* part, int nchunk,
                              const TabOut& o) {
  const int r = o.r;
  Cx<double> d[2];
  wg_dot_sums<2>({part, part}, {0, 1}, r, nchunk, d);
  if (threadIdx.x != 0) return;
  const long rk = (long)r * s.kmax;
  const Cx<double> al = d[0];
  if (o.wr) {
    s.alpha[rk + i] = d2(al);
    s.tnorm2[rk + i] = d[1].re;
  }
  const Cx<double> gprev = (i > 0) ? c64(s.gamma[rk + i - 1]) : Cx<double>{0.0, 0.0};
  const double bprev = (i > 0) ? s.beta[rk + i - 1] : 0.0;
  o.put(kTabV, 0, {1.0, 0.0});
  o.put(kTabV, 1, -al);
  o.put(kTabV, 2, -gprev);
  o.put(kTabW, 0, {1.0, 0.0});
  o.put(kTabW, 1, -cconj(al));
  o.put(kTabW, 2, {-bprev, 0.0});
}
__global__ void __launch_bounds__(kScalarWG) k_gf_alpha(GradScalars s, int i, const double* part, int nchunk) {
  step_gf_alpha(s, i, part, nchunk, TabOut{nullptr, s.coef, s.nrhs, (int)blockIdx.x, true});
}

// beta_i = |v~|, delta_i = w~^dagger v~, gamma_i = delta_i / beta_i, with the
// breakdown tests of the forward recurrences (lucky: |v~| <= 1e-14 |t|;
// serious: |delta| <= 1e-13 |v~| |w~|).
__device__ void step_gf_beta(const GradScalars& s, int i, const double* part_v,
                             const double* part_w, int nchunk, const TabOut& o) {
  const int r = o.r;
  Cx<double> d[3];
  wg_dot_sums<3>({part_v, part_w, part_w}, {0, 0, 1}, r, nchunk, d);
  if (threadIdx.x != 0) return;
  const long rk = (long)r * s.kmax;
  const double vn = sqrt(d[0].re);
  const Cx<double> delta = cconj(d[1]);  // dot 0 of part_w = v~^dagger w~
  const double wn = sqrt(d[2].re);
  const Cx<double> g = vn > 0.0 ? scale(1.0 / vn, delta) : Cx<double>{0.0, 0.0};
  if (o.wr) {
    if (s.status[r] == 0) {
      if (vn <= 1e-14 * sqrt(s.tnorm2[rk + i])) s.status[r] = 1;
      else if (cabs1(delta) <= 1e-13 * vn * wn) s.status[r] = 2;
    }
    s.beta[rk + i] = vn;
    s.gamma[rk + i] = d2(g);
  }
  o.put(kTabSV, 0, {vn > 0.0 ? 1.0 / vn : 0.0, 0.0});
  const bool gz = g.re == 0.0 && g.im == 0.0;
  o.put(kTabSW, 0, gz ? Cx<double>{0.0, 0.0} : cdiv({1.0, 0.0}, cconj(g)));
}

void launch_gf_norm(const GradScalars& s, const double* part, int nchunk, hipStream_t st) {
  hipLaunchKernelGGL(k_gf_norm, dim3(s.nrhs), dim3(kScalarWG), 0, st, s, part, nchunk);
}
void launch_gf_start(const GradScalars& s, const double* part, const double* part_b, int nchunk,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_gf_start, dim3(s.nrhs), dim3(kScalarWG), 0, st, s, part, part_b, nchunk);
}
void launch_gf_alpha(const GradScalars& s, int i, const double* part, int nchunk, hipStream_t st) {
  hipLaunchKernelGGL(k_gf_alpha, dim3(s.nrhs), dim3(kScalarWG), 0, st, s, i, part, nchunk);
}

// ---- reverse scalar steps ------------------------------------------------------
// Adjoint rules used below (zbar = dL/dRe z + i dL/dIm z, dL = Re <zbar, dz>):
//   z = c u         : ubar += conj(c) zbar,   cbar += u^dagger zbar
//   z = u^dagger v  : vbar += zbar u,         ubar += conj(zbar) v
//   z = u / conj(c) : ubar += zbar / c,       cbar += -(zbar^dagger z) / conj(c)
//   r = |u| (real)  : ubar += rbar u / r

// Last step (i = k-1): only t = A v_{k-1} and alpha_{k-1} = w_{k-1}^dagger t exist.
__global__ void k_gr_first(GradScalars s) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= s.nrhs) return;  // scalar only: one thread per source
  const int i = s.kmax - 1;
  const long rk = (long)r * s.kmax;
  const Cx<double> ab = c64(s.abar[rk + i]);
  set_coef(s, kTabSV, 0, r, ab);                                           // tbar = abar w_i
  set_coef(s, kTabSW, 0, r, scale(s.nb[r], cconj(c64(s.x[rk + i]))));     // vbar = nb conj(x_i) chi
  set_coef(s, kTabWB, 0, r, cconj(ab));                                    // wbar = conj(abar) t_i
  set_coef(s, kTabY, 0, r, scale(s.nb[r], c64(s.x[rk + i])));              // y += nb x_i v_i
}

// Step i < k-1, first half.  Inputs: dots of the completed vbar_{i+1}, wbar_{i+1}
// with v_{i+1}, w_{i+1}.  Through v_{i+1} = v~/beta_i, w_{i+1} = w~/conj(gamma_i),
// gamma_i = delta_i/beta_i, beta_i = |v~|, delta_i = w~^dagger v~:
//   gbar_i += -(wbar_{i+1}^dagger w_{i+1}) / conj(gamma_i)
//   bbar_i += -Re(vbar_{i+1}^dagger v_{i+1}) / beta_i - Re(conj(gbar_i) gamma_i) / beta_i
//   dbar    = gbar_i / beta_i
//   vbar~_i = vbar_{i+1}/beta_i + bbar_i v_{i+1} + dbar conj(gamma_i) w_{i+1}
//   wbar~_i = wbar_{i+1}/gamma_i + conj(dbar) beta_i v_{i+1}
// gbar_i and bbar_i are read here and used nowhere after this step, so the
// updated values are not written back (a combination launch that forms them
// in every workgroup could not write them without racing its own reads).
__device__ void step_gr_s1(const GradScalars& s, int i, const double* part_v, const double* part_w,
                           int nchunk, const TabOut& o) {
  const int r = o.r;
  Cx<double> d[2];
  wg_dot_sums<2>({part_v, part_w}, {0, 0}, r, nchunk, d);
  if (threadIdx.x != 0) return;
  const long rk = (long)r * s.kmax;
  const Cx<double> d2v = cconj(d[0]);  // vbar^dagger v
  const Cx<double> d1w = cconj(d[1]);  // wbar^dagger w
  const double be = s.beta[rk + i];
  const Cx<double> ga = c64(s.gamma[rk + i]);
  Cx<double> gb = c64(s.gbar[rk + i]);
  double bb = s.bbar[rk + i];
  gb = gb - cdiv(d1w, cconj(ga));
  bb -= d2v.re / be;
  const Cx<double> db = scale(1.0 / be, gb);
  bb -= (gb.re * ga.re + gb.im * ga.im) / be;  // Re(conj(gbar) gamma)
  o.put(kTabV, 0, {1.0 / be, 0.0});
  o.put(kTabV, 1, {bb, 0.0});
  o.put(kTabV, 2, cmul(db, cconj(ga)));
  o.put(kTabW, 0, cdiv({1.0, 0.0}, ga));
  o.put(kTabW, 1, scale(be, cconj(db)));
}

// Step i < k-1, second half.  Inputs: v_i^dagger vbar~ (d5), v_{i-1}^dagger vbar~
// (d6), w_i^dagger wbar~ (conj d4), w_{i-1}^dagger wbar~ (d3).  Through
// v~ = t_i - alpha_i v_i - gamma_{i-1} v_{i-1}, w~ = s_i - conj(alpha_i) w_i -
// beta_{i-1} w_{i-1} and alpha_i = w_i^dagger t_i:
//   abar_i += -d4 - d5;  bbar_{i-1} += -Re d3;  gbar_{i-1} += -d6
//   tbar_i = vbar~_i + abar_i w_i                (then vbar_i += A^dagger tbar_i)
//   sbar_i = wbar~_i                              (then wbar_i += A sbar_i)
//   vbar_i = nb conj(x_i) chi - conj(gamma_i) vbar~_{i+1} - conj(alpha_i) vbar~_i
//   wbar_i = -beta_i wbar~_{i+1} - alpha_i wbar~_i + conj(abar_i) t_i,
//            t_i = beta_i v_{i+1} + alpha_i v_i + gamma_{i-1} v_{i-1}
// abar_i is read here and used nowhere after this step (not written back, as
// gbar_i in step 1); bbar_{i-1}, gbar_{i-1} are written for step i-1.
__device__ void step_gr_s2(const GradScalars& s, int i, const double* part_v, const double* part_w,
                           int nchunk, const TabOut& o) {
  const int r = o.r;
  // dots 1 exist for i > 0 only; at i = 0 their sums are formed and not used
  Cx<double> d[4];
  wg_dot_sums<4>({part_v, part_w, part_v, part_w}, {0, 0, 1, 1}, r, nchunk, d);
  if (threadIdx.x != 0) return;
  const long rk = (long)r * s.kmax;
  const Cx<double> d5 = d[0];
  const Cx<double> d4 = cconj(d[1]);
  const Cx<double> ab = c64(s.abar[rk + i]) - d4 - d5;
  if (o.wr && i > 0) {
    const Cx<double> d6 = d[2];
    const Cx<double> d3 = d[3];
    s.bbar[rk + i - 1] -= d3.re;
    s.gbar[rk + i - 1] = d2(c64(s.gbar[rk + i - 1]) - d6);
  }
  const Cx<double> al = c64(s.alpha[rk + i]);
  const Cx<double> ga = c64(s.gamma[rk + i]);
  const double be = s.beta[rk + i];
  const Cx<double> gprev = (i > 0) ? c64(s.gamma[rk + i - 1]) : Cx<double>{0.0, 0.0};
  o.put(kTabSV, 0, {1.0, 0.0});
  o.put(kTabSV, 1, ab);
  o.put(kTabSW, 0, scale(s.nb[r], cconj(c64(s.x[rk + i]))));
  o.put(kTabSW, 1, -cconj(ga));
  o.put(kTabSW, 2, -cconj(al));
  const Cx<double> cab = cconj(ab);
  o.put(kTabWB, 0, {-be, 0.0});
  o.put(kTabWB, 1, -al);
  o.put(kTabWB, 2, scale(be, cab));
  o.put(kTabWB, 3, cmul(cab, al));
  o.put(kTabWB, 4, cmul(cab, gprev));
  o.put(kTabY, 0, scale(s.nb[r], c64(s.x[rk + i])));
}

// v_1 = w_1 = b/|b|: grad_b = ubar/|b| + nbar v_1 with ubar = vbar_1 + wbar_1 and
// nbar = Re(chi^dagger y)/|b| - Re(ubar^dagger v_1)/|b|, chi^dagger y = sum_i x_i conj(xbar_i).
__global__ void __launch_bounds__(kScalarWG) k_gr_final(GradScalars s, const double* part, int nchunk) {
  __shared__ double lds[kScalarWG / 64];
  const int r = blockIdx.x;
  const long rk = (long)r * s.kmax;
  Cx<double> d[1];
  wg_dot_sums<1>({part}, {0}, r, nchunk, d);
  double cy[1] = {0.0};
  for (int i = threadIdx.x; i < s.kmax; i += blockDim.x) {
    const Cx<double> p = cmulc(c64(s.xbar[rk + i]), c64(s.x[rk + i]));
    cy[0] += p.re;
  }
  block_sum<1>(cy, lds);
  if (threadIdx.x != 0) return;
  const double nb = s.nb[r];
  const double uv = d[0].re;  // Re(v_1^dagger ubar)
  const double nbar = (cy[0] - uv) / nb;
  set_coef(s, kTabFin, 0, r, {1.0 / nb, 0.0});
  set_coef(s, kTabFin, 1, r, {nbar, 0.0});
}

__global__ void __launch_bounds__(kScalarWG) k_gr_final_defl(GradScalars s, const double* part_v,
                                                             const double* part_w, int nchunk) {
  __shared__ double lds[kScalarWG / 64];
  const int r = blockIdx.x;
  const long rk = (long)r * s.kmax;
  Cx<double> d[2];
  wg_dot_sums<2>({part_v, part_w}, {0, 0}, r, nchunk, d);
  double cy[1] = {0.0};
  for (int i = threadIdx.x; i < s.kmax; i += blockDim.x) {
    const Cx<double> p = cmulc(c64(s.xbar[rk + i]), c64(s.x[rk + i]));
    cy[0] += p.re;
  }
  block_sum<1>(cy, lds);
  if (threadIdx.x != 0) return;
  const double nb = s.nb[r];
  const Cx<double> sig = c64(s.sigma[r]);
  const Cx<double> rho = cconj(d[1]);           // wbar_1^dagger w_1
  const double nbar = (cy[0] - d[0].re + rho.re) / nb;
  const Cx<double> tau = -cdiv(rho, cconj(sig));
  set_coef(s, kTabFin, 0, r, {1.0 / nb, 0.0});
  set_coef(s, kTabFin, 1, r, tau);
  set_coef(s, kTabFin, 2, r, {nbar / nb, 0.0});
  set_coef(s, kTabFinW, 0, r, cdiv(Cx<double>{nb, 0.0}, sig));
  set_coef(s, kTabFinW, 1, r, cconj(tau));
}

void launch_gr_final_defl(const GradScalars& s, const double* part_v, const double* part_w,
                          int nchunk, hipStream_t st) {
  hipLaunchKernelGGL(k_gr_final_defl, dim3(s.nrhs), dim3(kScalarWG), 0, st, s, part_v, part_w,
                     nchunk);
}

void launch_gr_first(const GradScalars& s, hipStream_t st) {
  hipLaunchKernelGGL(k_gr_first, dim3((s.nrhs + 63) / 64), dim3(64), 0, st, s);
}
void launch_gr_final(const GradScalars& s, const double* part, int nchunk, hipStream_t st) {
  hipLaunchKernelGGL(k_gr_final, dim3(s.nrhs), dim3(kScalarWG), 0, st, s, part, nchunk);
}

// ---- source projections and replay coefficients -----------------------------

__device__ void step_gf_xbar(const GradScalars& s, int i, const double* part, int nchunk,
                             const TabOut& o) {
  const int r = o.r;
  Cx<double> d[1];
  wg_dot_sums<1>({part}, {0}, r, nchunk, d);  // chi^dagger v_i
  if (threadIdx.x != 0 || !o.wr) return;
  s.xbar[(long)r * s.kmax + i] = d2(scale(s.nb[r], cconj(d[0])));
}
__global__ void __launch_bounds__(kScalarWG) k_gf_xbar(GradScalars s, int i, const double* part, int nchunk) {
  step_gf_xbar(s, i, part, nchunk, TabOut{nullptr, nullptr, s.nrhs, (int)blockIdx.x, true});
}

void launch_gf_xbar(const GradScalars& s, int i, const double* part, int nchunk, hipStream_t st) {
  hipLaunchKernelGGL(k_gf_xbar, dim3(s.nrhs), dim3(kScalarWG), 0, st, s, i, part, nchunk);
}

// The rows of the forward update and normalisation of step i from the stored
// coefficients, with the arithmetic of steps alpha and beta (one thread).
__device__ void gp_coef_rows(const GradScalars& s, int i, const TabOut& o) {
  const int r = o.r;
  const long rk = (long)r * s.kmax;
  const Cx<double> al = c64(s.alpha[rk + i]);
  const Cx<double> gprev = (i > 0) ? c64(s.gamma[rk + i - 1]) : Cx<double>{0.0, 0.0};
  const double bprev = (i > 0) ? s.beta[rk + i - 1] : 0.0;
  o.put(kTabV, 0, {1.0, 0.0});
  o.put(kTabV, 1, -al);
  o.put(kTabV, 2, -gprev);
  o.put(kTabW, 0, {1.0, 0.0});
  o.put(kTabW, 1, -cconj(al));
  o.put(kTabW, 2, {-bprev, 0.0});
  const double vn = s.beta[rk + i];
  const Cx<double> g = c64(s.gamma[rk + i]);
  o.put(kTabSV, 0, {vn > 0.0 ? 1.0 / vn : 0.0, 0.0});
  const bool gz = g.re == 0.0 && g.im == 0.0;
  o.put(kTabSW, 0, gz ? Cx<double>{0.0, 0.0} : cdiv({1.0, 0.0}, cconj(g)));
}


// ---- linear combinations preceded by their scalar step ------------------------
// Every workgroup of source r forms the step's coefficient rows itself (the
// same dot sums in the same order, kWG = kScalarWG threads, so the same
// values as the separate scalar kernel) and keeps them in LDS; the first
// workgroup of each source also writes the step's scalars and, with
// global_tabs, the global tables.  That saves the scalar kernel's launch.
// Every value a step reads is written by earlier launches and none is
// written in this one, except the scalars of workgroup 0, which no other
// workgroup of the launch reads.
__device__ void run_step(const ScalarStep& st, double2 (*tab)[kLinTerms]) {
  const bool first = blockIdx.x == 0;
  const TabOut o{tab, (st.global_tabs && first) ? st.s.coef : nullptr, st.s.nrhs, (int)blockIdx.y,
                 first};
  switch (st.kind) {
    case kStepAlpha: step_gf_alpha(st.s, st.i, st.pa, st.nchunk, o); break;
    case kStepBeta: step_gf_beta(st.s, st.i, st.pa, st.pb, st.nchunk, o); break;
    case kStepXbar: step_gf_xbar(st.s, st.i, st.pa, st.nchunk, o); break;
    case kStepCoef:
      if (threadIdx.x == 0) gp_coef_rows(st.s, st.i, o);
      break;
    case kStepS1: step_gr_s1(st.s, st.i, st.pa, st.pb, st.nchunk, o); break;
    case kStepS2: step_gr_s2(st.s, st.i, st.pa, st.pb, st.nchunk, o); break;
    default: break;
  }
  __syncthreads();  // the rows in LDS for every thread
}

__global__ void __launch_bounds__(kWG) k_lin_step(LinArgs a, long stride, int nrhs, ScalarStep st) {
  __shared__ double lds[(kWG / 64) * 2 * kLinDots];
  __shared__ double2 tab[kCoefTables][kLinTerms];
  run_step(st, tab);
  lin_body<true>(a, stride, nrhs, lds, tab);
}

__global__ void __launch_bounds__(kWG) k_lin_multi_step(LinMulti m, long stride, int nrhs,
                                                        ScalarStep st) {
  __shared__ double lds[(kWG / 64) * 2 * kLinDots];
  __shared__ double2 tab[kCoefTables][kLinTerms];
  run_step(st, tab);
  for (int j = 0; j < m.n; ++j) {
    __syncthreads();  // lds of the previous combination
    lin_body<true>(m.a[j], stride, nrhs, lds, tab);
  }
}

void launch_lin_step(const LinArgs& a, long stride, int nrhs, const ScalarStep& st, hipStream_t s) {
  hipLaunchKernelGGL(k_lin_step, dim3(lin_nchunk(stride), nrhs), dim3(kWG), 0, s, a, stride, nrhs,
                     st);
}
void launch_lin_multi_step(const LinMulti& m, long stride, int nrhs, const ScalarStep& st,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_lin_multi_step, dim3(lin_nchunk(stride), nrhs), dim3(kWG), 0, s, m, stride,
                     nrhs, st);
}

// ---- inner sign and its vector-Jacobian product -----------------------------------
// One thread per (node, sign): LU with row interchanges of the tridiagonal
// M = G + i sigma (sigma = +-tau), then q = M^{-1} e_1 and p = M^{-H} xbar.
// Per-thread arrays live in scratch as [entry][thread] (coalesced).

struct VjpScratch {
  double2 *dl, *d, *du, *du2, *q, *p;
  unsigned char* piv;
};

static VjpScratch carve(void* base, int k, int nthr) {
  VjpScratch v;
  double2* b = (double2*)base;
  const long n = (long)k * nthr;
  v.dl = b;
  v.d = b + n;
  v.du = b + 2 * n;
  v.du2 = b + 3 * n;
  v.q = b + 4 * n;
  v.p = b + 5 * n;
  v.piv = (unsigned char*)(b + 6 * n);
  return v;
}

size_t isign_vjp_scratch_bytes(int k, int nnode) {
  const long n = (long)k * 2 * nnode;
  return (size_t)n * (6 * sizeof(double2) + 1) + 256;
}

__global__ void k_isign_vjp(const double2* alpha, const double* beta, const double2* gamma,
                            const double2* xbar, int k, double h, int n0, int nnode,
                            VjpScratch sc) {
  const int nthr = 2 * nnode;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nthr) return;
  const double tau = exp((double)(n0 + (t >> 1)) * h);
  const double sigma = (t & 1) ? -tau : tau;
#define AT(arr, i) arr[(long)(i) * nthr + t]
  for (int i = 0; i < k; ++i) {
    const Cx<double> a = c64(alpha[i]);
    AT(sc.d, i) = make_double2(a.re, a.im + sigma);
    if (i < k - 1) {
      AT(sc.dl, i) = make_double2(beta[i], 0.0);
      AT(sc.du, i) = gamma[i];
    }
  }
  // factor
  for (int i = 0; i < k - 1; ++i) {
    const Cx<double> di = c64(AT(sc.d, i)), li = c64(AT(sc.dl, i));
    if (cabs1(di) >= cabs1(li)) {
      const Cx<double> f = cdiv(li, di);
      AT(sc.dl, i) = d2(f);
      AT(sc.d, i + 1) = d2(c64(AT(sc.d, i + 1)) - cmul(f, c64(AT(sc.du, i))));
      if (i < k - 2) AT(sc.du2, i) = make_double2(0.0, 0.0);
      AT(sc.piv, i) = 0;
    } else {
      const Cx<double> f = cdiv(di, li);
      const Cx<double> dn = c64(AT(sc.d, i + 1));
      const Cx<double> ui = c64(AT(sc.du, i));
      AT(sc.d, i) = d2(li);
      AT(sc.dl, i) = d2(f);
      AT(sc.du, i) = d2(dn);
      AT(sc.d, i + 1) = d2(ui - cmul(f, dn));
      if (i < k - 2) {
        const Cx<double> un = c64(AT(sc.du, i + 1));
        AT(sc.du2, i) = d2(un);
        AT(sc.du, i + 1) = d2(-cmul(f, un));
      }
      AT(sc.piv, i) = 1;
    }
  }
  // q = M^{-1} e_1: L then U
  for (int i = 0; i < k; ++i) AT(sc.q, i) = make_double2(i == 0 ? 1.0 : 0.0, 0.0);
  for (int i = 0; i < k - 1; ++i) {
    const Cx<double> f = c64(AT(sc.dl, i));
    if (AT(sc.piv, i)) {
      const Cx<double> bi = c64(AT(sc.q, i)), bn = c64(AT(sc.q, i + 1));
      AT(sc.q, i) = d2(bn);
      AT(sc.q, i + 1) = d2(bi - cmul(f, bn));
    } else {
      AT(sc.q, i + 1) = d2(c64(AT(sc.q, i + 1)) - cmul(f, c64(AT(sc.q, i))));
    }
  }
  for (int i = k - 1; i >= 0; --i) {
    Cx<double> b = c64(AT(sc.q, i));
    if (i + 1 < k) b = b - cmul(c64(AT(sc.du, i)), c64(AT(sc.q, i + 1)));
    if (i + 2 < k) b = b - cmul(c64(AT(sc.du2, i)), c64(AT(sc.q, i + 2)));
    AT(sc.q, i) = d2(cdiv(b, c64(AT(sc.d, i))));
  }
  // p = M^{-H} xbar: U^H then L^H
  for (int i = 0; i < k; ++i) {
    Cx<double> b = c64(xbar[i]);
    if (i >= 1) b = b - cmulc(c64(AT(sc.du, i - 1)), c64(AT(sc.p, i - 1)));
    if (i >= 2) b = b - cmulc(c64(AT(sc.du2, i - 2)), c64(AT(sc.p, i - 2)));
    AT(sc.p, i) = d2(cdiv(b, cconj(c64(AT(sc.d, i)))));
  }
  for (int i = k - 2; i >= 0; --i) {
    const Cx<double> f = c64(AT(sc.dl, i));
    const Cx<double> bi = c64(AT(sc.p, i)), bn = c64(AT(sc.p, i + 1));
    const Cx<double> v = bi - cmulc(f, bn);
    if (AT(sc.piv, i)) {
      AT(sc.p, i) = d2(bn);
      AT(sc.p, i + 1) = d2(v);
    } else {
      AT(sc.p, i) = d2(v);
    }
  }
#undef AT
}

// Sums over nodes (fixed order) with the trapezoid weights h tau / pi.  With
// coarse.x set, also the rule of step 2h (the nodes of even index, weights
// 2 h tau / pi) into coarse (x, gd, gsup), for the first comparison of two
// levels without a launch at step 2h.
__global__ void k_isign_vjp_reduce(int k, double h, int n0, int nnode, VjpScratch sc,
                                   IsignVjpOut out, IsignVjpOut coarse) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const int nthr = 2 * nnode;
  const bool two = coarse.x != nullptr;
  Cx<double> x = {0.0, 0.0}, gd = {0.0, 0.0}, gs = {0.0, 0.0}, gu = {0.0, 0.0};
  Cx<double> xc = {0.0, 0.0}, gdc = {0.0, 0.0}, guc = {0.0, 0.0};
  for (int t = 0; t < nthr; ++t) {
    const int node = n0 + (t >> 1);
    const double w = h * exp((double)node * h) / M_PI;
    const Cx<double> qi = c64(sc.q[(long)i * nthr + t]);
    const Cx<double> pi_ = c64(sc.p[(long)i * nthr + t]);
    x = x + scale(w, qi);
    gd = gd - scale(w, cmulc(qi, pi_));
    const bool even = two && (node & 1) == 0;
    if (even) {
      xc = xc + scale(2.0 * w, qi);
      gdc = gdc - scale(2.0 * w, cmulc(qi, pi_));
    }
    if (i + 1 < k) {
      const Cx<double> qn = c64(sc.q[(long)(i + 1) * nthr + t]);
      const Cx<double> pn = c64(sc.p[(long)(i + 1) * nthr + t]);
      gs = gs - scale(w, cmulc(qi, pn));   // Gbar_{i+1,i} = -p_{i+1} conj(q_i)
      gu = gu - scale(w, cmulc(qn, pi_));  // Gbar_{i,i+1} = -p_i conj(q_{i+1})
      if (even) guc = guc - scale(2.0 * w, cmulc(qn, pi_));
    }
  }
  out.x[i] = d2(x);
  out.gd[i] = d2(gd);
  if (i + 1 < k) {
    out.gsub_re[i] = gs.re;
    out.gsup[i] = d2(gu);
  }
  if (two) {
    coarse.x[i] = d2(xc);
    coarse.gd[i] = d2(gdc);
    if (i + 1 < k) coarse.gsup[i] = d2(guc);
  }
}

void launch_isign_vjp(const double2* alpha, const double* beta, const double2* gamma,
                      const double2* xbar, int k, double h, int n0, int nnode, void* scratch,
                      const IsignVjpOut& out, hipStream_t st, const IsignVjpOut* coarse) {
  const int nthr = 2 * nnode;
  const VjpScratch sc = carve(scratch, k, nthr);
  hipLaunchKernelGGL(k_isign_vjp, dim3((nthr + 63) / 64), dim3(64), 0, st, alpha, beta, gamma,
                     xbar, k, h, n0, nnode, sc);
  const IsignVjpOut none{};
  hipLaunchKernelGGL(k_isign_vjp_reduce, dim3((k + 63) / 64), dim3(64), 0, st, k, h, n0, nnode, sc,
                     out, coarse ? *coarse : none);
}

// ---- link force -----------------------------------------------------------------
// For Re <pbar, A p>, A = gamma5 Dw with hop coefficient k eta on packed links
// U~ (boundary signs folded in), the gradient with respect to U~_nu(x) is
//   forward hop into x+nu : -k eta+ sum_s [(1+g_nu) g5 pbar(x+nu)]_s [p(x)]_s^dagger
//   backward hop into x   : -k eta- sum_s [(1-g_nu) p(x+nu)]_s [g5 pbar(x)]_s^dagger
// (colour outer products summed over spin).  With (1 +- g_nu) = E P, P the
// two-row projection of the stencil and E = P^dagger, each sum reduces to two
// outer products of projected half spinors.

struct HopPair {
  double fA[4], bA[4], fAd[4], bAd[4];
};

__device__ __forceinline__ void load_sp(const double2* f, long Vs, int s, bool g5,
                                        Cx<double> (&p)[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    p[c] = c64(f[fidx(c, s, Vs)]);
    if (g5 && c >= 6) p[c] = -p[c];
  }
}

// F[a][b] += c * sum_k h_k[a] conj(g_k[b])
__device__ __forceinline__ void outer_acc(Cx<double> (&F)[9], const Cx<double> (&h)[6],
                                          const Cx<double> (&g)[6], double c) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const Cx<double> v = cmulc(g[b], h[a]) + cmulc(g[3 + b], h[3 + a]);
      F[3 * a + b] = F[3 * a + b] + scale(c, v);
    }
}

// forward and backward hop terms of one (adjoint, input) pair
template <int NU>
__device__ __forceinline__ void force_pair(Cx<double> (&Ff)[9], Cx<double> (&Fb)[9],
                                           const double2* bar, const double2* in, long Vs, int s,
                                           int sf, double cf, double cb) {
  Cx<double> a[12], b[12], h[6], g[6];
  load_sp(bar, Vs, sf, true, a);
  project<double, NU, +1>(a, h);
  load_sp(in, Vs, s, false, b);
  project<double, NU, +1>(b, g);
  outer_acc(Ff, h, g, -cf);
  load_sp(in, Vs, sf, false, a);
  project<double, NU, -1>(a, h);
  load_sp(bar, Vs, s, true, b);
  project<double, NU, -1>(b, g);
  outer_acc(Fb, h, g, -cb);
}

template <int NU>
__device__ __forceinline__ void force_dir(double2* F, const double2* pbar, const double2* p,
                                          const double2* qbar, const double2* q, long stride,
                                          int nrhs, const Geometry& g, int s, int sf,
                                          const HopPair& hp) {
  const long Vs = g.Vs;
  Cx<double> fp[9], fm[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) fp[e] = fm[e] = {0.0, 0.0};
  for (int r = 0; r < nrhs; ++r) {
    const long o = (long)r * stride;
    // A(mu): forward carries e^{+mu}, backward e^{-mu}
    if constexpr (NU == 3) force_pair<NU>(fp, fm, pbar + o, p + o, Vs, s, sf, hp.fA[NU], hp.bA[NU]);
    else force_pair<NU>(fp, fp, pbar + o, p + o, Vs, s, sf, hp.fA[NU], hp.bA[NU]);
    if (qbar) {
      // A(mu)^dagger = A(-mu): forward carries e^{-mu}, backward e^{+mu}
      if constexpr (NU == 3)
        force_pair<NU>(fm, fp, qbar + o, q + o, Vs, s, sf, hp.fAd[NU], hp.bAd[NU]);
      else force_pair<NU>(fp, fp, qbar + o, q + o, Vs, s, sf, hp.fAd[NU], hp.bAd[NU]);
    }
  }
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    double2* dst = F + ((long)NU * 9 + e) * Vs + s;
    *dst = d2(c64(*dst) + fp[e]);
  }
  if constexpr (NU == 3) {
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      double2* dst = F + ((long)4 * 9 + e) * Vs + s;
      *dst = d2(c64(*dst) + fm[e]);
    }
  }
}

__global__ void __launch_bounds__(kWG) k_gforce(double2* F, const double2* pbar, const double2* p,
                                                const double2* qbar, const double2* q, long stride,
                                                int nrhs, Geometry g, HopPair hp) {
  // one thread per site and direction (blockIdx.y): each direction writes
  // only its own slots of F, so the directions are independent
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const Nbr nb = neighbours(s, g);
  switch (blockIdx.y) {
    case 0: force_dir<0>(F, pbar, p, qbar, q, stride, nrhs, g, s, nb.f[0], hp); break;
    case 1: force_dir<1>(F, pbar, p, qbar, q, stride, nrhs, g, s, nb.f[1], hp); break;
    case 2: force_dir<2>(F, pbar, p, qbar, q, stride, nrhs, g, s, nb.f[2], hp); break;
    default: force_dir<3>(F, pbar, p, qbar, q, stride, nrhs, g, s, nb.f[3], hp); break;
  }
}

static HopPair hop_pair(const Hop& hA, const Hop& hAd) {
  HopPair hp;
  for (int nu = 0; nu < 4; ++nu) {
    hp.fA[nu] = hA.fwd[nu];
    hp.bA[nu] = hA.bwd[nu];
    hp.fAd[nu] = hAd.fwd[nu];
    hp.bAd[nu] = hAd.bwd[nu];
  }
  return hp;
}

void launch_gforce(double2* F, const double2* pbar, const double2* p, const double2* qbar,
                   const double2* q, long stride, int nrhs, const Geometry& g, const Hop& hA,
                   const Hop& hAd, hipStream_t st) {
  const HopPair hp = hop_pair(hA, hAd);
  hipLaunchKernelGGL(k_gforce, dim3((g.V + kWG - 1) / kWG, 4), dim3(kWG), 0, st, F, pbar, p, qbar,
                     q, stride, nrhs, g, hp);
}

// The force of n consecutive reverse steps in one pass: the contributions of
// every step and source are summed in registers (steps in order, then
// sources, as force_dir sums the sources of one step) and F is read and
// written once, not once per step.  Step j's fields are at pbar0 + j *
// step_stride etc.
template <int NU>
__device__ __forceinline__ void force_dir_group(double2* F, const double2* pbar0,
                                                const double2* p0, const double2* qbar0,
                                                const double2* q0, int nsteps, long step_stride,
                                                long stride, int nrhs, const Geometry& g, int s,
                                                int sf, const HopPair& hp) {
  const long Vs = g.Vs;
  Cx<double> fp[9], fm[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) fp[e] = fm[e] = {0.0, 0.0};
  for (int j = 0; j < nsteps; ++j) {
    const long js = (long)j * step_stride;
    for (int r = 0; r < nrhs; ++r) {
      const long o = js + (long)r * stride;
      if constexpr (NU == 3) {
        force_pair<NU>(fp, fm, pbar0 + o, p0 + o, Vs, s, sf, hp.fA[NU], hp.bA[NU]);
        force_pair<NU>(fm, fp, qbar0 + o, q0 + o, Vs, s, sf, hp.fAd[NU], hp.bAd[NU]);
      } else {
        force_pair<NU>(fp, fp, pbar0 + o, p0 + o, Vs, s, sf, hp.fA[NU], hp.bA[NU]);
        force_pair<NU>(fp, fp, qbar0 + o, q0 + o, Vs, s, sf, hp.fAd[NU], hp.bAd[NU]);
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    double2* dst = F + ((long)NU * 9 + e) * Vs + s;
    *dst = d2(c64(*dst) + fp[e]);
  }
  if constexpr (NU == 3) {
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      double2* dst = F + ((long)4 * 9 + e) * Vs + s;
      *dst = d2(c64(*dst) + fm[e]);
    }
  }
}

__global__ void __launch_bounds__(kWG) k_gforce_group(double2* F, const double2* pbar0,
                                                      const double2* p0, const double2* qbar0,
                                                      const double2* q0, int nsteps,
                                                      long step_stride, long stride, int nrhs,
                                                      Geometry g, HopPair hp) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const Nbr nb = neighbours(s, g);
  switch (blockIdx.y) {
    case 0: force_dir_group<0>(F, pbar0, p0, qbar0, q0, nsteps, step_stride, stride, nrhs, g, s, nb.f[0], hp); break;
    case 1: force_dir_group<1>(F, pbar0, p0, qbar0, q0, nsteps, step_stride, stride, nrhs, g, s, nb.f[1], hp); break;
    case 2: force_dir_group<2>(F, pbar0, p0, qbar0, q0, nsteps, step_stride, stride, nrhs, g, s, nb.f[2], hp); break;
    default: force_dir_group<3>(F, pbar0, p0, qbar0, q0, nsteps, step_stride, stride, nrhs, g, s, nb.f[3], hp); break;
  }
}

void launch_gforce_group(double2* F, const double2* pbar0, const double2* p0,
                         const double2* qbar0, const double2* q0, int nsteps, long step_stride,
                         long stride, int nrhs, const Geometry& g, const Hop& hA, const Hop& hAd,
                         hipStream_t st) {
  const HopPair hp = hop_pair(hA, hAd);
  hipLaunchKernelGGL(k_gforce_group, dim3((g.V + kWG - 1) / kWG, 4), dim3(kWG), 0, st, F, pbar0,
                     p0, qbar0, q0, nsteps, step_stride, stride, nrhs, g, hp);
}

__global__ void __launch_bounds__(kWG) k_gforce_out(const double2* F, const double2* links,
                                                    Geometry g, int bc0, int bc1, int bc2, int bc3,
                                                    double2* grad_U, double* partials) {
  __shared__ double lds[(kWG / 64)];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double part[1] = {0.0};
  if (s < g.V) {
    const int x = s % g.lx, y = (s / g.lx) % g.ly, z = (s / (g.lx * g.ly)) % g.lz,
              t = s / (g.lx * g.ly * g.lz);
    const int coord[4] = {x, y, z, t};
    const int ext[4] = {g.lx, g.ly, g.lz, g.lt};
    const int bc[4] = {bc0, bc1, bc2, bc3};
    for (int nu = 0; nu < 4; ++nu) {
      const double sg = (coord[nu] == ext[nu] - 1 && bc[nu] < 0) ? -1.0 : 1.0;
      for (int e = 0; e < 9; ++e) {
        Cx<double> v = c64(F[((long)nu * 9 + e) * g.Vs + s]);
        if (nu == 3) {
          const Cx<double> vm = c64(F[((long)4 * 9 + e) * g.Vs + s]);
          const Cx<double> u = c64(links[lidx(3, e, s, g.Vs)]);
          part[0] += cmulc(v, u).re - cmulc(vm, u).re;
          v = v + vm;
        }
        grad_U[((long)s * 4 + nu) * 9 + e] = d2(scale(sg, v));
      }
    }
  }
  block_sum<1>(part, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = part[0];
}

__global__ void k_sum_partials(const double* partials, int n, double* out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double a = 0.0;
  for (int i = 0; i < n; ++i) a += partials[i];
  *out = a;
}

void launch_gforce_out(const double2* F, const double2* links, const Geometry& g, const int bc[4],
                       double2* grad_U, double* partials, double* grad_mu, hipStream_t st) {
  const int nb = (g.V + kWG - 1) / kWG;
  hipLaunchKernelGGL(k_gforce_out, dim3(nb), dim3(kWG), 0, st, F, links, g, bc[0], bc[1], bc[2],
                     bc[3], grad_U, partials);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1), 0, st, partials, nb, grad_mu);
}

}  // namespace ovs

namespace ovs {

// ---- su(3) link force ------------------------------------------------------
// F = -TA(U G^dagger) per link, TA(M) = (M - M^dagger)/2 - tr(M - M^dagger)/6:
// the force of a real L(U) for U -> exp(eps X) U, X in su(3), from its link
// gradient G = dL/dRe U + i dL/dIm U.  Canonical layout [V][4][3][3].
__global__ void __launch_bounds__(kWG) k_link_force(const double2* __restrict__ U,
                                                    const double2* __restrict__ G,
                                                    double2* __restrict__ F, long nlinks) {
  const long n = (long)blockIdx.x * kWG + threadIdx.x;
  if (n >= nlinks) return;
  Cx<double> u[9], g[9], m[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    u[e] = c64(U[n * 9 + e]);
    g[e] = c64(G[n * 9 + e]);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      Cx<double> s = {0.0, 0.0};
#pragma unroll
      for (int c = 0; c < 3; ++c) s = cfmac(g[b * 3 + c], u[a * 3 + c], s);  // U_ac conj(G_bc)
      m[a * 3 + b] = s;
    }
  // trace of the anti-Hermitian part: i Im tr M
  const double imtr = (m[0].im + m[4].im + m[8].im) / 3.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const Cx<double> x = m[a * 3 + b], y = m[b * 3 + a];
      Cx<double> t = {0.5 * (x.re - y.re), 0.5 * (x.im + y.im)};  // (M - M^dagger)/2
      if (a == b) t.im -= imtr;
      F[n * 9 + a * 3 + b] = d2(-t);
    }
}

void launch_link_force(const double2* U, const double2* G, double2* F, long nlinks,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_link_force, dim3((unsigned)((nlinks + kWG - 1) / kWG)), dim3(kWG), 0, s,
                     U, G, F, nlinks);
}

}  // namespace ovs
