// Coefficient steps of the two-sided Lanczos iteration (Section 4): the
// bodies shared by the per-step kernels (krylov.hip) and the persistent
// Lanczos kernel.  Each body takes its workgroup's (virtual) index and the
// iteration index explicitly; every return is uniform over the workgroup.
#pragma once

#include "ovs_common.h"
#include "ovs_device.h"

namespace ovs {

// alpha_i = conj(sw_i) sv_i (W~^dag A V~),  |t|^2 = sv_i^2 |A V~|^2, from the
// dual stencil's per-tile partials of source slot rhs_map[jj].
__device__ __forceinline__ void alpha_body(int jj, int i, const double* __restrict__ partials,
                                           int nparts, const CoefArrays& co,
                                           const int* __restrict__ rhs_map, int na) {
  __shared__ double lds[4 * 3];
  if (jj >= na) return;
  const int slot = rhs_map[jj];
  double v[3] = {0, 0, 0};
  for (int p = threadIdx.x; p < nparts; p += blockDim.x)
    for (int t = 0; t < 3; ++t) v[t] += partials[((long)slot * nparts + p) * 3 + t];
  block_sum<3>(v, lds);
  if (threadIdx.x == 0) {
    const double sv = co.sv[(long)slot * (co.kmax + 1) + i];
    const Cx<double> sw = c64(co.sw[(long)slot * (co.kmax + 1) + i]);
    const Cx<double> a = scale(sv, cmulc(sw, Cx<double>{v[0], v[1]}));
    co.alpha[(long)slot * co.kmax + i] = d2(a);
    co.tnorm2[(long)slot * co.kmax + i] = sv * sv * v[2];
  }
}

// v~ = sv_i T - alpha sv_i V~_i - gamma_{i-1} sv_{i-1} V~_{i-1}
// w~ = sw_i S - conj(alpha) sw_i W~_i - conj(beta_{i-1}) sw_{i-1} W~_{i-1}
// partials [slot][gx][4] = (delta.re, delta.im, |v~|^2, |w~|^2) for workgroup
// (bx, by) of a gx-wide grid over the field (by: the active source).
//
// With apart != nullptr alpha is formed here: every workgroup reduces the dual
// stencil's partials of its source in alpha_body's order (same workgroup
// size, so the same alpha to the last bit), and workgroup bx = 0 stores alpha
// and |t|^2; otherwise alpha is read from co.
template <typename T2>
__device__ __forceinline__ void update_body(int bx, int by, int gx, int i,
                                            const T2* __restrict__ T, const T2* __restrict__ S,
                                            T2* __restrict__ basis, long basis_stride,
                                            T2* __restrict__ wbuf, long slot_stride, long N,
                                            const CoefArrays& co, const int* __restrict__ rhs_map,
                                            int na, double* __restrict__ partials,
                                            int two_pass_ring, const double* __restrict__ apart,
                                            int anparts, int nt) {
  __shared__ double lds[4 * 4];
  __shared__ double abc[2];
  const int jj = by;
  if (jj >= na) return;
  const int slot = rhs_map[jj];
  const long ks = co.kmax;
  const double svi = co.sv[slot * (ks + 1) + i];
  const Cx<double> swi = c64(co.sw[slot * (ks + 1) + i]);
  Cx<double> a;
  if (apart) {
    double av[3] = {0, 0, 0};
    for (int p = threadIdx.x; p < anparts; p += blockDim.x)
      for (int t = 0; t < 3; ++t) av[t] += apart[((long)slot * anparts + p) * 3 + t];
    block_sum<3>(av, lds);
    if (threadIdx.x == 0) {
      const Cx<double> aa = scale(svi, cmulc(swi, Cx<double>{av[0], av[1]}));
      abc[0] = aa.re;
      abc[1] = aa.im;
      if (bx == 0) {
        co.alpha[slot * ks + i] = d2(aa);
        co.tnorm2[slot * ks + i] = svi * svi * av[2];
      }
    }
    __syncthreads();
    a = {abc[0], abc[1]};
  } else {
    a = c64(co.alpha[slot * ks + i]);
  }
  const bool prev = i > 0;
  const double svm = prev ? co.sv[slot * (ks + 1) + i - 1] : 0.0;
  const Cx<double> swm = prev ? c64(co.sw[slot * (ks + 1) + i - 1]) : Cx<double>{0, 0};
  const Cx<double> gm = prev ? c64(co.gamma[slot * ks + i - 1]) : Cx<double>{0, 0};
  const double bm = prev ? co.beta[slot * ks + i - 1] : 0.0;
  const Cx<double> c1 = {svi, 0.0};
  const Cx<double> c2 = scale(-svi, a);
  const Cx<double> c3 = scale(-svm, gm);
  const Cx<double> d1 = swi;
  const Cx<double> d2_ = -cmulc(a, swi);           // -conj(alpha) sw_i
  const Cx<double> d3 = scale(-bm, swm);           // -conj(beta) sw_{i-1}, beta real
  // basis slots: ring of 3 in two-pass mode, else the full basis
  const long vi = two_pass_ring ? (i % 3) : i;
  const long vm = two_pass_ring ? ((i + 2) % 3) : (i - 1);
  const long vn = two_pass_ring ? ((i + 1) % 3) : (i + 1);
  const T2* Vi = basis + vi * basis_stride + slot * slot_stride;
  const T2* Vm = basis + (prev ? vm : vi) * basis_stride + slot * slot_stride;
  T2* Vn = basis + vn * basis_stride + slot * slot_stride;
  const T2* Wi = wbuf + (long)(i % 3) * basis_stride + slot * slot_stride;
  const T2* Wm = wbuf + (long)((i + 2) % 3) * basis_stride + slot * slot_stride;
  T2* Wn = wbuf + (long)((i + 1) % 3) * basis_stride + slot * slot_stride;
  const T2* Ts = T + slot * slot_stride;
  const T2* Ss = S + slot * slot_stride;
  double v[4] = {0, 0, 0, 0};
  // two adjacent complex elements per thread (one 16-byte access per vector in
  // FP32); N is even (12 Vs)
  for (long e = 2 * (bx * (long)blockDim.x + threadIdx.x); e < N;
       e += 2 * (long)gx * blockDim.x) {
    Cx<double> vt[2], wt[2];
    {
      Cx<double> x0, x1, y0, y1;
      ld_pair64(Ts + e, x0, x1);
      ld_pair64(Vi + e, y0, y1);
      vt[0] = cfma(c2, y0, cmul(c1, x0));
      vt[1] = cfma(c2, y1, cmul(c1, x1));
      ld_pair64(Ss + e, x0, x1);
      ld_pair64(Wi + e, y0, y1);
      wt[0] = cfma(d2_, y0, cmul(d1, x0));
      wt[1] = cfma(d2_, y1, cmul(d1, x1));
      if (prev) {
        ld_pair64(Vm + e, x0, x1);
        ld_pair64(Wm + e, y0, y1);
        vt[0] = cfma(c3, x0, vt[0]);
        vt[1] = cfma(c3, x1, vt[1]);
        wt[0] = cfma(d3, y0, wt[0]);
        wt[1] = cfma(d3, y1, wt[1]);
      }
    }
    if (nt) {
      st_pair64_nt(Vn + e, vt[0], vt[1]);
      st_pair64_nt(Wn + e, wt[0], wt[1]);
    } else {
      st_pair64(Vn + e, vt[0], vt[1]);
      st_pair64(Wn + e, wt[0], wt[1]);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const Cx<double> vr = round_to(Vn, vt[q]), wr = round_to(Wn, wt[q]);
      const Cx<double> dl = cmulc(wr, vr);
      v[0] += dl.re;
      v[1] += dl.im;
      v[2] += cnorm2(vr);
      v[3] += cnorm2(wr);
    }
  }
  block_sum<4>(v, lds);
  if (threadIdx.x == 0)
    for (int t = 0; t < 4; ++t) partials[((long)slot * gx + bx) * 4 + t] = v[t];
}

// beta_i = |v~|, gamma_i = delta / beta_i, and the breakdown tests: lucky
// when |v~| <= 1e-14 |A v_i| (the Krylov space is invariant), serious when
// |delta| <= 1e-13 |v~| |w~| (no biorthogonal continuation); either stops the
// source at k = i + 1 with zero coefficients from there on.  With probes !=
// nullptr the entries idx[0..P) of the new V~_{i+1} are gathered as well.
template <typename T2>
__device__ __forceinline__ void beta_body(int jj, int i, const double* __restrict__ partials,
                                          int nparts, const CoefArrays& co,
                                          const int* __restrict__ rhs_map, int na,
                                          const T2* __restrict__ basis, long basis_stride, long N,
                                          int ring, const int* __restrict__ idx, int P,
                                          double2* __restrict__ probes) {
  __shared__ double lds[4 * 4];
  if (jj >= na) return;
  const int slot = rhs_map[jj];
  double v[4] = {0, 0, 0, 0};
  for (int p = threadIdx.x; p < nparts; p += blockDim.x)
    for (int t = 0; t < 4; ++t) v[t] += partials[((long)slot * nparts + p) * 4 + t];
  block_sum<4>(v, lds);
  if (threadIdx.x == 0) {
    const long ks = co.kmax;
    const double bn = sqrt(v[2]), wn = sqrt(v[3]);
    const Cx<double> delta = {v[0], v[1]};
    const double tn = sqrt(co.tnorm2[slot * ks + i]);
    int st_ = co.status[slot];
    if (st_ == 0) {
      const bool forced = co.inject_plus1 == i + 1;
      if (co.dnorm) co.dnorm[slot * ks + i] = forced ? 0.0 : cabs1(delta) / (bn * wn);
      if (!(bn > 1e-14 * tn)) st_ = 1;
      else if (forced || !(cabs1(delta) > 1e-13 * bn * wn)) st_ = 2;
      if (st_ != 0) {
        co.status[slot] = st_;
        co.kstop[slot] = i + 1;
      }
    }
    if (st_ == 0) {
      const Cx<double> g = scale(1.0 / bn, delta);
      co.beta[slot * ks + i] = bn;
      co.gamma[slot * ks + i] = d2(g);
      co.sv[slot * (ks + 1) + i + 1] = 1.0 / bn;
      co.sw[slot * (ks + 1) + i + 1] = d2(cdiv(Cx<double>{1.0, 0.0}, Cx<double>{g.re, -g.im}));
    } else {
      co.beta[slot * ks + i] = 0.0;
      co.gamma[slot * ks + i] = make_double2(0.0, 0.0);
      co.sv[slot * (ks + 1) + i + 1] = 0.0;
      co.sw[slot * (ks + 1) + i + 1] = make_double2(0.0, 0.0);
    }
  }
  const int j = i + 1;
  if (probes && j < co.kmax) {
    const long sl = ring ? (j % 3) : j;
    const T2* vb = basis + sl * basis_stride + (long)slot * N;
    for (int p = threadIdx.x; p < P; p += blockDim.x)
      probes[((long)slot * co.kmax + j) * P + p] = d2(ld64(vb + idx[p]));
  }
}

}  // namespace ovs
