// Spin structure of the Wilson hops (chiral gamma basis) and lattice
// neighbours, shared by the stencil and the link-force kernels.
#pragma once

#include "ovs_common.h"
#include "ovs_device.h"

namespace ovs {

// ---- spin projection and reconstruction (chiral basis) -------------------
// Component index 3*spin + colour.  For direction NU and sign S (+1: the
// (1 + g_nu) hop from y - nu, -1: the (1 - g_nu) hop from y + nu) the half
// spinor h = (h0, h1) carries the two independent spin rows; the lower rows
// of (1 + S g_nu) psi are fixed multiples of h0, h1.

template <typename R, int NU, int S>
__device__ __forceinline__ void project(const Cx<R> (&p)[12], Cx<R> (&h)[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const Cx<R> p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
    if constexpr (NU == 0) {        // h0 = p0 - S i p3, h1 = p1 - S i p2
      h[c] = (S > 0) ? p0 - mul_i(p3) : p0 + mul_i(p3);
      h[3 + c] = (S > 0) ? p1 - mul_i(p2) : p1 + mul_i(p2);
    } else if constexpr (NU == 1) { // h0 = p0 - S p3, h1 = p1 + S p2
      h[c] = (S > 0) ? p0 - p3 : p0 + p3;
      h[3 + c] = (S > 0) ? p1 + p2 : p1 - p2;
    } else if constexpr (NU == 2) { // h0 = p0 - S i p2, h1 = p1 + S i p3
      h[c] = (S > 0) ? p0 - mul_i(p2) : p0 + mul_i(p2);
      h[3 + c] = (S > 0) ? p1 + mul_i(p3) : p1 - mul_i(p3);
    } else {                        // h0 = p0 + S p2, h1 = p1 + S p3
      h[c] = (S > 0) ? p0 + p2 : p0 - p2;
      h[3 + c] = (S > 0) ? p1 + p3 : p1 - p3;
    }
  }
}

// acc += coef * (1 + S g_nu)-expansion of uh
template <typename R, int NU, int S>
__device__ __forceinline__ void expand_acc(Cx<R> (&acc)[12], const Cx<R> (&uh)[6], R coef) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const Cx<R> a = scale(coef, uh[c]);      // coef * U h0
    const Cx<R> b = scale(coef, uh[3 + c]);  // coef * U h1
    acc[c] = acc[c] + a;
    acc[3 + c] = acc[3 + c] + b;
    if constexpr (NU == 0) {        // r2 = S i h1, r3 = S i h0
      acc[6 + c] = (S > 0) ? acc[6 + c] + mul_i(b) : acc[6 + c] - mul_i(b);
      acc[9 + c] = (S > 0) ? acc[9 + c] + mul_i(a) : acc[9 + c] - mul_i(a);
    } else if constexpr (NU == 1) { // r2 = S h1, r3 = -S h0
      acc[6 + c] = (S > 0) ? acc[6 + c] + b : acc[6 + c] - b;
      acc[9 + c] = (S > 0) ? acc[9 + c] - a : acc[9 + c] + a;
    } else if constexpr (NU == 2) { // r2 = S i h0, r3 = -S i h1
      acc[6 + c] = (S > 0) ? acc[6 + c] + mul_i(a) : acc[6 + c] - mul_i(a);
      acc[9 + c] = (S > 0) ? acc[9 + c] - mul_i(b) : acc[9 + c] + mul_i(b);
    } else {                        // r2 = S h0, r3 = S h1
      acc[6 + c] = (S > 0) ? acc[6 + c] + a : acc[6 + c] - a;
      acc[9 + c] = (S > 0) ? acc[9 + c] + b : acc[9 + c] - b;
    }
  }
}

// U h (DAG = false) or U^dagger h (DAG = true) on both halves.
template <typename R, bool DAG>
__device__ __forceinline__ void link_mul(const Cx<R> (&u)[9], const Cx<R> (&h)[6], Cx<R> (&uh)[6]) {
#pragma unroll
  for (int half = 0; half < 2; ++half) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Cx<R> sum = {R(0), R(0)};
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if constexpr (DAG) sum = cfmac(u[3 * b + a], h[3 * half + b], sum);
        else sum = cfma(u[3 * a + b], h[3 * half + b], sum);
      }
      uh[3 * half + a] = sum;
    }
  }
}

template <typename R, int NU, int S, bool DAG>
__device__ __forceinline__ void hop(Cx<R> (&acc)[12], const Cx<R> (&u)[9], const Cx<R> (&psi)[12], R coef) {
  Cx<R> h[6], uh[6];
  project<R, NU, S>(psi, h);
  link_mul<R, DAG>(u, h, uh);
  expand_acc<R, NU, S>(acc, uh, coef);
}

// Neighbour sites of s in the four directions (periodic index wrap; the
// boundary signs live in the packed links).
struct Nbr {
  int b[4], f[4];
};

__device__ __forceinline__ Nbr neighbours(int s, const Geometry& g) {
  Nbr n;
  const int x = s % g.lx;
  const int r1 = s / g.lx;
  const int y = r1 % g.ly;
  const int r2 = r1 / g.ly;
  const int z = r2 % g.lz;
  const int t = r2 / g.lz;
  const int sy = g.lx, sz = g.lx * g.ly, st_ = g.lx * g.ly * g.lz;
  n.f[0] = (x == g.lx - 1) ? s - (g.lx - 1) : s + 1;
  n.b[0] = (x == 0) ? s + (g.lx - 1) : s - 1;
  n.f[1] = (y == g.ly - 1) ? s - (g.ly - 1) * sy : s + sy;
  n.b[1] = (y == 0) ? s + (g.ly - 1) * sy : s - sy;
  n.f[2] = (z == g.lz - 1) ? s - (g.lz - 1) * sz : s + sz;
  n.b[2] = (z == 0) ? s + (g.lz - 1) * sz : s - sz;
  n.f[3] = (t == g.lt - 1) ? s - (g.lt - 1) * st_ : s + st_;
  n.b[3] = (t == 0) ? s + (g.lt - 1) * st_ : s - st_;
  return n;
}

// ---- field and link access (component-pair layout) ----------------------

template <typename T2, typename R>
__device__ __forceinline__ void load_spinor(const T2* __restrict__ f, int V, int site, bool g5,
                                            Cx<R> (&p)[12]) {
#pragma unroll
  for (int q = 0; q < 6; ++q) ld_pair(f + fidx(2 * q, site, V), p[2 * q], p[2 * q + 1]);
  if (g5) {
#pragma unroll
    for (int c = 6; c < 12; ++c) p[c] = -p[c];
  }
}

template <typename T2, typename R>
__device__ __forceinline__ void load_link(const T2* __restrict__ links, int V, int nu, int site,
                                          Cx<R> (&u)[9]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) ld_pair(links + lidx(nu, 2 * q, site, V), u[2 * q], u[2 * q + 1]);
  u[8] = ld(links + lidx(nu, 8, site, V));
}

// out[c] for c = 0..11 of one site, as six pair stores (streaming if nt).
template <typename T2, typename R>
__device__ __forceinline__ void store_spinor(T2* __restrict__ f, int V, int site, int nt,
                                             const Cx<R> (&o)[12]) {
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    if (nt) st_pair_nt(f + fidx(2 * q, site, V), o[2 * q], o[2 * q + 1]);
    else st_pair(f + fidx(2 * q, site, V), o[2 * q], o[2 * q + 1]);
  }
}


template <typename R> struct HopR;
template <> struct HopR<double> {
  double fwd[4], bwd[4];
  static HopR make(const Hop& h) {
    HopR r;
    for (int i = 0; i < 4; ++i) { r.fwd[i] = h.fwd[i]; r.bwd[i] = h.bwd[i]; }
    return r;
  }
};
template <> struct HopR<float> {
  float fwd[4], bwd[4];
  static HopR make(const Hop& h) {
    HopR r;
    for (int i = 0; i < 4; ++i) { r.fwd[i] = h.f32_fwd[i]; r.bwd[i] = h.f32_bwd[i]; }
    return r;
  }
};

}  // namespace ovs
