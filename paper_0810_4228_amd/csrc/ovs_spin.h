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

// acc += coef * (1 + S g_nu)-expansion of uh.  Each of the four spin rows
// takes +-coef times h0, h1 or i h0, i h1 (i z = (-Im z, Re z)), accumulated
// with one fused multiply-add per real component.
template <typename R>
__device__ __forceinline__ void acc_add(Cx<R>& acc, R coef, Cx<R> a) {
  acc.re = fma(coef, a.re, acc.re);
  acc.im = fma(coef, a.im, acc.im);
}
template <typename R, int NU, int S>
__device__ __forceinline__ void expand_acc(Cx<R> (&acc)[12], const Cx<R> (&uh)[6], R coef) {
  const R cs = (S > 0) ? coef : -coef;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const Cx<R> a = uh[c];      // U h0
    const Cx<R> b = uh[3 + c];  // U h1
    acc_add(acc[c], coef, a);
    acc_add(acc[3 + c], coef, b);
    if constexpr (NU == 0) {        // r2 = S i h1, r3 = S i h0
      acc_add(acc[6 + c], cs, mul_i(b));
      acc_add(acc[9 + c], cs, mul_i(a));
    } else if constexpr (NU == 1) { // r2 = S h1, r3 = -S h0
      acc_add(acc[6 + c], cs, b);
      acc_add(acc[9 + c], -cs, a);
    } else if constexpr (NU == 2) { // r2 = S i h0, r3 = -S i h1
      acc_add(acc[6 + c], cs, mul_i(a));
      acc_add(acc[9 + c], -cs, mul_i(b));
    } else {                        // r2 = S h0, r3 = S h1
      acc_add(acc[6 + c], cs, a);
      acc_add(acc[9 + c], cs, b);
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
// A pair plane (the two components c = 2q, 2q+1 of every site, or two entries
// of one link direction) starts at a workgroup-uniform address; within it
// site s sits at byte 2 s sizeof(T2).  That offset is formed in 32 bits
// (sites < 2^27), so a load takes a scalar base and one 32-bit vector offset
// per site shared by all planes, instead of a 64-bit address per load.

template <typename T2>
__device__ __forceinline__ const T2* pair_at(const T2* plane, int site) {
  return reinterpret_cast<const T2*>(reinterpret_cast<const char*>(plane) +
                                     (unsigned)site * (unsigned)(2 * sizeof(T2)));
}
template <typename T2>
__device__ __forceinline__ T2* pair_at(T2* plane, int site) {
  return reinterpret_cast<T2*>(reinterpret_cast<char*>(plane) +
                               (unsigned)site * (unsigned)(2 * sizeof(T2)));
}

template <typename T2, typename R>
__device__ __forceinline__ void load_spinor(const T2* __restrict__ f, int V, int site, bool g5,
                                            Cx<R> (&p)[12]) {
#pragma unroll
  for (int q = 0; q < 6; ++q) ld_pair(pair_at(f + (long)q * 2 * V, site), p[2 * q], p[2 * q + 1]);
  if (g5) {
#pragma unroll
    for (int c = 6; c < 12; ++c) p[c] = -p[c];
  }
}

template <typename T2, typename R>
__device__ __forceinline__ void load_link(const T2* __restrict__ links, int V, int nu, int site,
                                          Cx<R> (&u)[9]) {
  const T2* lnu = links + (long)nu * 5 * 2 * V;
#pragma unroll
  for (int q = 0; q < 4; ++q) ld_pair(pair_at(lnu + (long)q * 2 * V, site), u[2 * q], u[2 * q + 1]);
  u[8] = ld(pair_at(lnu + (long)4 * 2 * V, site));
}

// Loads through a raw buffer resource, for a workgroup-uniform field or link
// base: the plane offset is a scalar byte offset and the site a 32-bit vector
// byte offset, so a load needs no per-lane address arithmetic.  The last
// descriptor word is the raw-buffer configuration of gfx9-family devices.
// Offsets must stay below the resource size (the library limits lattices to
// 2^24 sites, so a source field or one link direction fits in 32 bits).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t uniform_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           0x00020000);
}
// The returned vector is converted as a whole (element-wise extraction of the
// builtin's result compiled to a single-dword load here).
__device__ __forceinline__ void ld_pair_rs(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff,
                                           Cx<float>& a, Cx<float>& b) {
  const float4 v = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  a = {v.x, v.y};
  b = {v.z, v.w};
}
__device__ __forceinline__ void ld_pair_rs(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff,
                                           Cx<double>& a, Cx<double>& b) {
  const double2 v = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  const double2 w =
      __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff + 16u, soff, 0));
  a = {v.x, v.y};
  b = {w.x, w.y};
}
__device__ __forceinline__ void ld_rs(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff,
                                      Cx<float>& a) {
  const float2 v = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  a = {v.x, v.y};
}
__device__ __forceinline__ void ld_rs(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff,
                                      Cx<double>& a) {
  const double2 v = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  a = {v.x, v.y};
}

// load_spinor / load_link for a workgroup-uniform base f / links.
template <typename T2, typename R>
__device__ __forceinline__ void load_spinor_u(const T2* __restrict__ f, int V, int site, bool g5,
                                              Cx<R> (&p)[12]) {
  constexpr unsigned e2 = 2 * sizeof(T2);  // bytes of one site in a pair plane
  const __amdgpu_buffer_rsrc_t r = uniform_rsrc(f, 6u * e2 * (unsigned)V);
  const unsigned voff = (unsigned)site * e2;
#pragma unroll
  for (int q = 0; q < 6; ++q) ld_pair_rs(r, voff, (unsigned)q * e2 * (unsigned)V, p[2 * q], p[2 * q + 1]);
  if (g5) {
#pragma unroll
    for (int c = 6; c < 12; ++c) p[c] = -p[c];
  }
}

template <typename T2, typename R>
__device__ __forceinline__ void load_link_u(const T2* __restrict__ links, int V, int nu, int site,
                                            Cx<R> (&u)[9]) {
  constexpr unsigned e2 = 2 * sizeof(T2);
  const __amdgpu_buffer_rsrc_t r = uniform_rsrc(links + (long)nu * 5 * 2 * V, 5u * e2 * (unsigned)V);
  const unsigned voff = (unsigned)site * e2;
#pragma unroll
  for (int q = 0; q < 4; ++q) ld_pair_rs(r, voff, (unsigned)q * e2 * (unsigned)V, u[2 * q], u[2 * q + 1]);
  ld_rs(r, voff, 4u * e2 * (unsigned)V, u[8]);
}

// out[c] for c = 0..11 of one site, as six pair stores (streaming if nt).
template <typename T2, typename R>
__device__ __forceinline__ void store_spinor(T2* __restrict__ f, int V, int site, int nt,
                                             const Cx<R> (&o)[12]) {
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    T2* d = pair_at(f + (long)q * 2 * V, site);
    if (nt) st_pair_nt(d, o[2 * q], o[2 * q + 1]);
    else st_pair(d, o[2 * q], o[2 * q + 1]);
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
