// Device-side helpers: complex arithmetic in registers, storage conversion,
// lattice neighbours and deterministic workgroup reductions.
#pragma once

#include <hip/hip_runtime.h>

namespace ovs {

template <typename R> struct Vec2;
template <> struct Vec2<double> { using T = double2; };
template <> struct Vec2<float> { using T = float2; };

template <typename R>
struct Cx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ Cx<R> cx(R a, R b) { return Cx<R>{a, b}; }

template <typename R>
__device__ __forceinline__ Cx<R> operator+(Cx<R> a, Cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> operator-(Cx<R> a, Cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> operator-(Cx<R> a) { return {-a.re, -a.im}; }
// i * a
template <typename R>
__device__ __forceinline__ Cx<R> mul_i(Cx<R> a) { return {-a.im, a.re}; }
template <typename R>
__device__ __forceinline__ Cx<R> scale(R s, Cx<R> a) { return {s * a.re, s * a.im}; }
// a * b
template <typename R>
__device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) {
  return {fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re)};
}
// conj(a) * b
template <typename R>
__device__ __forceinline__ Cx<R> cmulc(Cx<R> a, Cx<R> b) {
  return {fma(a.re, b.re, a.im * b.im), fma(a.re, b.im, -(a.im * b.re))};
}
// acc + a * b
template <typename R>
__device__ __forceinline__ Cx<R> cfma(Cx<R> a, Cx<R> b, Cx<R> acc) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
  return acc;
}
// acc + conj(a) * b
template <typename R>
__device__ __forceinline__ Cx<R> cfmac(Cx<R> a, Cx<R> b, Cx<R> acc) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
  return acc;
}
template <typename R>
__device__ __forceinline__ R cnorm2(Cx<R> a) { return fma(a.re, a.re, a.im * a.im); }

__device__ __forceinline__ Cx<double> ld(const double2* p) {
  double2 v = *p;
  return {v.x, v.y};
}
__device__ __forceinline__ Cx<float> ld(const float2* p) {
  float2 v = *p;
  return {v.x, v.y};
}
__device__ __forceinline__ void st(double2* p, Cx<double> a) { *p = make_double2(a.re, a.im); }
__device__ __forceinline__ void st(float2* p, Cx<float> a) { *p = make_float2(a.re, a.im); }
// FP64 view of a stored value
__device__ __forceinline__ Cx<double> ld64(const double2* p) { return ld(p); }
__device__ __forceinline__ Cx<double> ld64(const float2* p) {
  float2 v = *p;
  return {(double)v.x, (double)v.y};
}
// store an FP64 value in storage precision (round to nearest)
__device__ __forceinline__ void st64(double2* p, Cx<double> a) { *p = make_double2(a.re, a.im); }
__device__ __forceinline__ void st64(float2* p, Cx<double> a) {
  *p = make_float2((float)a.re, (float)a.im);
}
// streaming (non-temporal) stores of an FP64 value in storage precision
__device__ __forceinline__ void st64_nt(double2* p, Cx<double> a) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  v2 v = {a.re, a.im};
  __builtin_nontemporal_store(v, reinterpret_cast<v2*>(p));
}
__device__ __forceinline__ void st64_nt(float2* p, Cx<double> a) {
  typedef float v2 __attribute__((ext_vector_type(2)));
  v2 v = {(float)a.re, (float)a.im};
  __builtin_nontemporal_store(v, reinterpret_cast<v2*>(p));
}
// the stored value as seen after rounding to storage precision
__device__ __forceinline__ Cx<double> round_to(const double2*, Cx<double> a) { return a; }
__device__ __forceinline__ Cx<double> round_to(const float2*, Cx<double> a) {
  return {(double)(float)a.re, (double)(float)a.im};
}

// Two adjacent complex values (a component pair of the field layout) in one
// access: a 16-byte load or store in FP32, two in FP64.
__device__ __forceinline__ void ld_pair(const float2* p, Cx<float>& a, Cx<float>& b) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  a = {v.x, v.y};
  b = {v.z, v.w};
}
__device__ __forceinline__ void ld_pair(const double2* p, Cx<double>& a, Cx<double>& b) {
  a = ld(p);
  b = ld(p + 1);
}
__device__ __forceinline__ void st_pair(float2* p, Cx<float> a, Cx<float> b) {
  *reinterpret_cast<float4*>(p) = make_float4(a.re, a.im, b.re, b.im);
}
__device__ __forceinline__ void st_pair(double2* p, Cx<double> a, Cx<double> b) {
  st(p, a);
  st(p + 1, b);
}
__device__ __forceinline__ void st_pair_nt(float2* p, Cx<float> a, Cx<float> b) {
  typedef float v4 __attribute__((ext_vector_type(4)));
  v4 v = {a.re, a.im, b.re, b.im};
  __builtin_nontemporal_store(v, reinterpret_cast<v4*>(p));
}
__device__ __forceinline__ void st_pair_nt(double2* p, Cx<double> a, Cx<double> b) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  v2 va = {a.re, a.im}, vb = {b.re, b.im};
  __builtin_nontemporal_store(va, reinterpret_cast<v2*>(p));
  __builtin_nontemporal_store(vb, reinterpret_cast<v2*>(p + 1));
}

// A pair of stored values as FP64, and a pair stored in storage precision
// (streaming), for the elementwise kernels.
__device__ __forceinline__ void ld_pair64(const float2* p, Cx<double>& a, Cx<double>& b) {
  Cx<float> x, y;
  ld_pair(p, x, y);
  a = {(double)x.re, (double)x.im};
  b = {(double)y.re, (double)y.im};
}
__device__ __forceinline__ void ld_pair64(const double2* p, Cx<double>& a, Cx<double>& b) {
  ld_pair(p, a, b);
}
__device__ __forceinline__ void st_pair64(float2* p, Cx<double> a, Cx<double> b) {
  st_pair(p, Cx<float>{(float)a.re, (float)a.im}, Cx<float>{(float)b.re, (float)b.im});
}
__device__ __forceinline__ void st_pair64(double2* p, Cx<double> a, Cx<double> b) {
  st_pair(p, a, b);
}
__device__ __forceinline__ void st_pair64_nt(float2* p, Cx<double> a, Cx<double> b) {
  st_pair_nt(p, Cx<float>{(float)a.re, (float)a.im}, Cx<float>{(float)b.re, (float)b.im});
}
__device__ __forceinline__ void st_pair64_nt(double2* p, Cx<double> a, Cx<double> b) {
  st_pair_nt(p, a, b);
}

__device__ __forceinline__ Cx<double> c64(double2 v) { return {v.x, v.y}; }
__device__ __forceinline__ double2 d2(Cx<double> a) { return make_double2(a.re, a.im); }
__device__ __forceinline__ Cx<double> cdiv(Cx<double> a, Cx<double> b) {
  // Smith's algorithm for a / b
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re, den = b.re + b.im * r;
    return {(a.re + a.im * r) / den, (a.im - a.re * r) / den};
  } else {
    double r = b.re / b.im, den = b.re * r + b.im;
    return {(a.re * r + a.im) / den, (a.im * r - a.re) / den};
  }
}
__device__ __forceinline__ double cabs1(Cx<double> a) { return hypot(a.re, a.im); }

// ---- XCD-aware workgroup -> (site tile, source block) map -----------------
// Workgroups are handed to the 8 XCDs round robin (bid % 8).  The map gives
// each XCD a contiguous range of tiles so that neighbour sites read by a tile
// were loaded into the same XCD's L2 by nearby tiles.  On "planar" lattices
// (the tile size divides Lx*Ly) the XCD ranges are chunks of time slices and
// the tiles inside a chunk are ordered plane-tile, then t, then z, so the
// x/y/z/t neighbours of a tile are at most (tiles per plane)*(t per chunk)
// tiles away.  The source blocks of one tile are adjacent, so its links are
// reused from L2 across blocks.
struct TileMap {
  int ntiles;      // site tiles of `wg` sites
  int nrb;         // source blocks
  int per_xcd;     // workgroups per XCD (grid = 8 * per_xcd)
  int planar;      // tile size divides Lx*Ly
  int ppt;         // tiles per xy plane (planar)
  int tchunk;      // time slices per XCD chunk (planar)
  int wg;          // sites per tile
  int plane;       // Lx*Ly
  int lz;
  int rb_slow;     // source block is the slowest index
  int group;       // > 0: each XCD sweeps its time chunk once per window of
                   // `group` source blocks (adjacent within the window)
  int tiles_xcd;   // tiles of one XCD's time chunk (group > 0)
};

// Tile map of a launch with nrb source blocks and wg-site tiles (stencil.hip).
// order 0: source blocks of a tile adjacent; 1: source block slowest; 2 to 7:
// per XCD time chunk, windows of 1, 2, 3, 4, 6 or all source blocks (planar
// lattices with Lt a multiple of 8; otherwise as order 0).
TileMap make_tile_map(const Geometry& g, int wg, int nrb, int order);

__device__ __forceinline__ bool map_tile(int bid, const TileMap& m, int& site0, int& rb, int& tile) {
  int tq;
  if (m.group > 0) {
    // XCD x owns time chunk x; it sweeps the chunk's tiles (plane tile, t, z)
    // once per window of `group` source blocks, so the sites, links and z / t
    // neighbours a window touches stay within that XCD's L2
    const int local = bid >> 3;
    const int span = m.tiles_xcd * m.group;
    const int grp = local / span, rem = local - grp * span;
    const int tl = rem / m.group;
    rb = grp * m.group + (rem - tl * m.group);
    if (rb >= m.nrb) return false;
    tq = (bid & 7) * m.tiles_xcd + tl;
  } else {
    const int q = (bid & 7) * m.per_xcd + (bid >> 3);
    if (q >= m.ntiles * m.nrb) return false;
    rb = m.rb_slow ? q / m.ntiles : q % m.nrb;
    tq = m.rb_slow ? q % m.ntiles : q / m.nrb;
  }
  tile = tq;
  if (m.planar) {
    const int p = tq % m.ppt;
    int r = tq / m.ppt;
    const int tin = r % m.tchunk;
    r /= m.tchunk;
    const int z = r % m.lz;
    const int tc = r / m.lz;
    site0 = p * m.wg + m.plane * (z + m.lz * (tc * m.tchunk + tin));
  } else {
    site0 = tq * m.wg;
  }
  return true;
}

// ---- deterministic reductions over one workgroup ------------------------
// Wave64 tree by shuffles, then a fixed-order pass over the waves in LDS.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sums `n` values per thread over the workgroup; result valid in thread 0.
// lds must hold blockDim.x/64 * n doubles.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) lds[wave * NV + j] = v[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      double a = lds[j];
      for (int w = 1; w < nw; ++w) a += lds[w * NV + j];
      v[j] = a;
    }
  }
  __syncthreads();
}

}  // namespace ovs
