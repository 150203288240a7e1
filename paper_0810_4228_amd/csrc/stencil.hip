// Wilson-Dirac stencil at chemical potential on gfx950 (Section 1):
//   (Dw psi)(y) = psi(y) - sum_nu [ k eta+_nu (1 + g_nu) U_nu(y-nu) psi(y-nu)
//                                  + k eta-_nu (1 - g_nu) U_nu(y)^dag psi(y+nu) ]
// with eta+-_4 = e^{+-mu}, 1 in space.  A = gamma5 Dw(mu); A^dagger = gamma5 Dw(-mu).
//
// One thread owns one site for a block of B sources: each link is loaded once
// per hop and reused for the B sources.  (1 +- g_nu) has rank two, so the
// neighbour spinor is first projected to two spin components, multiplied by
// the link and then expanded again (chiral basis of the library header).
// Loads and stores are coalesced: the field layout is [src][12][V].
#include <atomic>
#include <mutex>
#include <type_traits>

#include "ovs_common.h"
#include "ovs_device.h"
#include "ovs_dual.h"
#include "ovs_spin.h"

namespace ovs {

// ---- canonical <-> internal layout ----------------------------------------

template <typename T2>
__global__ void k_pack(const double2* __restrict__ canon, T2* __restrict__ field, int nrhs, int V,
                       int Vs) {
  const long n = (long)nrhs * 12 * Vs;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    // e indexes the padded output (layout of fidx) so the store is coalesced;
    // pad entries are zero
    const long r = e / (12L * Vs);
    const long loc = e - r * 12L * Vs;
    const long t = loc >> 1;
    const int s = (int)(t % Vs);
    const int c = (int)(2 * (t / Vs) + (loc & 1));
    st64(field + e, s < V ? c64(canon[(r * V + s) * 12 + c]) : Cx<double>{0.0, 0.0});
  }
}

template <typename T2>
__global__ void k_unpack(const T2* __restrict__ field, double2* __restrict__ canon, int nrhs, int V,
                         int Vs) {
  const long n = (long)nrhs * 12 * V;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    // e indexes the output [r][s][c]
    const int c = (int)(e % 12);
    const long rs = e / 12;
    const int s = (int)(rs % V);
    const long r = rs / V;
    canon[e] = d2(ld64(field + r * 12 * Vs + fidx(c, s, Vs)));
  }
}

static int grid_for(long n) {
  long b = (n + kWG - 1) / kWG;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (int)b;
}

void launch_pack_f64(const double2* canon, double2* field, int nrhs, const Geometry& g, hipStream_t s) {
  long n = (long)nrhs * 12 * g.Vs;
  hipLaunchKernelGGL(k_pack<double2>, dim3(grid_for(n)), dim3(kWG), 0, s, canon, field, nrhs, g.V, g.Vs);
}
void launch_pack_f32(const double2* canon, float2* field, int nrhs, const Geometry& g, hipStream_t s) {
  long n = (long)nrhs * 12 * g.Vs;
  hipLaunchKernelGGL(k_pack<float2>, dim3(grid_for(n)), dim3(kWG), 0, s, canon, field, nrhs, g.V, g.Vs);
}
void launch_unpack_f64(const double2* field, double2* canon, int nrhs, const Geometry& g, hipStream_t s) {
  long n = (long)nrhs * 12 * g.V;
  hipLaunchKernelGGL(k_unpack<double2>, dim3(grid_for(n)), dim3(kWG), 0, s, field, canon, nrhs, g.V, g.Vs);
}
void launch_unpack_f32(const float2* field, double2* canon, int nrhs, const Geometry& g, hipStream_t s) {
  long n = (long)nrhs * 12 * g.V;
  hipLaunchKernelGGL(k_unpack<float2>, dim3(grid_for(n)), dim3(kWG), 0, s, field, canon, nrhs, g.V, g.Vs);
}

// nplanes component planes (an even number) = nplanes/2 planes of pairs; the
// pad entries of a pair plane are the contiguous range [2V, 2Vs).
template <typename T2>
__global__ void k_zero_pad(T2* __restrict__ base, long nplanes, int V, int Vs) {
  const long w = 2L * (Vs - V);
  const long n = (nplanes / 2) * w;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    st64(base + (e / w) * 2L * Vs + 2L * V + (e % w), Cx<double>{0.0, 0.0});
}

void launch_zero_pad(void* base, bool f32, long nplanes, const Geometry& g, hipStream_t s) {
  const long n = (nplanes / 2) * 2L * (g.Vs - g.V);
  if (n <= 0) return;
  if (f32)
    hipLaunchKernelGGL(k_zero_pad<float2>, dim3(grid_for(n)), dim3(kWG), 0, s, (float2*)base, nplanes, g.V, g.Vs);
  else
    hipLaunchKernelGGL(k_zero_pad<double2>, dim3(grid_for(n)), dim3(kWG), 0, s, (double2*)base, nplanes, g.V, g.Vs);
}

// Links: canonical [V][4][3][3] -> the packed layout of lidx, with the
// boundary sign folded in; pad sites and the unused slot are zero.
template <typename T2>
__global__ void k_pack_links(const double2* __restrict__ canon, T2* __restrict__ links, Geometry g,
                             int bc0, int bc1, int bc2, int bc3) {
  const long n = 4L * kLinkSlots * g.Vs;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const long t = e >> 1;
    const int s = (int)(t % g.Vs);
    const int np = (int)(t / g.Vs);
    const int nu = np / 5, ent = 2 * (np % 5) + (int)(e & 1);
    if (s >= g.V || ent >= 9) {
      st64(links + e, Cx<double>{0.0, 0.0});
      continue;
    }
    int coord;
    int ext;
    int bc;
    if (nu == 0) { coord = s % g.lx; ext = g.lx; bc = bc0; }
    else if (nu == 1) { coord = (s / g.lx) % g.ly; ext = g.ly; bc = bc1; }
    else if (nu == 2) { coord = (s / (g.lx * g.ly)) % g.lz; ext = g.lz; bc = bc2; }
    else { coord = s / (g.lx * g.ly * g.lz); ext = g.lt; bc = bc3; }
    Cx<double> u = c64(canon[((long)s * 4 + nu) * 9 + ent]);
    if (coord == ext - 1 && bc < 0) u = -u;
    st64(links + e, u);
  }
}

void launch_pack_links(const double2* canon, void* links, bool f32, const Geometry& g,
                       const int bc[4], hipStream_t s) {
  long n = 4L * kLinkSlots * g.Vs;
  if (f32)
    hipLaunchKernelGGL(k_pack_links<float2>, dim3(grid_for(n)), dim3(kWG), 0, s, canon,
                       (float2*)links, g, bc[0], bc[1], bc[2], bc[3]);
  else
    hipLaunchKernelGGL(k_pack_links<double2>, dim3(grid_for(n)), dim3(kWG), 0, s, canon,
                       (double2*)links, g, bc[0], bc[1], bc[2], bc[3]);
}

// Accumulate all eight hops of one direction pair for B sources.  UNI: `in`
// is workgroup-uniform (buffer loads); otherwise per-lane global loads.
template <typename R, typename T2, int NU, int B, bool UNI>
__device__ __forceinline__ void dir_hops(Cx<R> (&acc)[B][12], const T2* __restrict__ links,
                                         const T2* __restrict__ in, int V, int s, const Nbr& nb,
                                         int nsrc, bool g5in, R cf, R cb) {
  Cx<R> u[9];
  Cx<R> psi[12];
  // forward hop: field from s - nu through U_nu(s - nu)
  if constexpr (UNI) load_link_u(links, V, NU, nb.b[NU], u);
  else load_link(links, V, NU, nb.b[NU], u);
#pragma unroll
  for (int r = 0; r < B; ++r) {
    if (r < nsrc) {
      if constexpr (UNI) load_spinor_u(in + (long)r * 12 * V, V, nb.b[NU], g5in, psi);
      else load_spinor(in + (long)r * 12 * V, V, nb.b[NU], g5in, psi);
      hop<R, NU, +1, false>(acc[r], u, psi, cf);
    }
  }
  // backward hop: field from s + nu through U_nu(s)^dagger
  if constexpr (UNI) load_link_u(links, V, NU, s, u);
  else load_link(links, V, NU, s, u);
#pragma unroll
  for (int r = 0; r < B; ++r) {
    if (r < nsrc) {
      if constexpr (UNI) load_spinor_u(in + (long)r * 12 * V, V, nb.f[NU], g5in, psi);
      else load_spinor(in + (long)r * 12 * V, V, nb.f[NU], g5in, psi);
      hop<R, NU, -1, true>(acc[r], u, psi, cb);
    }
  }
}

// Staged form of the hops of one direction: neighbours inside the workgroup's
// tile come from the LDS copy `plane` ([source][component][tile site]).
template <typename R, typename T2, int NU, int B>
__device__ __forceinline__ void dir_hops_staged(Cx<R> (&acc)[B][12], const T2* __restrict__ links,
                                                const T2* __restrict__ in, const T2* plane,
                                                int site0, int wg, int V, int s, const Nbr& nb,
                                                int nsrc, bool g5in, R cf, R cb) {
  Cx<R> u[9];
  Cx<R> psi[12];
  auto nb_spinor = [&](int r, int n) {
    const unsigned d = (unsigned)(n - site0);
    if (d < (unsigned)wg) {
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const T2 v = plane[(r * 12 + c) * 256 + d];
        psi[c] = (g5in && c >= 6) ? Cx<R>{-v.x, -v.y} : Cx<R>{v.x, v.y};
      }
    } else {
      load_spinor_u(in + (long)r * 12 * V, V, n, g5in, psi);
    }
  };
  load_link_u(links, V, NU, nb.b[NU], u);
#pragma unroll
  for (int r = 0; r < B; ++r) {
    if (r < nsrc) {
      nb_spinor(r, nb.b[NU]);
      hop<R, NU, +1, false>(acc[r], u, psi, cf);
    }
  }
  load_link_u(links, V, NU, s, u);
#pragma unroll
  for (int r = 0; r < B; ++r) {
    if (r < nsrc) {
      nb_spinor(r, nb.f[NU]);
      hop<R, NU, -1, true>(acc[r], u, psi, cb);
    }
  }
}

// STAGE: the tile's own input spinors (wg consecutive sites) are first copied
// to LDS with one coalesced load per component, and neighbours inside the
// tile are read from there; on lattices with Lx Ly = wg = 256 a tile is an
// xy-plane and only the z and t hops go to L2/HBM.
template <typename R, int B, bool STAGE>
__global__ void __launch_bounds__(256)
k_wilson(const typename Vec2<R>::T* __restrict__ links, const typename Vec2<R>::T* __restrict__ in,
         typename Vec2<R>::T* __restrict__ out, Geometry g, HopR<R> hop_c, int nrhs, int g5in,
         int g5out, int nt, TileMap tm) {
  using T2 = typename Vec2<R>::T;
  __shared__ T2 plane[STAGE ? B * 12 * 256 : 1];
  int site0, rb, tile;
  if (!map_tile(blockIdx.x, tm, site0, rb, tile)) return;  // uniform over the workgroup
  const int s = site0 + threadIdx.x;
  const int r0 = rb * B;
  const int nsrc = min(B, nrhs - r0);
  const int Vs = g.Vs;
  const T2* inb = in + (long)r0 * 12 * Vs;
  T2* outb = out + (long)r0 * 12 * Vs;
  if constexpr (STAGE) {
    if (s < g.V) {
#pragma unroll
      for (int r = 0; r < B; ++r) {
        if (r < nsrc) {
#pragma unroll
          for (int q = 0; q < 6; ++q) {  // component pairs: one 16-byte load each in FP32
            Cx<R> x0, x1;
            ld_pair(pair_at(inb + (long)r * 12 * Vs + (long)q * 2 * Vs, s), x0, x1);
            plane[(r * 12 + 2 * q) * 256 + threadIdx.x] = T2{x0.re, x0.im};
            plane[(r * 12 + 2 * q + 1) * 256 + threadIdx.x] = T2{x1.re, x1.im};
          }
        }
      }
    }
    __syncthreads();
  }
  if (s >= g.V) return;
  const Nbr nb = neighbours(s, g);
  Cx<R> acc[B][12];
#pragma unroll
  for (int r = 0; r < B; ++r)
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[r][c] = {R(0), R(0)};
  if constexpr (STAGE) {
    const int wg = blockDim.x;
    dir_hops_staged<R, T2, 0, B>(acc, links, inb, plane, site0, wg, Vs, s, nb, nsrc, g5in, hop_c.fwd[0], hop_c.bwd[0]);
    dir_hops_staged<R, T2, 1, B>(acc, links, inb, plane, site0, wg, Vs, s, nb, nsrc, g5in, hop_c.fwd[1], hop_c.bwd[1]);
    dir_hops_staged<R, T2, 2, B>(acc, links, inb, plane, site0, wg, Vs, s, nb, nsrc, g5in, hop_c.fwd[2], hop_c.bwd[2]);
    dir_hops_staged<R, T2, 3, B>(acc, links, inb, plane, site0, wg, Vs, s, nb, nsrc, g5in, hop_c.fwd[3], hop_c.bwd[3]);
  } else {
    dir_hops<R, T2, 0, B, true>(acc, links, inb, Vs, s, nb, nsrc, g5in, hop_c.fwd[0], hop_c.bwd[0]);
    dir_hops<R, T2, 1, B, true>(acc, links, inb, Vs, s, nb, nsrc, g5in, hop_c.fwd[1], hop_c.bwd[1]);
    dir_hops<R, T2, 2, B, true>(acc, links, inb, Vs, s, nb, nsrc, g5in, hop_c.fwd[2], hop_c.bwd[2]);
    dir_hops<R, T2, 3, B, true>(acc, links, inb, Vs, s, nb, nsrc, g5in, hop_c.fwd[3], hop_c.bwd[3]);
  }
#pragma unroll
  for (int r = 0; r < B; ++r) {
    if (r < nsrc) {
      Cx<R> psi[12];
      if constexpr (STAGE) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          const T2 v = plane[(r * 12 + c) * 256 + threadIdx.x];
          psi[c] = (g5in && c >= 6) ? Cx<R>{-v.x, -v.y} : Cx<R>{v.x, v.y};
        }
      } else {
        load_spinor_u(inb + (long)r * 12 * Vs, Vs, s, g5in, psi);
      }
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        psi[c] = psi[c] - acc[r][c];
        if (g5out && c >= 6) psi[c] = -psi[c];
      }
      store_spinor(outb + (long)r * 12 * Vs, Vs, s, nt, psi);
    }
  }
}

// Variant with G lanes per site: lane j of a site group takes source rb*G + j,
// so one wave load of a link serves G sources without holding G
// accumulators per thread.  Workgroup tiles hold blockDim/G sites.
template <typename R, int G>
__global__ void __launch_bounds__(256)
k_wilson_g(const typename Vec2<R>::T* __restrict__ links, const typename Vec2<R>::T* __restrict__ in,
           typename Vec2<R>::T* __restrict__ out, Geometry g, HopR<R> hop_c, int nrhs, int g5in,
           int g5out, int nt, TileMap tm) {
  using T2 = typename Vec2<R>::T;
  int site0, rb, tile;
  if (!map_tile(blockIdx.x, tm, site0, rb, tile)) return;
  const int s = site0 + (int)threadIdx.x / G;
  const int r = rb * G + (int)threadIdx.x % G;
  if (s >= g.V || r >= nrhs) return;
  const int Vs = g.Vs;
  const T2* inr = in + (long)r * 12 * Vs;
  T2* outr = out + (long)r * 12 * Vs;
  const Nbr nb = neighbours(s, g);
  Cx<R> acc[1][12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[0][c] = {R(0), R(0)};
  // a source count the optimiser cannot see: with a literal 1 the per-source
  // guards fold away and every load of the site is hoisted (spills)
  int one = 1;
  __asm__ volatile("" : "+s"(one));
  dir_hops<R, T2, 0, 1, false>(acc, links, inr, Vs, s, nb, one, g5in, hop_c.fwd[0], hop_c.bwd[0]);
  dir_hops<R, T2, 1, 1, false>(acc, links, inr, Vs, s, nb, one, g5in, hop_c.fwd[1], hop_c.bwd[1]);
  dir_hops<R, T2, 2, 1, false>(acc, links, inr, Vs, s, nb, one, g5in, hop_c.fwd[2], hop_c.bwd[2]);
  dir_hops<R, T2, 3, 1, false>(acc, links, inr, Vs, s, nb, one, g5in, hop_c.fwd[3], hop_c.bwd[3]);
  Cx<R> psi[12];
  load_spinor(inr, Vs, s, g5in, psi);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    psi[c] = psi[c] - acc[0][c];
    if (g5out && c >= 6) psi[c] = -psi[c];
  }
  store_spinor(outr, Vs, s, nt, psi);
}

// Dynamic LDS requests above the default per-workgroup limit need a
// per-kernel opt-in; the limit is set once per process from the device query.
static std::atomic<int> g_lds_limit_kb{64};
void set_lds_limit(int kb) { g_lds_limit_kb = kb; }
// A launch whose static plus dynamic LDS exceeds the per-workgroup limit is an
// invalid dispatch (the queue aborts): launchers check before launching.
static bool lds_fits(const void* fn, int dyn_kb) {
  hipFuncAttributes at;
  if (hipFuncGetAttributes(&at, fn) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return (long)at.sharedSizeBytes + (long)dyn_kb * 1024 <= (long)g_lds_limit_kb * 1024;
}
static void apply_lds_limit(const void* fn) {
  if (g_lds_limit_kb > 64) {
    // a rejected request only means larger LDS caps fail at launch (and are
    // skipped by the autotuner); it must not leave a sticky error behind
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (g_lds_limit_kb - 1) * 1024) != hipSuccess)
      (void)hipGetLastError();
  }
}

TileMap make_tile_map(const Geometry& g, int wg, int nrb, int order) {
  TileMap m;
  m.wg = wg;
  m.nrb = nrb;
  m.plane = g.lx * g.ly;
  m.lz = g.lz;
  m.planar = (m.plane % wg == 0) ? 1 : 0;
  m.ntiles = (g.V + wg - 1) / wg;
  m.ppt = m.planar ? m.plane / wg : 1;
  m.tchunk = (m.planar && g.lt % 8 == 0) ? g.lt / 8 : g.lt;
  m.group = 0;
  m.tiles_xcd = 0;
  if (order >= 2 && m.planar && g.lt % 8 == 0) {
    // windows of 1, 2, 3, 4, 6 or all source blocks over each XCD's time chunk
    static const int kWindow[6] = {1, 2, 3, 4, 6, 1 << 30};
    m.rb_slow = 0;
    m.group = kWindow[order - 2] < nrb ? kWindow[order - 2] : nrb;
    m.tiles_xcd = m.ntiles / 8;
    const int ngroups = (nrb + m.group - 1) / m.group;
    m.per_xcd = ngroups * m.tiles_xcd * m.group;
    return m;
  }
  m.rb_slow = order == 1 ? 1 : 0;
  const long nb = (long)m.ntiles * nrb;
  m.per_xcd = (int)((nb + 7) / 8);
  return m;
}

template <typename R, int B>
static hipError_t launch_w(const void* links, const void* in, void* out, int nrhs, const Geometry& g,
                     const Hop& hop_c, bool g5in, bool g5out, int wg, int lds_kb, int order,
                     int nt, bool stage, hipStream_t s) {
  using T2 = typename Vec2<R>::T;
  // the staged tile takes B 12 256 values of LDS
  constexpr bool kStage = B * 12 * 256 * sizeof(T2) <= 100 * 1024;
  const TileMap tm = make_tile_map(g, wg, (nrhs + B - 1) / B, order);
  static std::once_flag lds_set;  // launches may come from several host threads
  std::call_once(lds_set, [] {
    apply_lds_limit((const void*)k_wilson<R, B, false>);
    if constexpr (kStage) apply_lds_limit((const void*)k_wilson<R, B, true>);
  });
  if constexpr (!kStage) {
    if (stage) return hipErrorInvalidValue;
  }
  const void* fn = stage ? (const void*)k_wilson<R, B, kStage> : (const void*)k_wilson<R, B, false>;
  if (!lds_fits(fn, lds_kb)) return hipErrorInvalidValue;
#define OVS_W(ST)                                                                             \
  hipLaunchKernelGGL((k_wilson<R, B, ST>), dim3(8 * tm.per_xcd), dim3(wg), lds_kb * 1024, s,  \
                     (const T2*)links, (const T2*)in, (T2*)out, g, HopR<R>::make(hop_c), nrhs, \
                     (int)g5in, (int)g5out, nt, tm)
  if (stage) OVS_W(kStage);
  else OVS_W(false);
#undef OVS_W
  return hipSuccess;
}

template <typename R, int G>
static hipError_t launch_wg(const void* links, const void* in, void* out, int nrhs, const Geometry& g,
                      const Hop& hop_c, bool g5in, bool g5out, int wg, int lds_kb, int order, int nt,
                      hipStream_t s) {
  using T2 = typename Vec2<R>::T;
  const TileMap tm = make_tile_map(g, wg / G, (nrhs + G - 1) / G, order);
  static std::once_flag lds_set;
  std::call_once(lds_set, [] { apply_lds_limit((const void*)k_wilson_g<R, G>); });
  if (!lds_fits((const void*)k_wilson_g<R, G>, lds_kb)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_wilson_g<R, G>), dim3(8 * tm.per_xcd), dim3(wg), lds_kb * 1024, s,
                     (const T2*)links, (const T2*)in, (T2*)out, g, HopR<R>::make(hop_c), nrhs,
                     (int)g5in, (int)g5out, nt, tm);
  return hipSuccess;
}

hipError_t launch_wilson(bool f32, const void* links, const void* in, void* out, int nrhs,
                         const Geometry& g, const Hop& hop_c, bool g5in, bool g5out,
                         const Tuning& tn, hipStream_t s) {
  const int wg = tn.wg;
  hipError_t e = hipSuccess;
  if (tn.g > 1) {
#define OVS_WG(RT, GG) e = launch_wg<RT, GG>(links, in, out, nrhs, g, hop_c, g5in, g5out, wg, tn.lds_kb, tn.order, tn.nt, s)
    if (f32) {
      switch (tn.g) {
        case 2: OVS_WG(float, 2); break;
        case 4: OVS_WG(float, 4); break;
        case 8: OVS_WG(float, 8); break;
        default: return hipErrorInvalidValue;
      }
    } else {
      switch (tn.g) {
        case 2: OVS_WG(double, 2); break;
        case 4: OVS_WG(double, 4); break;
        case 8: OVS_WG(double, 8); break;
        default: return hipErrorInvalidValue;
      }
    }
#undef OVS_WG
    if (e != hipSuccess) return e;
    return hipGetLastError();
  }
  if (f32) {
    switch (tn.rhs_block) {
      case 1: e = launch_w<float, 1>(links, in, out, nrhs, g, hop_c, g5in, g5out, wg, tn.lds_kb, tn.order, tn.nt, tn.stage != 0, s); break;
      case 2: e = launch_w<float, 2>(links, in, out, nrhs, g, hop_c, g5in, g5out, wg, tn.lds_kb, tn.order, tn.nt, tn.stage != 0, s); break;
      case 3: e = launch_w<float, 3>(links, in, out, nrhs, g, hop_c, g5in, g5out, wg, tn.lds_kb, tn.order, tn.nt, tn.stage != 0, s); break;
      case 4: e = launch_w<float, 4>(links, in, out, nrhs, g, hop_c, g5in, g5out, wg, tn.lds_kb, tn.order, tn.nt, tn.stage != 0, s); break;
      case 6: e = launch_w<float, 6>(links, in, out, nrhs, g, hop_c, g5in, g5out, wg, tn.lds_kb, tn.order, tn.nt, tn.stage != 0, s); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (tn.rhs_block) {
      case 1: e = launch_w<double, 1>(links, in, out, nrhs, g, hop_c, g5in, g5out, wg, tn.lds_kb, tn.order, tn.nt, tn.stage != 0, s); break;
      case 2: e = launch_w<double, 2>(links, in, out, nrhs, g, hop_c, g5in, g5out, wg, tn.lds_kb, tn.order, tn.nt, tn.stage != 0, s); break;
      case 3: e = launch_w<double, 3>(links, in, out, nrhs, g, hop_c, g5in, g5out, wg, tn.lds_kb, tn.order, tn.nt, tn.stage != 0, s); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

// ---- dual stencil for the two-sided Lanczos step ---------------------------
// For each active source slot r: T_r = A V~_r, S_r = A^dag W~_r, and per
// workgroup the partial sums of W~_r^dagger T_r (complex) and |T_r|^2, in FP64.

template <typename R, int B>
__global__ void __launch_bounds__(256)
k_dual(const typename Vec2<R>::T* __restrict__ links, const typename Vec2<R>::T* __restrict__ basis,
       const typename Vec2<R>::T* __restrict__ wbuf, long basis_stride, int ring,
       const int* __restrict__ it, typename Vec2<R>::T* __restrict__ out_t,
       typename Vec2<R>::T* __restrict__ out_s, double* __restrict__ partials, Geometry g,
       HopR<R> hA, HopR<R> hAd, const int* __restrict__ rhs_map, const int* __restrict__ n_active,
       int nt, TileMap tm) {
  using T2 = typename Vec2<R>::T;
  __shared__ double lds[(256 / 64) * 3 * B];
  int site0, rb, tile;
  if (!map_tile(blockIdx.x, tm, site0, rb, tile)) return;  // uniform over the workgroup
  const int na = *n_active;
  const int iter = *it;
  const T2* in_v = basis + (long)(ring ? iter % 3 : iter) * basis_stride;
  const T2* in_w = wbuf + (long)(iter % 3) * basis_stride;
  const int j0 = rb * B;
  if (j0 >= na) return;  // uniform over the workgroup
  // opaque to the optimiser, as in k_dual_pair: keeps the per-source guards
  int nsrc = min(B, na - j0);
  __asm__ volatile("" : "+s"(nsrc));
  const int s = site0 + threadIdx.x;
  const bool live = s < g.V;
  const int V = g.Vs;  // stride of the padded component planes
  int slot[B];
#pragma unroll
  for (int r = 0; r < B; ++r) slot[r] = (r < nsrc) ? rhs_map[j0 + r] : 0;

  double part[3 * B];
#pragma unroll
  for (int q = 0; q < 3 * B; ++q) part[q] = 0.0;

  if (live) {
    const Nbr nb = neighbours(s, g);
    Cx<R> accv[B][12], accw[B][12];
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < 12; ++c) accv[r][c] = accw[r][c] = {R(0), R(0)};
    Cx<R> u[9], psi[12];
#define OVS_DUAL_DIR(NU)                                                                 \
  load_link_u(links, V, NU, nb.b[NU], u);                                                  \
  _Pragma("unroll") for (int r = 0; r < B; ++r) {                                        \
    if (r < nsrc) {                                                                      \
      load_spinor_u(in_v + (long)slot[r] * 12 * V, V, nb.b[NU], false, psi);               \
      hop<R, NU, +1, false>(accv[r], u, psi, hA.fwd[NU]);                                \
      load_spinor_u(in_w + (long)slot[r] * 12 * V, V, nb.b[NU], false, psi);               \
      hop<R, NU, +1, false>(accw[r], u, psi, hAd.fwd[NU]);                               \
    }                                                                                    \
  }                                                                                      \
  load_link_u(links, V, NU, s, u);                                                         \
  _Pragma("unroll") for (int r = 0; r < B; ++r) {                                        \
    if (r < nsrc) {                                                                      \
      load_spinor_u(in_v + (long)slot[r] * 12 * V, V, nb.f[NU], false, psi);               \
      hop<R, NU, -1, true>(accv[r], u, psi, hA.bwd[NU]);                                 \
      load_spinor_u(in_w + (long)slot[r] * 12 * V, V, nb.f[NU], false, psi);               \
      hop<R, NU, -1, true>(accw[r], u, psi, hAd.bwd[NU]);                                \
    }                                                                                    \
  }
    OVS_DUAL_DIR(0)
    OVS_DUAL_DIR(1)
    OVS_DUAL_DIR(2)
    OVS_DUAL_DIR(3)
#undef OVS_DUAL_DIR
#pragma unroll
    for (int r = 0; r < B; ++r) {
      if (r < nsrc) {
        const long base = (long)slot[r] * 12 * V;
        Cx<R> pv[12], pw[12];
        load_spinor_u(in_v + base, V, s, false, pv);
        load_spinor_u(in_w + base, V, s, false, pw);
        Cx<R> t[12], sv[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          t[c] = pv[c] - accv[r][c];
          sv[c] = pw[c] - accw[r][c];
          if (c >= 6) { t[c] = -t[c]; sv[c] = -sv[c]; }
        }
        store_spinor(out_t + base, V, s, nt, t);
        store_spinor(out_s + base, V, s, nt, sv);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          const Cx<double> t64 = {(double)t[c].re, (double)t[c].im};
          const Cx<double> w64 = {(double)pw[c].re, (double)pw[c].im};
          const Cx<double> p = cmulc(w64, t64);
          part[3 * r + 0] += p.re;
          part[3 * r + 1] += p.im;
          part[3 * r + 2] += cnorm2(t64);
        }
      }
    }
  }
  block_sum<3 * B>(part, lds);
  if (threadIdx.x == 0) {
    // compile-time bound: part[] stays in registers (a runtime bound makes it
    // an indexed array that the compiler may place in LDS or scratch)
#pragma unroll
    for (int r = 0; r < B; ++r) {
      if (r < nsrc) {
        double* p = partials + ((long)slot[r] * tm.ntiles + tile) * 3;
        p[0] = part[3 * r + 0];
        p[1] = part[3 * r + 1];
        p[2] = part[3 * r + 2];
      }
    }
  }
}

// Operator-pair variant: lanes 2j and 2j+1 of a 512-thread workgroup take
// the same site, lane 2j computing T = A V~ and lane 2j+1 S = A^dag W~ for the
// source block.  Both operators are the same stencil with e^{+mu} and e^{-mu}
// swapped on the time hops, so the pair loads the same link addresses (one
// fetch serves both lanes) and each lane holds one set of accumulators: half
// the registers of k_dual, twice the waves in flight.  Tiles are the same 256
// sites, so the partial-sum layout is unchanged; the even lane also reads
// W~ at its own site for W~^dagger T.
//
// STAGE: the tile's own V~ and W~ spinors are first copied to LDS (one
// coalesced load per component), and every neighbour inside the tile is read
// from there.  A tile is 256 consecutive sites, so on lattices with
// Lx Ly = 256 it is one xy-plane and all x and y hops are served from LDS;
// only the z and t neighbours go to L2/HBM.
template <typename R, int B, bool STAGE>
__global__ void __launch_bounds__(512)
k_dual_pair(const typename Vec2<R>::T* __restrict__ links,
            const typename Vec2<R>::T* __restrict__ basis,
            const typename Vec2<R>::T* __restrict__ wbuf, long basis_stride, int ring,
            const int* __restrict__ it, typename Vec2<R>::T* __restrict__ out_t,
            typename Vec2<R>::T* __restrict__ out_s, double* __restrict__ partials, Geometry g,
            HopR<R> hA, HopR<R> hAd, const int* __restrict__ rhs_map,
            const int* __restrict__ n_active, int nt, TileMap tm) {
  using T2 = typename Vec2<R>::T;
  __shared__ double lds[(512 / 64) * 3 * B];
  __shared__ T2 plane[STAGE ? 2 * B * 12 * 256 : 1];  // [op][source][component][tile site]
  int site0, rb, tile;
  if (!map_tile(blockIdx.x, tm, site0, rb, tile)) return;  // uniform over the workgroup
  const int na = *n_active;
  const int iter = *it;
  const T2* in_v = basis + (long)(ring ? iter % 3 : iter) * basis_stride;
  const T2* in_w = wbuf + (long)(iter % 3) * basis_stride;
  const int j0 = rb * B;
  if (j0 >= na) return;  // uniform over the workgroup
  // The empty asm hides that nsrc >= 1 from the optimiser: the per-source
  // guards below stay scalar branches that bound each hop's load batch (with
  // the guards folded away the scheduler hoists every load of the site and spills).
  int nsrc = min(B, na - j0);
  __asm__ volatile("" : "+s"(nsrc));
  const int op = threadIdx.x & 1;
  const int ts = threadIdx.x >> 1;
  const int s = site0 + ts;
  const bool live = s < g.V;
  const int V = g.Vs;
  const T2* in = op ? in_w : in_v;
  T2* out = op ? out_s : out_t;
  R cf[4], cb[4];
#pragma unroll
  for (int nu = 0; nu < 4; ++nu) {
    cf[nu] = op ? hAd.fwd[nu] : hA.fwd[nu];
    cb[nu] = op ? hAd.bwd[nu] : hA.bwd[nu];
  }
  int slot[B];
#pragma unroll
  for (int r = 0; r < B; ++r) slot[r] = (r < nsrc) ? rhs_map[j0 + r] : 0;

  if constexpr (STAGE) {
#pragma unroll
    for (int r = 0; r < B; ++r) {
      if (r < nsrc && live) {
        const T2* f = in + (long)slot[r] * 12 * V;
#pragma unroll
        for (int q = 0; q < 6; ++q) {  // component pairs: one 16-byte load each in FP32
          Cx<R> x0, x1;
          ld_pair(pair_at(f + (long)q * 2 * V, s), x0, x1);
          plane[((op * B + r) * 12 + 2 * q) * 256 + ts] = T2{x0.re, x0.im};
          plane[((op * B + r) * 12 + 2 * q + 1) * 256 + ts] = T2{x1.re, x1.im};
        }
      }
    }
    __syncthreads();
  }
  // spinor of source r at site n: from the staged tile when n is inside it
  auto load_nb = [&](int r, int n, Cx<R>(&p)[12]) {
    const unsigned d = (unsigned)(n - site0);
    if (STAGE && d < 256u) {
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const T2 v = plane[((op * B + r) * 12 + c) * 256 + d];
        p[c] = {v.x, v.y};
      }
    } else {
      load_spinor(in + (long)slot[r] * 12 * V, V, n, false, p);
    }
  };

  double part[3 * B];
#pragma unroll
  for (int q = 0; q < 3 * B; ++q) part[q] = 0.0;

  if (live) {
    const Nbr nb = neighbours(s, g);
    Cx<R> acc[B][12];
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[r][c] = {R(0), R(0)};
    Cx<R> u[9], psi[12];
#define OVS_PAIR_DIR(NU)                                                                 \
  load_link(links, V, NU, nb.b[NU], u);                                                  \
  _Pragma("unroll") for (int r = 0; r < B; ++r) {                                        \
    if (r < nsrc) {                                                                      \
      load_nb(r, nb.b[NU], psi);                                                         \
      hop<R, NU, +1, false>(acc[r], u, psi, cf[NU]);                                     \
    }                                                                                    \
  }                                                                                      \
  load_link(links, V, NU, s, u);                                                         \
  _Pragma("unroll") for (int r = 0; r < B; ++r) {                                        \
    if (r < nsrc) {                                                                      \
      load_nb(r, nb.f[NU], psi);                                                         \
      hop<R, NU, -1, true>(acc[r], u, psi, cb[NU]);                                      \
    }                                                                                    \
  }
    OVS_PAIR_DIR(0)
    OVS_PAIR_DIR(1)
    OVS_PAIR_DIR(2)
    OVS_PAIR_DIR(3)
#undef OVS_PAIR_DIR
#pragma unroll
    for (int r = 0; r < B; ++r) {
      if (r < nsrc) {
        const long base = (long)slot[r] * 12 * V;
        Cx<R> p[12], pw[12];
        load_nb(r, s, p);
        if (!op) {
          if constexpr (STAGE) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
              const T2 v = plane[((B + r) * 12 + c) * 256 + ts];
              pw[c] = {v.x, v.y};
            }
          } else {
            load_spinor(in_w + base, V, s, false, pw);
          }
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          p[c] = p[c] - acc[r][c];
          if (c >= 6) p[c] = -p[c];
        }
        store_spinor(out + base, V, s, nt, p);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          const Cx<R> o = p[c];
          if (!op) {
            const Cx<double> t64 = {(double)o.re, (double)o.im};
            const Cx<double> w64 = {(double)pw[c].re, (double)pw[c].im};
            const Cx<double> q = cmulc(w64, t64);
            part[3 * r + 0] += q.re;
            part[3 * r + 1] += q.im;
            part[3 * r + 2] += cnorm2(t64);
          }
        }
      }
    }
  }
  block_sum<3 * B>(part, lds);
  if (threadIdx.x == 0) {
    // compile-time bound: part[] stays in registers (a runtime bound makes it
    // an indexed array that the compiler may place in LDS or scratch)
#pragma unroll
    for (int r = 0; r < B; ++r) {
      if (r < nsrc) {
        double* p = partials + ((long)slot[r] * tm.ntiles + tile) * 3;
        p[0] = part[3 * r + 0];
        p[1] = part[3 * r + 1];
        p[2] = part[3 * r + 2];
      }
    }
  }
}

// Operator-per-workgroup variant (body in ovs_dual.h, shared with the
// persistent Lanczos kernel).
template <typename R, int B, bool STAGE>
__global__ void __launch_bounds__(256)
k_dual_op(const typename Vec2<R>::T* __restrict__ links,
          const typename Vec2<R>::T* __restrict__ basis,
          const typename Vec2<R>::T* __restrict__ wbuf, long basis_stride, int ring,
          const int* __restrict__ it, typename Vec2<R>::T* __restrict__ out_t,
          typename Vec2<R>::T* __restrict__ out_s, double* __restrict__ partials, Geometry g,
          HopR<R> hA, HopR<R> hAd, const int* __restrict__ rhs_map,
          const int* __restrict__ n_active, int nt, TileMap tm) {
  dual_op_body<R, B, STAGE>(blockIdx.x, *it, links, basis, wbuf, basis_stride, ring, out_t, out_s,
                            partials, g, hA, hAd, rhs_map, *n_active, nt, tm);
}

// Dual stencil marching along t (variant 6): one operator and one source per
// workgroup, over one (xy tile, z) column of the XCD's chunk of time slices.
// Each thread keeps its own site's spinors at t-1, t and t+1 and the time link
// at t-1 in registers while the workgroup steps through the chunk, so the time
// hops fetch nothing twice; at every step the tile's spinors at t go from the
// registers to LDS, where the in-tile x and y neighbours are read.  The z
// neighbours (and x, y ones outside the tile) are loaded as in the other
// variants (the workgroups of neighbouring z, and of the other sources at the
// same column, run at the same time and share them in L2).  The
// arithmetic, its order and the per-tile partial sums are those of the
// operator-per-workgroup body with one source per thread, so the results agree
// bit for bit.  Needs xy planes of 256 sites (the tile) and Lt a multiple of
// 8 (the launch checks).  order 0: the sources of a column
// adjacent in dispatch order; 1: the columns of a source adjacent.
template <typename R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_dual_march(const typename Vec2<R>::T* __restrict__ links,
             const typename Vec2<R>::T* __restrict__ basis,
             const typename Vec2<R>::T* __restrict__ wbuf, long basis_stride, int ring,
             const int* __restrict__ it, typename Vec2<R>::T* __restrict__ out_t,
             typename Vec2<R>::T* __restrict__ out_s, double* __restrict__ partials, Geometry g,
             HopR<R> hA, HopR<R> hAd, const int* __restrict__ rhs_map,
             const int* __restrict__ n_active, int nslots, int nt, TileMap tm, int order) {
  using T2 = typename Vec2<R>::T;
  __shared__ double lds[(256 / 64) * 3];
  __shared__ T2 plane[12 * 256];  // the tile's spinors at the current t: [component][site]
  const int tc = blockIdx.x & 7;  // the XCD's time chunk
  int local = blockIdx.x >> 3;
  const int op = local & 1;       // the A and A^dag workgroups of a column are adjacent
  local >>= 1;
  const int ncol = tm.ppt * tm.lz;
  int col, j;
  if (order == 1) {
    j = local / ncol;
    col = local - j * ncol;
  } else {
    col = local / nslots;
    j = local - col * nslots;
  }
  if (col >= ncol || j >= *n_active) return;  // uniform over the workgroup
  const int iter = *it;
  const T2* in_v = basis + (long)(ring ? iter % 3 : iter) * basis_stride;
  const T2* in_w = wbuf + (long)(iter % 3) * basis_stride;
  const int slot = rhs_map[j];
  const int V = g.Vs;
  const long base = (long)slot * 12 * V;
  const T2* f = (op ? in_w : in_v) + base;
  T2* out = (op ? out_s : out_t) + base;
  const HopR<R>& hc = op ? hAd : hA;
  const int p = col % tm.ppt, z = col / tm.ppt;
  const int st = tm.plane * tm.lz;                         // sites per time slice
  const int s0 = p * 256 + (int)threadIdx.x + tm.plane * z;  // the thread's site at t = 0
  const int t0 = tc * tm.tchunk;
  const int tprev = t0 == 0 ? g.lt - 1 : t0 - 1;
  // opaque to the optimiser, as nsrc in the other variants: loads stay behind
  // their direction's guard instead of being hoisted all at once
  int gate = 1;
  __asm__ volatile("" : "+s"(gate));
  Cx<R> pm[12], pc[12], um[9];
  load_spinor_u(f, V, s0 + tprev * st, false, pm);
  load_spinor_u(f, V, s0 + t0 * st, false, pc);
  load_link_u(links, V, 3, s0 + tprev * st, um);
#pragma unroll 1
  for (int i = 0; i < tm.tchunk; ++i) {
    const int s = s0 + (t0 + i) * st;
    const int site0 = s - (int)threadIdx.x;  // the tile's first site at this t
    const Nbr nb = neighbours(s, g);
    // the tile's spinors at t go to LDS from the registers: in-tile x and y
    // neighbours are read there
    __syncthreads();  // the previous step's readers are done
#pragma unroll
    for (int c = 0; c < 12; ++c) plane[c * 256 + threadIdx.x] = T2{pc[c].re, pc[c].im};
    __syncthreads();
    // the xy plane is the tile (256 sites): x and y neighbours are in LDS
    auto load_lds = [&](int n, Cx<R>(&q)[12]) {
      const int d = n - site0;
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const T2 v = plane[c * 256 + d];
        q[c] = {v.x, v.y};
      }
    };
    Cx<R> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = {R(0), R(0)};
    Cx<R> u[9], psi[12];
#define OVS_MARCH_DIR(NU, LOAD)                                    \
  if (gate) {                                                      \
    load_link_u(links, V, NU, nb.b[NU], u);                        \
    LOAD(nb.b[NU], psi);                                           \
    hop<R, NU, +1, false>(acc, u, psi, hc.fwd[NU]);                \
  }                                                                \
  if (gate) {                                                      \
    load_link_u(links, V, NU, s, u);                               \
    LOAD(nb.f[NU], psi);                                           \
    hop<R, NU, -1, true>(acc, u, psi, hc.bwd[NU]);                 \
  }
#define OVS_GLOBAL(n, q) load_spinor_u(f, V, n, false, q)
    OVS_MARCH_DIR(0, load_lds)
    OVS_MARCH_DIR(1, load_lds)
    OVS_MARCH_DIR(2, OVS_GLOBAL)
#undef OVS_GLOBAL
#undef OVS_MARCH_DIR
    hop<R, 3, +1, false>(acc, um, pm, hc.fwd[3]);
    if (gate) {
      load_link_u(links, V, 3, s, um);
      load_spinor_u(f, V, nb.f[3], false, psi);
      hop<R, 3, -1, true>(acc, um, psi, hc.bwd[3]);
    }
    Cx<R> o[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      o[c] = pc[c] - acc[c];
      if (c >= 6) o[c] = -o[c];
    }
    store_spinor(out, V, s, nt, o);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      pm[c] = pc[c];
      pc[c] = psi[c];
    }
    if (!op) {  // uniform over the workgroup
      double part[3] = {0.0, 0.0, 0.0};
      Cx<R> pw[12];
      load_spinor_u(in_w + base, V, s, false, pw);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const Cx<double> t64 = {(double)o[c].re, (double)o[c].im};
        const Cx<double> w64 = {(double)pw[c].re, (double)pw[c].im};
        const Cx<double> q = cmulc(w64, t64);
        part[0] += q.re;
        part[1] += q.im;
        part[2] += cnorm2(t64);
      }
      block_sum<3>(part, lds);
      if (threadIdx.x == 0) {
        const int tile = p + tm.ppt * (i + tm.tchunk * (z + tm.lz * tc));
        double* d = partials + ((long)slot * tm.ntiles + tile) * 3;
        d[0] = part[0];
        d[1] = part[1];
        d[2] = part[2];
      }
    }
  }
}

int dual_num_wg(const Geometry& g) { return (g.V + 255) / 256; }

template <typename R, int B>
static hipError_t launch_d(const DualArgs& a, const Geometry& g, const Hop& hA, const Hop& hAd,
                     hipStream_t s) {
  using T2 = typename Vec2<R>::T;
  if (a.tile != 256 && (a.tile != 64 || a.pair != 0)) return hipErrorInvalidValue;
  const TileMap tm = make_tile_map(g, a.tile, (a.nrhs_slots + B - 1) / B, a.order);
  // the staged planes take 2 B 12 256 complex values of LDS: one or two sources
  constexpr bool kStage = 2 * B * 12 * 256 * sizeof(T2) <= 100 * 1024;
  // the operator-per-workgroup variant stages one field: B 12 256 values
  constexpr bool kStageOp = B * 12 * 256 * sizeof(T2) <= 100 * 1024;
  static std::once_flag lds_set;
  std::call_once(lds_set, [] {
    apply_lds_limit((const void*)k_dual<R, B>);
    apply_lds_limit((const void*)k_dual_pair<R, B, false>);
    if constexpr (kStage) apply_lds_limit((const void*)k_dual_pair<R, B, true>);
    apply_lds_limit((const void*)k_dual_op<R, B, false>);
    if constexpr (kStageOp) apply_lds_limit((const void*)k_dual_op<R, B, true>);
  });
  if (a.pair == 5) {
    // marching along t: FP32 storage (the FP64 ring does not fit the register
    // budget), one source per thread, xy planes of 256 sites, Lt % 8 == 0
    if constexpr (std::is_same_v<R, float> && B == 1) {
      if (g.lx * g.ly != 256 || g.lt % 8 != 0) return hipErrorInvalidValue;
      static std::once_flag march_lds;
      std::call_once(march_lds, [] { apply_lds_limit((const void*)k_dual_march<R>); });
      if (!lds_fits((const void*)k_dual_march<R>, a.lds_kb)) return hipErrorInvalidValue;
      const int per_xcd = 2 * tm.ppt * tm.lz * a.nrhs_slots;
      hipLaunchKernelGGL((k_dual_march<R>), dim3(8 * per_xcd), dim3(256), a.lds_kb * 1024, s,
                         (const T2*)a.links, (const T2*)a.basis, (const T2*)a.wbuf,
                         a.basis_stride, (int)a.ring, a.it, (T2*)a.out_t, (T2*)a.out_s,
                         a.partials, g, HopR<R>::make(hA), HopR<R>::make(hAd), a.rhs_map,
                         a.n_active, a.nrhs_slots, a.nt, tm, a.order == 1 ? 1 : 0);
      return hipSuccess;
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (a.pair == 3 || a.pair == 4) {
    const bool stage = a.pair == 4;
    if constexpr (!kStageOp) {
      if (stage) return hipErrorInvalidValue;
    }
    const void* fn = stage ? (const void*)k_dual_op<R, B, kStageOp> : (const void*)k_dual_op<R, B, false>;
    if (!lds_fits(fn, a.lds_kb)) return hipErrorInvalidValue;
#define OVS_DUAL_OP(ST)                                                                        \
  hipLaunchKernelGGL((k_dual_op<R, B, ST>), dim3(16 * tm.per_xcd), dim3(256), a.lds_kb * 1024, s, \
                     (const T2*)a.links, (const T2*)a.basis, (const T2*)a.wbuf, a.basis_stride, \
                     (int)a.ring, a.it, (T2*)a.out_t, (T2*)a.out_s, a.partials, g,             \
                     HopR<R>::make(hA), HopR<R>::make(hAd), a.rhs_map, a.n_active, a.nt, tm)
    if (stage) OVS_DUAL_OP(kStageOp);
    else OVS_DUAL_OP(false);
#undef OVS_DUAL_OP
    return hipSuccess;
  }
  if (a.pair == 2) {
    if constexpr (kStage) {
      if (!lds_fits((const void*)k_dual_pair<R, B, true>, a.lds_kb)) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_dual_pair<R, B, true>), dim3(8 * tm.per_xcd), dim3(512),
                         a.lds_kb * 1024, s, (const T2*)a.links, (const T2*)a.basis,
                         (const T2*)a.wbuf, a.basis_stride, (int)a.ring, a.it, (T2*)a.out_t,
                         (T2*)a.out_s, a.partials, g, HopR<R>::make(hA), HopR<R>::make(hAd),
                         a.rhs_map, a.n_active, a.nt, tm);
      return hipSuccess;
    } else {
      return hipErrorInvalidValue;
    }
  }
  const void* fn = a.pair == 1 ? (const void*)k_dual_pair<R, B, false> : (const void*)k_dual<R, B>;
  if (!lds_fits(fn, a.lds_kb)) return hipErrorInvalidValue;
  if (a.pair == 1)
    hipLaunchKernelGGL((k_dual_pair<R, B, false>), dim3(8 * tm.per_xcd), dim3(512),
                       a.lds_kb * 1024, s, (const T2*)a.links, (const T2*)a.basis,
                       (const T2*)a.wbuf, a.basis_stride, (int)a.ring, a.it, (T2*)a.out_t,
                       (T2*)a.out_s, a.partials, g, HopR<R>::make(hA), HopR<R>::make(hAd),
                       a.rhs_map, a.n_active, a.nt, tm);
  else
    hipLaunchKernelGGL((k_dual<R, B>), dim3(8 * tm.per_xcd), dim3(a.tile), a.lds_kb * 1024, s,
                       (const T2*)a.links, (const T2*)a.basis, (const T2*)a.wbuf, a.basis_stride,
                       (int)a.ring, a.it, (T2*)a.out_t, (T2*)a.out_s, a.partials, g,
                       HopR<R>::make(hA), HopR<R>::make(hAd), a.rhs_map, a.n_active, a.nt, tm);
  return hipSuccess;
}

hipError_t launch_dual(bool f32, const DualArgs& a, const Geometry& g, const Hop& hA,
                       const Hop& hAd, int rhs_block, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (f32) {
    switch (rhs_block) {
      case 1: e = launch_d<float, 1>(a, g, hA, hAd, s); break;
      case 2: e = launch_d<float, 2>(a, g, hA, hAd, s); break;
      case 3: e = launch_d<float, 3>(a, g, hA, hAd, s); break;
      case 4: e = launch_d<float, 4>(a, g, hA, hAd, s); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (rhs_block) {
      case 1: e = launch_d<double, 1>(a, g, hA, hAd, s); break;
      case 2: e = launch_d<double, 2>(a, g, hA, hAd, s); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace ovs
