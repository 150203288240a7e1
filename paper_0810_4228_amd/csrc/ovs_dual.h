// Dual stencil of the two-sided Lanczos step (Section 4), one operator per
// workgroup: the body shared by k_dual_op and the persistent Lanczos kernel.
#pragma once

#include "ovs_common.h"
#include "ovs_device.h"
#include "ovs_spin.h"

namespace ovs {

// Operator-per-workgroup dual stencil: the launch holds two workgroups per tile
// and source block, adjacent in dispatch order on the same XCD, one computing
// T = A V~ and the other S = A^dag W~.  Each runs the single-operator stencil
// (one thread per site, one set of accumulators per source), and the two
// fetches of every link meet in that XCD's L2.  The A workgroup also reads
// W~ at its own site for the partial sums; the A^dag workgroup writes none.
// STAGE: as in k_dual_pair, the tile's spinors of the workgroup's own field
// are copied to LDS first and in-tile neighbours read from there.
// bid: the workgroup's index in the launch (or a virtual one of the same XCD
// in a persistent grid); iter, na: the iteration index and the number of
// active sources.  Every return is uniform over the workgroup.  The LDS
// arrays are declared here (not passed in) so that their accesses keep the
// LDS address space.
template <typename R, int B, bool STAGE>
__device__ __forceinline__ void dual_op_body(
    int bid, int iter, const typename Vec2<R>::T* __restrict__ links,
    const typename Vec2<R>::T* __restrict__ basis, const typename Vec2<R>::T* __restrict__ wbuf,
    long basis_stride, int ring, typename Vec2<R>::T* __restrict__ out_t,
    typename Vec2<R>::T* __restrict__ out_s, double* __restrict__ partials, const Geometry& g,
    const HopR<R>& hA, const HopR<R>& hAd, const int* __restrict__ rhs_map, int na, int nt,
    const TileMap& tm) {
  using T2 = typename Vec2<R>::T;
  __shared__ double lds[(256 / 64) * 3 * B];
  __shared__ T2 plane[STAGE ? B * 12 * 256 : 1];  // [source][component][tile site]
  // workgroups go round robin over the 8 XCDs: consecutive workgroups of one
  // XCD alternate the operator over the same tile
  const int op = (bid >> 3) & 1;
  const int vb = (int)(((bid >> 4) << 3) | (bid & 7));
  int site0, rb, tile;
  if (!map_tile(vb, tm, site0, rb, tile)) return;
  const T2* in_v = basis + (long)(ring ? iter % 3 : iter) * basis_stride;
  const T2* in_w = wbuf + (long)(iter % 3) * basis_stride;
  const int j0 = rb * B;
  if (j0 >= na) return;  // uniform over the workgroup
  // opaque to the optimiser, as in k_dual_pair
  int nsrc = min(B, na - j0);
  __asm__ volatile("" : "+s"(nsrc));
  const int s = site0 + threadIdx.x;
  const bool live = s < g.V;
  const int V = g.Vs;
  const T2* in = op ? in_w : in_v;
  T2* out = op ? out_s : out_t;
  const HopR<R>& hc = op ? hAd : hA;
  int slot[B];
#pragma unroll
  for (int r = 0; r < B; ++r) slot[r] = (r < nsrc) ? rhs_map[j0 + r] : 0;

  if constexpr (STAGE) {
#pragma unroll
    for (int r = 0; r < B; ++r) {
      if (r < nsrc && live) {
        const T2* f = in + (long)slot[r] * 12 * V;
        constexpr unsigned e2 = 2 * sizeof(T2);
        const __amdgpu_buffer_rsrc_t rs = uniform_rsrc(f, 6u * e2 * (unsigned)V);
#pragma unroll
        for (int q = 0; q < 6; ++q) {  // component pairs: one 16-byte load each in FP32
          Cx<R> x0, x1;
          ld_pair_rs(rs, (unsigned)s * e2, (unsigned)q * e2 * (unsigned)V, x0, x1);
          plane[(r * 12 + 2 * q) * 256 + threadIdx.x] = T2{x0.re, x0.im};
          plane[(r * 12 + 2 * q + 1) * 256 + threadIdx.x] = T2{x1.re, x1.im};
        }
      }
    }
    __syncthreads();
  }
  auto load_nb = [&](int r, int n, Cx<R>(&p)[12]) {
    const unsigned d = (unsigned)(n - site0);
    if (STAGE && d < 256u) {
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const T2 v = plane[(r * 12 + c) * 256 + d];
        p[c] = {v.x, v.y};
      }
    } else {
      load_spinor_u(in + (long)slot[r] * 12 * V, V, n, false, p);
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
#define OVS_OP_DIR(NU)                                                                   \
  load_link_u(links, V, NU, nb.b[NU], u);                                                  \
  _Pragma("unroll") for (int r = 0; r < B; ++r) {                                        \
    if (r < nsrc) {                                                                      \
      load_nb(r, nb.b[NU], psi);                                                         \
      hop<R, NU, +1, false>(acc[r], u, psi, hc.fwd[NU]);                                 \
    }                                                                                    \
  }                                                                                      \
  load_link_u(links, V, NU, s, u);                                                         \
  _Pragma("unroll") for (int r = 0; r < B; ++r) {                                        \
    if (r < nsrc) {                                                                      \
      load_nb(r, nb.f[NU], psi);                                                         \
      hop<R, NU, -1, true>(acc[r], u, psi, hc.bwd[NU]);                                  \
    }                                                                                    \
  }
    OVS_OP_DIR(0)
    OVS_OP_DIR(1)
    OVS_OP_DIR(2)
    OVS_OP_DIR(3)
#undef OVS_OP_DIR
#pragma unroll
    for (int r = 0; r < B; ++r) {
      if (r < nsrc) {
        const long base = (long)slot[r] * 12 * V;
        Cx<R> p[12];
        load_nb(r, s, p);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          p[c] = p[c] - acc[r][c];
          if (c >= 6) p[c] = -p[c];
        }
        store_spinor(out + base, V, s, nt, p);
        if (!op) {
          Cx<R> pw[12];
          load_spinor_u(in_w + base, V, s, false, pw);
#pragma unroll
          for (int c = 0; c < 12; ++c) {
            const Cx<double> t64 = {(double)p[c].re, (double)p[c].im};
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
  if (op) return;  // uniform over the workgroup: only the A workgroup sums
  block_sum<3 * B>(part, lds);
  if (threadIdx.x == 0) {
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

}  // namespace ovs
