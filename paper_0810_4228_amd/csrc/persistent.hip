// Persistent chunked two-sided Lanczos (Section 4 recurrences).
//
// One cooperative launch runs `nit` full iterations.  An iteration is three
// phases: the dual stencil (T = A V~, S = A^dag W~ with per-tile partials),
// the update (alpha, then v~, w~ with their partials) and beta with the probe
// gather, with grid barriers after the stencil and after the update (beta
// runs beside the next iteration's stencil, which does not read it).  In every phase each workgroup loops over the
// virtual workgroups of that phase's separate kernel and runs the same body,
// so an iteration computes exactly what the per-step kernels compute (the
// partial sums keep their layout and order): results agree to the last bit.
// The grid is a multiple of 8, so virtual workgroup v runs on the XCD of
// workgroup v mod 8, as in the XCD-aware tile map of the separate launches.
//
// All workgroups are resident at once (cooperative launch), every workgroup
// passes the same number of barriers, and the loop count is fixed at launch:
// every wait ends.  The wait is also bounded: a workgroup that polls the
// barrier kBarrierPolls times sets an error word and goes on, so the launch
// ends even if residency were not met (the host then reports an error): once
// one workgroup has given up, the others stop waiting too.
#include "ovs_common.h"
#include "ovs_device.h"
#include "ovs_dual.h"
#include "ovs_krylov.h"
#include "ovs_lanczos.h"

namespace ovs {

// Barrier words in device memory (zero before the first launch, and zero
// again after every barrier except the generation word): an arrival counter
// per group of workgroups with equal index mod 8 (the workgroups of one XCD),
// a top counter and the generation, each in its own 128-byte line, and the
// error word.
constexpr int kBarCnt = 0;      // 8 counters, 32 words apart
constexpr int kBarTop = 256;
constexpr int kBarGen = 288;
constexpr int kBarErr = kPersistBarErr;
constexpr unsigned kBarrierPolls = 1u << 22;

// The workgroup meets (its waves' stores have reached L2).  Thread 0 reads
// the generation and arrives at its group counter with a release RMW (the
// workgroup's one agent-scope release, an L2 write-back).  The last of the
// group takes an acquire fence (it now orders after every arrival of its
// group), resets the counter and arrives at the top counter the same way; the
// last there advances the generation with a release RMW.  Waiters poll the
// generation with relaxed loads (an acquire load per poll would invalidate the
// caches every time) and take one acquire fence when it has moved; then the
// workgroup meets again and every wave takes an agent-scope acquire fence.
// Every workgroup's writes before the barrier are then visible to every
// workgroup after it.
__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned per_group) {
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned* gen = bar + kBarGen;
    const unsigned g0 = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned* cnt = bar + kBarCnt + 32 * (blockIdx.x & 7);
    if (__hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) ==
        per_group - 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      unsigned* top = bar + kBarTop;
      if (__hip_atomic_fetch_add(top, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) == 7u) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    // bounded: after kBarrierPolls polls, or once any workgroup has given up
    // (error word set, checked every 1024 polls), stop waiting
    unsigned polls = 0;
    while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
      __builtin_amdgcn_s_sleep(1);
      if (++polls >= kBarrierPolls) {
        __hip_atomic_fetch_or(bar + kBarErr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      if ((polls & 1023u) == 0 &&
          __hip_atomic_load(bar + kBarErr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
        break;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

template <typename R, int B, bool STAGE>
__global__ void __launch_bounds__(256)
k_persistent_2sl(const typename Vec2<R>::T* __restrict__ links, typename Vec2<R>::T* basis,
                 typename Vec2<R>::T* wbuf, long basis_stride, int ring, int* __restrict__ it,
                 typename Vec2<R>::T* T, typename Vec2<R>::T* S, double* part1, double* part2,
                 Geometry g, HopR<R> hA, HopR<R> hAd, const int* __restrict__ rhs_map,
                 const int* __restrict__ n_active, int nt_dual, int nt_update, TileMap tm,
                 int nv_dual, CoefArrays co, long N, int nwg_d, int nwg_u, int nslots,
                 const int* __restrict__ idx, int P, double2* probes, int nit,
                 unsigned* __restrict__ bar) {
  using T2 = typename Vec2<R>::T;
  const unsigned per_group = gridDim.x / 8;
  const int i0 = *it;
  const int na = *n_active;
  // The dual stencil of iteration i reads only the basis vectors, not the
  // coefficients that beta of iteration i-1 forms, so the two share one
  // interval between barriers: two barriers per iteration.
  for (int c = 0; c <= nit; ++c) {
    const int i = i0 + c;
    if (c > 0) {
      for (int jj = blockIdx.x; jj < nslots; jj += gridDim.x) {
        __syncthreads();
        beta_body<T2>(jj, i - 1, part2, nwg_u, co, rhs_map, na, basis, basis_stride, N, ring, idx,
                      P, probes);
      }
    }
    if (c == nit) break;  // the launch's end orders the last beta before later work
    for (int v = blockIdx.x; v < nv_dual; v += gridDim.x) {
      __syncthreads();  // LDS of the previous virtual workgroup
      dual_op_body<R, B, STAGE>(v, i, links, basis, wbuf, basis_stride, ring, T, S, part1, g, hA,
                                hAd, rhs_map, na, nt_dual, tm);
    }
    grid_barrier(bar, per_group);
    // the update forms alpha from the dual partials (as the per-step update does)
    for (int v = blockIdx.x; v < nwg_u * nslots; v += gridDim.x) {
      __syncthreads();
      update_body<T2>(v % nwg_u, v / nwg_u, nwg_u, i, T, S, basis, basis_stride, wbuf, N, N, co,
                      rhs_map, na, part2, ring, part1, nwg_d, nt_update);
    }
    grid_barrier(bar, per_group);
  }
  // every workgroup read *it before the first barrier
  if (blockIdx.x == 0 && threadIdx.x == 0) *it = i0 + nit;
}

template <typename R, int B, bool STAGE>
static hipError_t launch_p(const PersistArgs& a, const Geometry& g, const Hop& hA, const Hop& hAd,
                           hipStream_t s) {
  using T2 = typename Vec2<R>::T;
  const void* fn = (const void*)k_persistent_2sl<R, B, STAGE>;
  int dev = 0, ncu = 0, coop = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0);
  if (e != hipSuccess) return e;
  if (!coop || per_cu < 1) return hipErrorNotSupported;
  const TileMap tm = make_tile_map(g, 256, (a.nslots + B - 1) / B, a.order);
  const int nv_dual = 16 * tm.per_xcd;
  const int nwg_d = dual_num_wg(g), nwg_u = update_nwg(12L * g.Vs);
  // as many workgroups as can be resident, a multiple of 8, no more than the
  // largest phase has virtual workgroups
  int most = nv_dual > nwg_u * a.nslots ? nv_dual : nwg_u * a.nslots;
  most = (most + 7) / 8 * 8;
  // One workgroup per CU (fewest arrivals per barrier), or two when the dual
  // phase has 16 or more virtual workgroups per CU: the memory-bound phases
  // then hide more latency than the extra arrivals cost (measured: 16^3 x 32,
  // 12 sources 34 -> 43 solves/s; 8^4 loses with two, 235 -> 213; three and
  // four per CU lose on both).
  const int per = (nv_dual >= 16 * ncu && per_cu >= 2) ? 2 : 1;
  int grid = ncu * per;
  grid -= grid % 8;
  if (grid > most) grid = most;
  if (grid < 8) return hipErrorNotSupported;
  const T2* links = (const T2*)a.links;
  T2* basis = (T2*)a.basis;
  T2* wbuf = (T2*)a.wbuf;
  long basis_stride = a.basis_stride;
  int ring = a.ring ? 1 : 0;
  int* it = a.it;
  T2* T = (T2*)a.T;
  T2* S = (T2*)a.S;
  double* part1 = a.part1;
  double* part2 = a.part2;
  Geometry gg = g;
  HopR<R> ha = HopR<R>::make(hA), had = HopR<R>::make(hAd);
  const int* rhs_map = a.rhs_map;
  const int* n_active = a.n_active;
  int nt_dual = a.nt_dual, nt_update = a.nt_update;
  TileMap tmm = tm;
  int nvd = nv_dual;
  CoefArrays co = a.co;
  long N = 12L * g.Vs;
  int nwd = nwg_d, nwu = nwg_u, nslots = a.nslots;
  const int* idx = a.idx;
  int P = a.P;
  double2* probes = a.probes;
  int nit = a.nit;
  unsigned* bar = a.bar;
  void* args[] = {&links, &basis,  &wbuf,  &basis_stride, &ring,   &it,     &T,   &S,
                  &part1, &part2,  &gg,    &ha,           &had,    &rhs_map, &n_active,
                  &nt_dual, &nt_update, &tmm, &nvd,      &co,     &N,      &nwd, &nwu,
                  &nslots, &idx,   &P,     &probes,       &nit,    &bar};
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(256), args, 0, s);
}

hipError_t launch_persistent(bool f32, const PersistArgs& a, const Geometry& g, const Hop& hA,
                             const Hop& hAd, hipStream_t s) {
  if (a.nit < 1 || a.nslots < 1) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  if (f32) {
    switch (a.rhs_block * 2 + (a.stage ? 1 : 0)) {
      case 2: e = launch_p<float, 1, false>(a, g, hA, hAd, s); break;
      case 3: e = launch_p<float, 1, true>(a, g, hA, hAd, s); break;
      case 4: e = launch_p<float, 2, false>(a, g, hA, hAd, s); break;
      case 5: e = launch_p<float, 2, true>(a, g, hA, hAd, s); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (a.rhs_block * 2 + (a.stage ? 1 : 0)) {
      case 2: e = launch_p<double, 1, false>(a, g, hA, hAd, s); break;
      case 3: e = launch_p<double, 1, true>(a, g, hA, hAd, s); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace ovs
