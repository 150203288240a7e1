// Elementwise kernels of the deflation eigensolver (blocks of nb FP64 fields,
// each of padded length Np = 12*Vs).
#include "ovs_common.h"
#include "ovs_device.h"
#include "ovs_eig.h"

namespace ovs {

static int egrid(long n) {
  long b = (n + 255) / 256;
  if (b > 16384) b = 16384;
  if (b < 1) b = 1;
  return (int)b;
}

// Counter-based fill: the entry at flat offset e of a block gets (u1, u2)
// uniform in [-1, 1) from splitmix64 of (seed, e); pad entries are zero.
__device__ __forceinline__ unsigned long long splitmix(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void k_fill_random(double2* __restrict__ X, long nfields, int V, int Vs,
                              unsigned long long seed) {
  const long n = nfields * 12 * Vs;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int s = (int)(((e % (12L * Vs)) >> 1) % Vs);  // site of the pair layout
    if (s >= V) {
      X[e] = make_double2(0.0, 0.0);
      continue;
    }
    const unsigned long long h1 = splitmix(seed * 0x100000001B3ull + 2 * (unsigned long long)e);
    const unsigned long long h2 = splitmix(seed * 0x100000001B3ull + 2 * (unsigned long long)e + 1);
    const double u1 = (double)(h1 >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    const double u2 = (double)(h2 >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    X[e] = make_double2(u1, u2);
  }
}

// Y_new = alpha (MY - c Y) + beta Y_old   (Y_old may be null): scaling and axpby
__global__ void k_cheb(double2* __restrict__ Ynew, const double2* __restrict__ MY,
                       const double2* __restrict__ Y, const double2* __restrict__ Yold, double alpha,
                       double c, double beta, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const double2 my = MY[e], y = Y[e];
    double re = alpha * (my.x - c * y.x), im = alpha * (my.y - c * y.y);
    if (Yold) {
      const double2 yo = Yold[e];
      re += beta * yo.x;
      im += beta * yo.y;
    }
    Ynew[e] = make_double2(re, im);
  }
}

// D_j = AR_j - theta_j R_j for nb fields of length Np (theta: device complex [nb])
__global__ void k_resid(double2* __restrict__ D, const double2* __restrict__ AR,
                        const double2* __restrict__ R, const double2* __restrict__ theta, long Np) {
  const int j = blockIdx.y;
  const Cx<double> th = c64(theta[j]);
  const long off = (long)j * Np;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < Np; e += (long)gridDim.x * blockDim.x)
    D[off + e] = d2(c64(AR[off + e]) - cmul(th, c64(R[off + e])));
}

// Conjugate gradients on the normal equations M^H M x = M^H y for n sources
// at once (fields of Np entries, source j in workgroup row j).  With rr = |r|^2
// and tt = |M p|^2 of the step: alpha = rr / tt, x += alpha p, r -= alpha w
// (w = M^H M p), and per-workgroup partials of the new |r|^2.
__global__ void __launch_bounds__(256) k_cg_xr(double2* __restrict__ X, double2* __restrict__ R,
                                               const double2* __restrict__ P,
                                               const double2* __restrict__ W,
                                               const double* __restrict__ rr,
                                               const double* __restrict__ tt, long Np,
                                               double* __restrict__ part) {
  __shared__ double lds[4];
  const int j = blockIdx.y;
  const double a = tt[j] > 0.0 ? rr[j] / tt[j] : 0.0;
  const long off = (long)j * Np;
  double v[1] = {0.0};
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < Np; e += (long)gridDim.x * blockDim.x) {
    const double2 p = P[off + e], w = W[off + e], x = X[off + e], r = R[off + e];
    X[off + e] = make_double2(x.x + a * p.x, x.y + a * p.y);
    const double2 rn = make_double2(r.x - a * w.x, r.y - a * w.y);
    R[off + e] = rn;
    v[0] += rn.x * rn.x + rn.y * rn.y;
  }
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) part[(long)j * gridDim.x + blockIdx.x] = v[0];
}

// beta = rr' / rr with rr' the sum of k_cg_xr's partials (every workgroup
// forms it; workgroup 0 stores it in rr_next); p = r + beta p.
__global__ void __launch_bounds__(256) k_cg_p(double2* __restrict__ P, const double2* __restrict__ R,
                                              const double* __restrict__ rr,
                                              double* __restrict__ rr_next,
                                              const double* __restrict__ part, long Np) {
  __shared__ double lds[4];
  __shared__ double beta;
  const int j = blockIdx.y;
  const int nch = gridDim.x;
  double v[1] = {0.0};
  for (int q = threadIdx.x; q < nch; q += blockDim.x) v[0] += part[(long)j * nch + q];
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) {
    beta = rr[j] > 0.0 ? v[0] / rr[j] : 0.0;
    if (blockIdx.x == 0) rr_next[j] = v[0];
  }
  __syncthreads();
  const double b = beta;
  const long off = (long)j * Np;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < Np; e += (long)gridDim.x * blockDim.x) {
    const double2 r = R[off + e], p = P[off + e];
    P[off + e] = make_double2(r.x + b * p.x, r.y + b * p.y);
  }
}

int cg_nchunk(long Np) {
  long b = (Np + 1023) / 1024;
  if (b > 256) b = 256;
  if (b < 1) b = 1;
  return (int)b;
}

void launch_cg_xr(double2* X, double2* R, const double2* P, const double2* W, const double* rr,
                  const double* tt, int n, long Np, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_xr, dim3(cg_nchunk(Np), n), dim3(256), 0, s, X, R, P, W, rr, tt, Np, part);
}

void launch_cg_p(double2* P, const double2* R, const double* rr, double* rr_next,
                 const double* part, int n, long Np, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_p, dim3(cg_nchunk(Np), n), dim3(256), 0, s, P, R, rr, rr_next, part, Np);
}

void launch_fill_random(double2* X, long nfields, const Geometry& g, unsigned long long seed,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_fill_random, dim3(egrid(nfields * 12 * g.Vs)), dim3(256), 0, s, X, nfields,
                     g.V, g.Vs, seed);
}

void launch_cheb(double2* Ynew, const double2* MY, const double2* Y, const double2* Yold,
                 double alpha, double c, double beta, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_cheb, dim3(egrid(n)), dim3(256), 0, s, Ynew, MY, Y, Yold, alpha, c, beta, n);
}

void launch_resid(double2* D, const double2* AR, const double2* R, const double2* theta, int nb,
                  long Np, hipStream_t s) {
  long b = (Np + 255) / 256;
  if (b > 1024) b = 1024;
  hipLaunchKernelGGL(k_resid, dim3((int)b, nb), dim3(256), 0, s, D, AR, R, theta, Np);
}

}  // namespace ovs
