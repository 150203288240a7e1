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

// Y_new = alpha (MY - c Y) + beta Y_old   (Y_old may be null)
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
