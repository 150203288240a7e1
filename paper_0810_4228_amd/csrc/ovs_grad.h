// Kernels of the sign-function gradient (grad.hip) and their launchers.
//
// The gradient is the reverse sweep of the two-sided Lanczos approximation
// y_k = |b| V_k sgn(G_k) e_1 (Section 4, no deflation).  All fields here are
// FP64, [nrhs][12][Vs] with pads zero; per-source scalars are [nrhs] or
// [nrhs][kmax] arrays of double / double2 in device memory.
#pragma once

#include "ovs_common.h"

namespace ovs {

constexpr int kLinTerms = 5;
constexpr int kLinDots = 2;

// out_r = sum_j coef[j*nrhs + r] * x_j,r (+ out_r when accumulate), and
// partial sums of dot_q,r = sum conj(y_q,r) * out_r (y_q = nullptr: the
// combination itself).  out may be null (dots only).  Source r's field is at
// offset r*stride of every pointer.
struct LinArgs {
  const double2* x[kLinTerms] = {};
  int nterm = 0;
  const double2* coef = nullptr;   // [kLinTerms][nrhs]
  double2* out = nullptr;
  int accumulate = 0;
  const double2* y[kLinDots] = {};
  int ndot = 0;
  double* partials = nullptr;      // [nrhs][lin_nchunk][kLinDots][2]
  int tab = -1;                    // >= 0: coefficients from this table of the
                                   // launch's scalar step (launch_lin_step), not coef
};
int lin_nchunk(long stride);
void launch_lin(const LinArgs& a, long stride, int nrhs, hipStream_t s);
// Up to kLinMulti combinations in one launch, each computed exactly as
// launch_lin computes it.  Every combination visits the elements in the same
// thread order, so one may read (as a term or a dot operand) the output of an
// earlier one in the list, element by element; nothing else of another's
// output.
constexpr int kLinMulti = 4;
struct LinMulti {
  LinArgs a[kLinMulti];
  int n = 0;
};
void launch_lin_multi(const LinMulti& m, long stride, int nrhs, hipStream_t s);
// su(3) force F = -TA(U G^dagger) of nlinks links (canonical [..][3][3] layout).
void launch_link_force(const double2* U, const double2* G, double2* F, long nlinks,
                       hipStream_t s);

// Per-source scalar steps (one thread per source); see grad.hip.
struct GradScalars {
  double2* alpha;    // [nrhs][kmax]
  double* beta;      // [nrhs][kmax]
  double2* gamma;    // [nrhs][kmax]
  double* tnorm2;    // [nrhs][kmax]
  double2* x;        // [nrhs][kmax]  sgn(G_k) e_1
  double2* xbar;     // [nrhs][kmax]
  double2* abar;     // [nrhs][kmax]
  double* bbar;      // [nrhs][kmax]
  double2* gbar;     // [nrhs][kmax]
  double* nb;        // [nrhs]
  double2* sigma;    // [nrhs] b_L^dagger b_R of LR-deflated starts (Section 3)
  int* status;       // [nrhs] 0 ok, 1 lucky breakdown, 2 serious breakdown
  double2* coef;     // [kCoefTables][kLinTerms][nrhs]
  int kmax;
  int nrhs;
};
constexpr int kCoefTables = 11;
// Coefficient tables (indices into GradScalars::coef).
enum {
  kTabNorm = 0,  // forward: [1/|b|]
  kTabV = 1,     // forward: v~ = t - alpha v_i - gamma_{i-1} v_{i-1};  reverse: vbar~_i
  kTabW = 2,     // forward: w~ = s - conj(alpha) w_i - beta_{i-1} w_{i-1}; reverse: wbar~_i
  kTabSV = 3,    // forward: [1/beta_i];  reverse: tbar_i
  kTabSW = 4,    // forward: [1/conj(gamma_i)];  reverse: vbar_i
  kTabWB = 5,    // reverse: wbar_i
  kTabOne = 6,   // [1, 1, 1, 1, 1]
  kTabFin = 7,   // reverse: grad_b = ubar/|b| + nbar v_1
  kTabY = 8,     // reverse: y += |b| x_i v_i
  kTabStartW = 9,  // deflated forward: w_1 = b_L |b_R| / conj(sigma)
  kTabFinW = 10    // deflated reverse: bbar_L
};
inline double2* coef_table(const GradScalars& s, int t) {
  return s.coef + (long)t * kLinTerms * s.nrhs;
}

// forward
void launch_gf_norm(const GradScalars& s, const double* part, int nchunk, hipStream_t st);
// LR-deflated starts (Section 3): from the dots |b_R|^2 (dot 0) and
// sigma = b_L^dagger b_R (dot 1) of part, and |b|^2 (dot 0 of part_b):
// nb = |b_R|, v_1 = b_R / nb (kTabNorm), w_1 = b_L nb / conj(sigma)
// (kTabStartW), so that w_1^dagger v_1 = 1; status 2 when sigma = 0 or
// |b_R| <= 1e-12 |b|.
void launch_gf_start(const GradScalars& s, const double* part, const double* part_b, int nchunk,
                     hipStream_t st);
void launch_gf_alpha(const GradScalars& s, int i, const double* part, int nchunk, hipStream_t st);
// reverse
void launch_gr_first(const GradScalars& s, hipStream_t st);
void launch_gr_final(const GradScalars& s, const double* part, int nchunk, hipStream_t st);
// Deflated starts: from v_1^dagger vbar_1 (part_v, dot 0) and w_1^dagger wbar_1
// (part_w, dot 0), the adjoints of b_R and b_L:
//   bbar_R = vbar_1 / nb + tau b_L + (nbar / nb) b_R     (kTabFin: 1/nb, tau, nbar/nb)
//   bbar_L = (nb / sigma) wbar_1 + conj(tau) b_R         (kTabFinW: nb/sigma, conj(tau))
// with rho = wbar_1^dagger w_1, tau = -rho / conj(sigma) and
// nbar = (Re chi^dagger y_K - Re vbar_1^dagger v_1 + Re rho) / nb.
void launch_gr_final_defl(const GradScalars& s, const double* part_v, const double* part_w,
                          int nchunk, hipStream_t st);

// A scalar step run at the start of a combination launch (launch_lin_step,
// launch_lin_multi_step), one workgroup per chunk and source, each forming
// the step's rows with the same sums: alpha (pa: partials of w_i^dagger t
// and |t|^2), beta (pa: |v~|^2; pb: v~^dagger w~ and |w~|^2), xbar (pa:
// chi^dagger v_i), the replay rows of step i from the stored coefficients
// (no dots, the arithmetic of alpha and beta, so replayed vectors are
// bitwise equal), reverse step 1 (pa: vbar_{i+1}^dagger v_{i+1}; pb:
// wbar_{i+1}^dagger w_{i+1}) and reverse step 2 (pa: v_i^dagger vbar~,
// v_{i-1}^dagger vbar~; pb: the same with w and wbar~).  The rows go to the
// launch's tables for combinations with LinArgs::tab >= 0; global_tabs: also
// to the global tables (for later launches).  Reverse steps 1 and 2 do not
// write back gbar_i, bbar_i and abar_i, which nothing reads after them.
enum { kStepNone = 0, kStepAlpha, kStepBeta, kStepXbar, kStepCoef, kStepS1, kStepS2 };
struct ScalarStep {
  int kind = kStepNone;
  int i = 0;
  const double* pa = nullptr;
  const double* pb = nullptr;
  int nchunk = 0;
  GradScalars s{};
  int global_tabs = 0;
};
void launch_lin_step(const LinArgs& a, long stride, int nrhs, const ScalarStep& st, hipStream_t s);
void launch_lin_multi_step(const LinMulti& m, long stride, int nrhs, const ScalarStep& st,
                           hipStream_t s);

// xbar_i = nb * conj(dot 0) for the dot chi^dagger v_i of the partials.
void launch_gf_xbar(const GradScalars& s, int i, const double* part, int nchunk, hipStream_t st);
// Inner sign and its vector-Jacobian product for one source by the tau = e^u
// trapezoid rule at step h: x = (1/pi) int sum_+- (G +- i tau)^{-1} e_1 dtau and
// Gbar (band of G) = -(1/pi) int sum_+- p conj(q)^T dtau with
// q = (G +- i tau)^{-1} e_1, p = (G +- i tau)^{-H} xbar.
struct IsignVjpOut {
  double2* x;        // [k]
  double2* gd;       // [k]   Gbar_{i,i}
  double* gsub_re;   // [k-1] Re Gbar_{i+1,i} (beta_i is real)
  double2* gsup;     // [k-1] Gbar_{i,i+1}
};
size_t isign_vjp_scratch_bytes(int k, int nnode);
// coarse (optional): also the rule of step 2h from the same solves (the
// nodes of even index), its x, gd and gsup, for comparing two levels with one
// launch.
void launch_isign_vjp(const double2* alpha, const double* beta, const double2* gamma,
                      const double2* xbar, int k, double h, int n0, int nnode, void* scratch,
                      const IsignVjpOut& out, hipStream_t st,
                      const IsignVjpOut* coarse = nullptr);

// Link force: F ([5][9][Vs] FP64, packed-link gradient; slot 3 the e^{+mu}
// part and slot 4 the e^{-mu} part of direction 4) += gradient of
//   Re <pbar, A(mu) p> + Re <qbar, A(mu)^dagger q>   summed over sources.
// q/qbar may be null.
void launch_gforce(double2* F, const double2* pbar, const double2* p, const double2* qbar,
                   const double2* q, long stride, int nrhs, const Geometry& g, const Hop& hA,
                   const Hop& hAd, hipStream_t st);
// The same force for nsteps reverse steps at once (both terms present):
// step j's pbar, p, qbar, q are at pbar0 + j step_stride etc.; their
// contributions are summed in registers and F is read and written once.
void launch_gforce_group(double2* F, const double2* pbar0, const double2* p0,
                         const double2* qbar0, const double2* q0, int nsteps, long step_stride,
                         long stride, int nrhs, const Geometry& g, const Hop& hA, const Hop& hAd,
                         hipStream_t st);
// grad_U (canonical [V][4][3][3]) = boundary sign * (F_nu + [nu=3] F_4), and
// grad_mu = Re sum tr(F_3^dagger U_4) - Re sum tr(F_4^dagger U_4) (packed links).
void launch_gforce_out(const double2* F, const double2* links, const Geometry& g, const int bc[4],
                       double2* grad_U, double* partials, double* grad_mu, hipStream_t st);

}  // namespace ovs
