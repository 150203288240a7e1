// ovs_sign_apply_vjp: the gradient of L = sum_r Re <chi_r, y_r> with
// y_r = |b_r| V_k sgn(G_k) e_1 (two-sided Lanczos of Section 4 at fixed k,
// no deflation) with respect to the sources b, the chemical potential mu and
// the links U.
//
// Forward: the recurrences (4.1)-(4.4) with FP64 bases V, W kept in HBM
// (2 k nrhs fields; 288 GB holds k = 1000 at 16^3 x 32 for several sources,
// so nothing is recomputed).  Inner sign: sgn(G_k) e_1 and its vector-Jacobian
// product from the same tau = e^u trapezoid rule, step h halved until two
// levels agree.  Reverse sweep: per iteration two linear-combination passes
// with fused dots, two scalar steps, the stencil adjoints A^dagger tbar and
// A sbar, and the link-force accumulation (grad.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "ovs_common.h"
#include "ovs_grad.h"
#include "ovs_host.h"

using namespace ovs;

namespace {

constexpr double kVjpULo = -40.0, kVjpUHi = 45.0;  // u range of the tau = e^u rule
constexpr double kVjpHStart = 0.25, kVjpHMin = 1.0 / 32.0;
constexpr double kVjpAccept = 1e-10;  // relative change between two step levels

void vjp_range(double h, int& n0, int& nnode) {
  n0 = (int)std::floor(kVjpULo / h);
  nnode = (int)std::ceil(kVjpUHi / h) - n0 + 1;
}

double max_rel_change(const std::vector<double2>& a, const std::vector<double2>& b) {
  double num = 0.0, den = 0.0;
  for (size_t i = 0; i < a.size(); ++i) {
    num = std::max(num, std::hypot(a[i].x - b[i].x, a[i].y - b[i].y));
    den = std::max(den, std::hypot(a[i].x, a[i].y));
  }
  return den > 0.0 ? num / den : num;
}

}  // namespace

extern "C" ovs_status ovs_sign_apply_vjp(ovs_lattice l, const void* b, const void* chi,
                                         int32_t nrhs, int32_t k, void* y, void* grad_b,
                                         double* grad_mu, void* grad_U, double* quad_err) {
  if (!l || !b || !chi || !grad_b || !grad_mu || !grad_U) return OVS_ERR_ARG;
  if (nrhs < 1 || nrhs > kMaxNrhs || k < 1 || k > 65535) return OVS_ERR_ARG;
  if (l->prec != OVS_F64) return OVS_ERR_ARG;
  if (!ready(l)) return OVS_ERR_STATE;
  const Geometry& g = l->g;
  const long F = 12L * g.Vs;        // elements of one source field
  const long NF = (long)nrhs * F;   // elements of one batch of fields
  const int nch = lin_nchunk(F);
  int n0max, nnmax;
  vjp_range(kVjpHMin, n0max, nnmax);

  // ---- workspace ----
  auto carve = [&](Arena& a, double2*& V, double2*& W, double2** fld, GradScalars& s,
                   double2*& Fg, double*& parts, double*& bparts, double*& fparts, double*& gmu,
                   void*& vjp, IsignVjpOut (&vo)[2]) {
    V = a.take<double2>((size_t)k * NF);
    W = a.take<double2>((size_t)k * NF);
    for (int j = 0; j < 16; ++j) fld[j] = a.take<double2>(NF);
    Fg = a.take<double2>(5L * 9 * g.Vs);
    const size_t nk = (size_t)nrhs * k;
    s.alpha = a.take<double2>(nk);
    s.beta = a.take<double>(nk);
    s.gamma = a.take<double2>(nk);
    s.tnorm2 = a.take<double>(nk);
    s.x = a.take<double2>(nk);
    s.xbar = a.take<double2>(nk);
    s.abar = a.take<double2>(nk);
    s.bbar = a.take<double>(nk);
    s.gbar = a.take<double2>(nk);
    s.nb = a.take<double>(nrhs);
    s.status = a.take<int>(nrhs);
    s.coef = a.take<double2>((size_t)kCoefTables * kLinTerms * nrhs);
    s.kmax = k;
    s.nrhs = nrhs;
    parts = a.take<double>((size_t)4 * nrhs * nch * 2 * kLinDots);
    bparts = a.take<double>((size_t)nrhs * k * 32 * 2);
    fparts = a.take<double>((size_t)(g.V + kWG - 1) / kWG + 1);
    gmu = a.take<double>(1);
    vjp = a.take<char>(isign_vjp_scratch_bytes(k, nnmax));
    for (int lv = 0; lv < 2; ++lv) {
      vo[lv].x = a.take<double2>(k);
      vo[lv].gd = a.take<double2>(k);
      vo[lv].gsub_re = a.take<double>(k);
      vo[lv].gsup = a.take<double2>(k);
    }
  };
  double2 *V, *W, *fld[16], *Fg;
  GradScalars S;
  double *parts, *bparts, *fparts, *gmu_dev;
  void* vjp;
  IsignVjpOut vo[2];
  Arena sizing{nullptr};
  carve(sizing, V, W, fld, S, Fg, parts, bparts, fparts, gmu_dev, vjp, vo);
  ovs_status st = ensure_ws(l, sizing.off + 256);
  if (st != OVS_OK) return st;
  StreamScope scope(l);
  Arena a{(char*)l->ws};
  carve(a, V, W, fld, S, Fg, parts, bparts, fparts, gmu_dev, vjp, vo);
  double2 *B = fld[0], *CHI = fld[1], *T = fld[2], *Sv = fld[3];
  double2* VB[2] = {fld[4], fld[5]};
  double2* WB[2] = {fld[6], fld[7]};
  double2* VTB[2] = {fld[8], fld[9]};
  double2* WTB[2] = {fld[10], fld[11]};
  double2 *TB = fld[12], *T1 = fld[13], *T2 = fld[14], *GB = fld[15];
  double* P[4];
  for (int j = 0; j < 4; ++j) P[j] = parts + (size_t)j * nrhs * nch * 2 * kLinDots;

  // every field starts at zero (pads stay zero: the stencil writes sites < V only)
  OVS_HIP(hipMemsetAsync(V, 0, (size_t)((char*)(fld[15] + NF) - (char*)V), l->stream));
  OVS_HIP(hipMemsetAsync(Fg, 0, sizeof(double2) * 5 * 9 * g.Vs, l->stream));
  {
    std::vector<double2> ones((size_t)kLinTerms * nrhs, make_double2(1.0, 0.0));
    OVS_HIP(hipMemcpyAsync(coef_table(S, kTabOne), ones.data(), sizeof(double2) * ones.size(),
                           hipMemcpyHostToDevice, l->stream));
    OVS_HIP(hipStreamSynchronize(l->stream));
  }
  launch_pack_f64((const double2*)b, B, nrhs, g, l->stream);
  launch_pack_f64((const double2*)chi, CHI, nrhs, g, l->stream);

  const Hop hA = make_hop(l->m_w, l->mu), hAd = make_hop(l->m_w, -l->mu);
  const Tuning tn = get_tuning(l, nrhs);
  auto applyA = [&](const double2* in, double2* out) {
    return launch_wilson(false, l->links, in, out, nrhs, g, hA, false, true, tn, l->stream);
  };
  auto applyAd = [&](const double2* in, double2* out) {
    return launch_wilson(false, l->links, in, out, nrhs, g, hAd, false, true, tn, l->stream);
  };
  auto Vi = [&](int i) { return V + (size_t)i * NF; };
  auto Wi = [&](int i) { return W + (size_t)i * NF; };
  auto lin = [&](std::initializer_list<const double2*> xs, int tab, double2* out, bool acc,
                 std::initializer_list<const double2*> ys, int ndot, double* part) {
    LinArgs la;
    int j = 0;
    for (const double2* p : xs) la.x[j++] = p;
    la.nterm = j;
    la.coef = coef_table(S, tab);
    la.out = out;
    la.accumulate = acc ? 1 : 0;
    j = 0;
    for (const double2* p : ys) {
      if (j < ndot) la.y[j] = p;
      ++j;
    }
    la.ndot = ndot;
    la.partials = part;
    launch_lin(la, F, nrhs, l->stream);
  };

  // ---- forward: v_1 = w_1 = b/|b|, then the recurrences ----
  lin({B}, kTabOne, nullptr, false, {nullptr}, 1, P[0]);
  launch_gf_norm(S, P[0], nch, l->stream);
  lin({B}, kTabNorm, Vi(0), false, {}, 0, nullptr);
  lin({B}, kTabNorm, Wi(0), false, {}, 0, nullptr);
  for (int i = 0; i < k; ++i) {
    OVS_HIP(applyA(Vi(i), T));
    lin({T}, kTabOne, nullptr, false, {Wi(i), nullptr}, 2, P[0]);
    launch_gf_alpha(S, i, P[0], nch, l->stream);
    if (i == k - 1) break;  // T keeps t_k = A v_k
    OVS_HIP(applyAd(Wi(i), Sv));
    if (i > 0) {
      lin({T, Vi(i), Vi(i - 1)}, kTabV, Vi(i + 1), false, {nullptr}, 1, P[1]);
      lin({Sv, Wi(i), Wi(i - 1)}, kTabW, Wi(i + 1), false, {Vi(i + 1), nullptr}, 2, P[2]);
    } else {
      lin({T, Vi(i)}, kTabV, Vi(i + 1), false, {nullptr}, 1, P[1]);
      lin({Sv, Wi(i)}, kTabW, Wi(i + 1), false, {Vi(i + 1), nullptr}, 2, P[2]);
    }
    launch_gf_beta(S, i, P[1], P[2], nch, l->stream);
    lin({Vi(i + 1)}, kTabSV, Vi(i + 1), false, {}, 0, nullptr);
    lin({Wi(i + 1)}, kTabSW, Wi(i + 1), false, {}, 0, nullptr);
  }
  OVS_HIP(hipGetLastError());
  std::vector<int> status(nrhs);
  OVS_HIP(hipMemcpyAsync(status.data(), S.status, sizeof(int) * nrhs, hipMemcpyDeviceToHost,
                         l->stream));
  OVS_HIP(hipStreamSynchronize(l->stream));
  for (int r = 0; r < nrhs; ++r)
    if (status[r] != 0) return OVS_WARN_BREAKDOWN;  // the gradient needs k full iterations

  // ---- xbar_i = |b| v_i^dagger chi; inner sign and its VJP ----
  launch_basis_dots(V, CHI, F, k, nrhs, bparts, S, l->stream);
  ovs_status result = OVS_OK;
  for (int r = 0; r < nrhs; ++r) {
    const size_t rk = (size_t)r * k;
    std::vector<double2> prev, cur;
    double h = kVjpHStart, change = 0.0;
    int lv = 0, used = 0;
    for (;; h *= 0.5, lv ^= 1) {
      int n0, nn;
      vjp_range(h, n0, nn);
      launch_isign_vjp(S.alpha + rk, S.beta + rk, S.gamma + rk, S.xbar + rk, k, h, n0, nn, vjp,
                       vo[lv], l->stream);
      OVS_HIP(hipGetLastError());
      cur.assign((size_t)3 * k, make_double2(0.0, 0.0));
      OVS_HIP(hipMemcpyAsync(cur.data(), vo[lv].x, sizeof(double2) * k, hipMemcpyDeviceToHost,
                             l->stream));
      OVS_HIP(hipMemcpyAsync(cur.data() + k, vo[lv].gd, sizeof(double2) * k,
                             hipMemcpyDeviceToHost, l->stream));
      if (k > 1)
        OVS_HIP(hipMemcpyAsync(cur.data() + 2 * k, vo[lv].gsup, sizeof(double2) * (k - 1),
                               hipMemcpyDeviceToHost, l->stream));
      OVS_HIP(hipStreamSynchronize(l->stream));
      used = lv;
      if (!prev.empty()) {
        change = max_rel_change(cur, prev);
        if (change <= kVjpAccept) break;
      }
      if (h <= kVjpHMin) break;
      prev.swap(cur);
    }
    if (quad_err) quad_err[r] = change;
    if (change > 1e-6) result = OVS_WARN_SIGN_AMBIGUOUS;
    OVS_HIP(hipMemcpyAsync(S.x + rk, vo[used].x, sizeof(double2) * k, hipMemcpyDeviceToDevice,
                           l->stream));
    OVS_HIP(hipMemcpyAsync(S.abar + rk, vo[used].gd, sizeof(double2) * k,
                           hipMemcpyDeviceToDevice, l->stream));
    if (k > 1) {
      OVS_HIP(hipMemcpyAsync(S.bbar + rk, vo[used].gsub_re, sizeof(double) * (k - 1),
                             hipMemcpyDeviceToDevice, l->stream));
      OVS_HIP(hipMemcpyAsync(S.gbar + rk, vo[used].gsup, sizeof(double2) * (k - 1),
                             hipMemcpyDeviceToDevice, l->stream));
    }
  }

  // ---- reverse sweep ----
  {
    const int i = k - 1, c = i & 1;
    launch_gr_first(S, l->stream);
    lin({Wi(i)}, kTabSV, TB, false, {}, 0, nullptr);                      // tbar
    lin({CHI}, kTabSW, VB[c], false, {}, 0, nullptr);                     // vbar (direct part)
    lin({T}, kTabWB, WB[c], false, {Wi(i)}, 1, P[3]);                     // wbar, complete
    OVS_HIP(applyAd(TB, T1));
    lin({T1}, kTabOne, VB[c], true, {Vi(i)}, 1, P[2]);                    // vbar += A^dag tbar
    launch_gforce(Fg, TB, Vi(i), nullptr, nullptr, F, nrhs, g, hA, hAd, l->stream);
  }
  for (int i = k - 2; i >= 0; --i) {
    const int c = i & 1, p = (i + 1) & 1;
    launch_gr_s1(S, i, P[2], P[3], nch, l->stream);
    if (i > 0) {
      lin({VB[p], Vi(i + 1), Wi(i + 1)}, kTabV, VTB[c], false, {Vi(i), Vi(i - 1)}, 2, P[0]);
      lin({WB[p], Vi(i + 1)}, kTabW, WTB[c], false, {Wi(i), Wi(i - 1)}, 2, P[1]);
    } else {
      lin({VB[p], Vi(i + 1), Wi(i + 1)}, kTabV, VTB[c], false, {Vi(i)}, 1, P[0]);
      lin({WB[p], Vi(i + 1)}, kTabW, WTB[c], false, {Wi(i)}, 1, P[1]);
    }
    launch_gr_s2(S, i, P[0], P[1], nch, l->stream);
    lin({VTB[c], Wi(i)}, kTabSV, TB, false, {}, 0, nullptr);
    lin({CHI, VTB[p], VTB[c]}, kTabSW, VB[c], false, {}, 0, nullptr);
    if (i > 0)
      lin({WTB[p], WTB[c], Vi(i + 1), Vi(i), Vi(i - 1)}, kTabWB, WB[c], false, {}, 0, nullptr);
    else
      lin({WTB[p], WTB[c], Vi(i + 1), Vi(i)}, kTabWB, WB[c], false, {}, 0, nullptr);
    OVS_HIP(applyAd(TB, T1));
    OVS_HIP(applyA(WTB[c], T2));
    lin({T1}, kTabOne, VB[c], true, {Vi(i)}, 1, P[2]);
    lin({T2}, kTabOne, WB[c], true, {Wi(i)}, 1, P[3]);
    launch_gforce(Fg, TB, Vi(i), WTB[c], Wi(i), F, nrhs, g, hA, hAd, l->stream);
  }
  // grad_b = ubar/|b| + nbar v_1,  ubar = vbar_1 + wbar_1
  lin({VB[0], WB[0]}, kTabOne, T1, false, {Vi(0)}, 1, P[0]);
  launch_gr_final(S, P[0], nch, l->stream);
  lin({T1, Vi(0)}, kTabFin, GB, false, {}, 0, nullptr);
  launch_unpack_f64(GB, (double2*)grad_b, nrhs, g, l->stream);
  launch_gforce_out(Fg, (const double2*)l->links, g, l->bc, (double2*)grad_U, fparts, gmu_dev,
                    l->stream);
  if (y) {
    launch_gcombine(V, F, k, nrhs, S, T2, l->stream);
    launch_unpack_f64(T2, (double2*)y, nrhs, g, l->stream);
  }
  OVS_HIP(hipGetLastError());
  OVS_HIP(hipMemcpyAsync(grad_mu, gmu_dev, sizeof(double), hipMemcpyDeviceToHost, l->stream));
  OVS_HIP(hipStreamSynchronize(l->stream));
  return result;
}
