// ovs_sign_apply_vjp: the gradient of L = sum_r Re <chi_r, y_r> with
// y_r = |b_r| V_k sgn(G_k) e_1 (two-sided Lanczos of Section 4 at fixed k,
// no deflation) with respect to the sources b, the chemical potential mu and
// the links U.
//
// Forward: the recurrences (4.1)-(4.4) in FP64.  By default only checkpoints
// are kept: the pairs (v_{jc-1}, v_{jc}), (w_{jc-1}, w_{jc}) every c = ceil(sqrt k)
// steps; the reverse sweep replays each segment forward from its checkpoint
// with the stored coefficients (the same kernels and coefficient arithmetic as
// the forward pass, so the replayed vectors are bitwise those of the forward)
// and then walks it backwards.  Memory: about 4k/c + 2c + 18 fields per
// source instead of 2k + 18; cost: one more forward pass.  With
// OVS_VJP_STORE_BASIS both bases are kept instead.
// Inner sign: sgn(G_k) e_1 and its vector-Jacobian product from the same
// tau = e^u trapezoid rule, step h halved until two levels agree.  Reverse
// sweep: per iteration linear-combination passes with fused dots, two scalar
// steps, the stencil adjoints A^dagger tbar and A sbar, and the link-force
// accumulation (grad.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
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

// The vjp proper; with ws_query != NULL only the workspace it needs is
// computed (the other pointers are not used).
static ovs_status vjp_impl(ovs_lattice l, const void* b, const void* chi, int32_t nrhs, int32_t k,
                           int32_t flags, void* y, void* grad_b, double* grad_mu, void* grad_U,
                           double* quad_err, void* user_ws, size_t user_ws_bytes,
                           size_t* ws_query) {
  if (!l || (!ws_query && (!b || !chi || !grad_b || !grad_mu || !grad_U))) return OVS_ERR_ARG;
  if (nrhs < 1 || nrhs > kMaxNrhs || k < 1 || k > 65535) return OVS_ERR_ARG;
  if (flags & ~OVS_VJP_STORE_BASIS) return OVS_ERR_ARG;
  if (l->prec != OVS_F64 || l->parent) return OVS_ERR_ARG;
  if (!ws_query && !ready(l)) return OVS_ERR_STATE;
  const bool store = (flags & OVS_VJP_STORE_BASIS) != 0;
  const Geometry& g = l->g;
  const long F = 12L * g.Vs;        // elements of one source field
  const long NF = (long)nrhs * F;   // elements of one batch of fields
  const int nch = lin_nchunk(F);
  const int cseg = store ? k : std::max(1, (int)std::ceil(std::sqrt((double)k)));
  const int nseg = (k + cseg - 1) / cseg;
  int n0max, nnmax;
  vjp_range(kVjpHMin, n0max, nnmax);
  constexpr int kFields = 18;

  // ---- workspace ----
  struct Ptrs {
    double2 *V, *W, *ckV, *ckW, *fld[kFields], *Fg;
    double *parts, *fparts, *gmu;
    void* vjp;
    IsignVjpOut vo[2];
  } P_{};
  GradScalars S{};
  auto carve = [&](Arena& a) {
    if (store) {
      P_.V = a.take<double2>((size_t)k * NF);
      P_.W = a.take<double2>((size_t)k * NF);
    } else {
      P_.V = a.take<double2>((size_t)(cseg + 2) * NF);   // segment buffer (forward ring)
      P_.W = a.take<double2>((size_t)(cseg + 2) * NF);
      P_.ckV = a.take<double2>((size_t)2 * nseg * NF);
      P_.ckW = a.take<double2>((size_t)2 * nseg * NF);
    }
    for (int j = 0; j < kFields; ++j) P_.fld[j] = a.take<double2>(NF);
    P_.Fg = a.take<double2>(5L * 9 * g.Vs);
    const size_t nk = (size_t)nrhs * k;
    S.alpha = a.take<double2>(nk);
    S.beta = a.take<double>(nk);
    S.gamma = a.take<double2>(nk);
    S.tnorm2 = a.take<double>(nk);
    S.x = a.take<double2>(nk);
    S.xbar = a.take<double2>(nk);
    S.abar = a.take<double2>(nk);
    S.bbar = a.take<double>(nk);
    S.gbar = a.take<double2>(nk);
    S.nb = a.take<double>(nrhs);
    S.status = a.take<int>(nrhs);
    S.coef = a.take<double2>((size_t)kCoefTables * kLinTerms * nrhs);
    S.kmax = k;
    S.nrhs = nrhs;
    P_.parts = a.take<double>((size_t)4 * nrhs * nch * 2 * kLinDots);
    P_.fparts = a.take<double>((size_t)(g.V + kWG - 1) / kWG + 1);
    P_.gmu = a.take<double>(1);
    P_.vjp = a.take<char>(isign_vjp_scratch_bytes(k, nnmax));
    for (int lv = 0; lv < 2; ++lv) {
      P_.vo[lv].x = a.take<double2>(k);
      P_.vo[lv].gd = a.take<double2>(k);
      P_.vo[lv].gsub_re = a.take<double>(k);
      P_.vo[lv].gsup = a.take<double2>(k);
    }
  };
  Arena sizing{nullptr};
  carve(sizing);
  if (ws_query) {
    *ws_query = sizing.off + 512;
    return OVS_OK;
  }
  char* ws_base;
  if (user_ws) {
    if (user_ws_bytes < sizing.off + 512) return OVS_ERR_ARG;
    ws_base = (char*)(((uintptr_t)user_ws + 255) & ~uintptr_t(255));
  } else {
    ovs_status st0 = ensure_ws(l, sizing.off + 256);
    if (st0 != OVS_OK) return st0;
    ws_base = (char*)l->ws;
  }
  ovs_status st = OVS_OK;
  StreamScope scope(l);
  Arena arena{ws_base};
  carve(arena);
  double2** fld = P_.fld;
  double2 *B = fld[0], *CHI = fld[1], *T = fld[2], *Sv = fld[3];
  double2* VB[2] = {fld[4], fld[5]};
  double2* WB[2] = {fld[6], fld[7]};
  double2* VTB[2] = {fld[8], fld[9]};
  double2* WTB[2] = {fld[10], fld[11]};
  double2 *TB = fld[12], *T1 = fld[13], *T2 = fld[14], *GB = fld[15], *TL = fld[16],
          *YA = fld[17];
  double* P[4];
  for (int j = 0; j < 4; ++j) P[j] = P_.parts + (size_t)j * nrhs * nch * 2 * kLinDots;

  // every field starts at zero (pads stay zero: the stencil writes sites < V only)
  OVS_HIP(hipMemsetAsync(P_.V, 0, (size_t)((char*)(fld[kFields - 1] + NF) - (char*)P_.V),
                         l->stream));
  OVS_HIP(hipMemsetAsync(P_.Fg, 0, sizeof(double2) * 5 * 9 * g.Vs, l->stream));
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
  auto mk = [&](std::initializer_list<const double2*> xs, int tab, double2* out, bool acc,
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
    return la;
  };
  auto lin = [&](std::initializer_list<const double2*> xs, int tab, double2* out, bool acc,
                 std::initializer_list<const double2*> ys, int ndot, double* part) {
    launch_lin(mk(xs, tab, out, acc, ys, ndot, part), F, nrhs, l->stream);
  };
  // independent combinations (none reads another's output) in one launch
  auto multi = [&](std::initializer_list<LinArgs> las) {
    LinMulti m;
    for (const LinArgs& a : las) m.a[m.n++] = a;
    launch_lin_multi(m, F, nrhs, l->stream);
  };
  auto copy = [&](double2* dst, const double2* src) {
    return hipMemcpyAsync(dst, src, sizeof(double2) * NF, hipMemcpyDeviceToDevice, l->stream);
  };
  // forward access: the whole basis, or a ring of three in the segment buffer
  auto Vf = [&](int i) { return store ? P_.V + (size_t)i * NF : P_.V + (size_t)(i % 3) * NF; };
  auto Wf = [&](int i) { return store ? P_.W + (size_t)i * NF : P_.W + (size_t)(i % 3) * NF; };
  // reverse access: the whole basis, or the current segment (indices base .. base + cseg + 1)
  int base = -1;
  auto Vr = [&](int i) { return store ? P_.V + (size_t)i * NF : P_.V + (size_t)(i - base) * NF; };
  auto Wr = [&](int i) { return store ? P_.W + (size_t)i * NF : P_.W + (size_t)(i - base) * NF; };
  // checkpoint j holds (v_{jc-1}, v_{jc}) and (w_{jc-1}, w_{jc}); v_{-1} = w_{-1} = 0
  auto save_ckpt = [&](int m) -> hipError_t {
    if (store || m % cseg) return hipSuccess;
    const int j = m / cseg;
    hipError_t e = copy(P_.ckV + (size_t)(2 * j + 1) * NF, Vf(m));
    if (e == hipSuccess) e = copy(P_.ckW + (size_t)(2 * j + 1) * NF, Wf(m));
    if (m > 0 && e == hipSuccess) e = copy(P_.ckV + (size_t)(2 * j) * NF, Vf(m - 1));
    if (m > 0 && e == hipSuccess) e = copy(P_.ckW + (size_t)(2 * j) * NF, Wf(m - 1));
    return e;
  };

  // ---- forward: v_1 = w_1 = b/|b|, then the recurrences ----
  lin({B}, kTabOne, nullptr, false, {nullptr}, 1, P[0]);
  launch_gf_norm(S, P[0], nch, l->stream);
  lin({B}, kTabNorm, Vf(0), false, {CHI}, 1, P[3]);
  launch_gf_xbar(S, 0, P[3], nch, l->stream);
  lin({B}, kTabNorm, Wf(0), false, {}, 0, nullptr);
  OVS_HIP(save_ckpt(0));
  for (int i = 0; i < k; ++i) {
    OVS_HIP(applyA(Vf(i), T));
    lin({T}, kTabOne, nullptr, false, {Wf(i), nullptr}, 2, P[0]);
    launch_gf_alpha(S, i, P[0], nch, l->stream);
    if (i == k - 1) break;
    OVS_HIP(applyAd(Wf(i), Sv));
    if (i > 0) {
      lin({T, Vf(i), Vf(i - 1)}, kTabV, Vf(i + 1), false, {nullptr}, 1, P[1]);
      lin({Sv, Wf(i), Wf(i - 1)}, kTabW, Wf(i + 1), false, {Vf(i + 1), nullptr}, 2, P[2]);
    } else {
      lin({T, Vf(i)}, kTabV, Vf(i + 1), false, {nullptr}, 1, P[1]);
      lin({Sv, Wf(i)}, kTabW, Wf(i + 1), false, {Vf(i + 1), nullptr}, 2, P[2]);
    }
    launch_gf_beta(S, i, P[1], P[2], nch, l->stream);
    multi({mk({Vf(i + 1)}, kTabSV, Vf(i + 1), false, {CHI}, 1, P[3]),
           mk({Wf(i + 1)}, kTabSW, Wf(i + 1), false, {}, 0, nullptr)});
    launch_gf_xbar(S, i + 1, P[3], nch, l->stream);
    OVS_HIP(save_ckpt(i + 1));
  }
  OVS_HIP(copy(TL, T));  // t_k = A v_k, needed by the first reverse step
  OVS_HIP(hipGetLastError());
  std::vector<int> status(nrhs);
  OVS_HIP(hipMemcpyAsync(status.data(), S.status, sizeof(int) * nrhs, hipMemcpyDeviceToHost,
                         l->stream));
  OVS_HIP(hipStreamSynchronize(l->stream));
  for (int r = 0; r < nrhs; ++r)
    if (status[r] != 0) return OVS_WARN_BREAKDOWN;  // the gradient needs k full iterations

  // ---- inner sign and its VJP ----
  ovs_status result = OVS_OK;
  for (int r = 0; r < nrhs; ++r) {
    const size_t rk = (size_t)r * k;
    std::vector<double2> prev, cur;
    double h = kVjpHStart, change = 0.0;
    int lv = 0, used = 0;
    for (;; h *= 0.5, lv ^= 1) {
      int n0, nn;
      vjp_range(h, n0, nn);
      launch_isign_vjp(S.alpha + rk, S.beta + rk, S.gamma + rk, S.xbar + rk, k, h, n0, nn,
                       P_.vjp, P_.vo[lv], l->stream);
      OVS_HIP(hipGetLastError());
      cur.assign((size_t)3 * k, make_double2(0.0, 0.0));
      OVS_HIP(hipMemcpyAsync(cur.data(), P_.vo[lv].x, sizeof(double2) * k,
                             hipMemcpyDeviceToHost, l->stream));
      OVS_HIP(hipMemcpyAsync(cur.data() + k, P_.vo[lv].gd, sizeof(double2) * k,
                             hipMemcpyDeviceToHost, l->stream));
      if (k > 1)
        OVS_HIP(hipMemcpyAsync(cur.data() + 2 * k, P_.vo[lv].gsup, sizeof(double2) * (k - 1),
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
    const IsignVjpOut& o = P_.vo[used];
    OVS_HIP(hipMemcpyAsync(S.x + rk, o.x, sizeof(double2) * k, hipMemcpyDeviceToDevice,
                           l->stream));
    OVS_HIP(hipMemcpyAsync(S.abar + rk, o.gd, sizeof(double2) * k, hipMemcpyDeviceToDevice,
                           l->stream));
    if (k > 1) {
      OVS_HIP(hipMemcpyAsync(S.bbar + rk, o.gsub_re, sizeof(double) * (k - 1),
                             hipMemcpyDeviceToDevice, l->stream));
      OVS_HIP(hipMemcpyAsync(S.gbar + rk, o.gsup, sizeof(double2) * (k - 1),
                             hipMemcpyDeviceToDevice, l->stream));
    }
  }

  // ---- reverse sweep, segment by segment from the last ----
  for (int j = nseg - 1; j >= 0; --j) {
    const int lo = j * cseg, hi = std::min((j + 1) * cseg, k) - 1;
    if (!store) {
      // replay v_{lo+1} .. v_{top} from the checkpoint, as in the forward pass
      base = lo - 1;
      const int top = std::min((j + 1) * cseg, k - 1);
      OVS_HIP(copy(Vr(lo - 1), P_.ckV + (size_t)(2 * j) * NF));
      OVS_HIP(copy(Vr(lo), P_.ckV + (size_t)(2 * j + 1) * NF));
      OVS_HIP(copy(Wr(lo - 1), P_.ckW + (size_t)(2 * j) * NF));
      OVS_HIP(copy(Wr(lo), P_.ckW + (size_t)(2 * j + 1) * NF));
      for (int i = lo; i < top; ++i) {
        launch_gp_coef(S, i, l->stream);
        OVS_HIP(applyA(Vr(i), T));
        OVS_HIP(applyAd(Wr(i), Sv));
        if (i > 0)
          multi({mk({T, Vr(i), Vr(i - 1)}, kTabV, Vr(i + 1), false, {}, 0, nullptr),
                 mk({Sv, Wr(i), Wr(i - 1)}, kTabW, Wr(i + 1), false, {}, 0, nullptr)});
        else
          multi({mk({T, Vr(i)}, kTabV, Vr(i + 1), false, {}, 0, nullptr),
                 mk({Sv, Wr(i)}, kTabW, Wr(i + 1), false, {}, 0, nullptr)});
        multi({mk({Vr(i + 1)}, kTabSV, Vr(i + 1), false, {}, 0, nullptr),
               mk({Wr(i + 1)}, kTabSW, Wr(i + 1), false, {}, 0, nullptr)});
      }
    }
    for (int i = hi; i >= lo; --i) {
      if (i == k - 1) {
        const int c = i & 1;
        launch_gr_first(S, l->stream);
        LinMulti m0;
        m0.a[m0.n++] = mk({Wr(i)}, kTabSV, TB, false, {}, 0, nullptr);    // tbar
        m0.a[m0.n++] = mk({CHI}, kTabSW, VB[c], false, {}, 0, nullptr);   // vbar (direct part)
        m0.a[m0.n++] = mk({TL}, kTabWB, WB[c], false, {Wr(i)}, 1, P[3]);  // wbar, complete
        if (y) m0.a[m0.n++] = mk({Vr(i)}, kTabY, YA, true, {}, 0, nullptr);
        launch_lin_multi(m0, F, nrhs, l->stream);
        OVS_HIP(applyAd(TB, T1));
        lin({T1}, kTabOne, VB[c], true, {Vr(i)}, 1, P[2]);    // vbar += A^dag tbar
        launch_gforce(P_.Fg, TB, Vr(i), nullptr, nullptr, F, nrhs, g, hA, hAd, l->stream);
        continue;
      }
      const int c = i & 1, p = (i + 1) & 1;
      launch_gr_s1(S, i, P[2], P[3], nch, l->stream);
      if (i > 0)
        multi({mk({VB[p], Vr(i + 1), Wr(i + 1)}, kTabV, VTB[c], false, {Vr(i), Vr(i - 1)}, 2, P[0]),
               mk({WB[p], Vr(i + 1)}, kTabW, WTB[c], false, {Wr(i), Wr(i - 1)}, 2, P[1])});
      else
        multi({mk({VB[p], Vr(i + 1), Wr(i + 1)}, kTabV, VTB[c], false, {Vr(i)}, 1, P[0]),
               mk({WB[p], Vr(i + 1)}, kTabW, WTB[c], false, {Wr(i)}, 1, P[1])});
      launch_gr_s2(S, i, P[0], P[1], nch, l->stream);
      LinMulti m2;
      m2.a[m2.n++] = mk({VTB[c], Wr(i)}, kTabSV, TB, false, {}, 0, nullptr);
      m2.a[m2.n++] = mk({CHI, VTB[p], VTB[c]}, kTabSW, VB[c], false, {}, 0, nullptr);
      if (i > 0)
        m2.a[m2.n++] = mk({WTB[p], WTB[c], Vr(i + 1), Vr(i), Vr(i - 1)}, kTabWB, WB[c], false, {},
                          0, nullptr);
      else
        m2.a[m2.n++] = mk({WTB[p], WTB[c], Vr(i + 1), Vr(i)}, kTabWB, WB[c], false, {}, 0, nullptr);
      if (y) m2.a[m2.n++] = mk({Vr(i)}, kTabY, YA, true, {}, 0, nullptr);
      launch_lin_multi(m2, F, nrhs, l->stream);
      OVS_HIP(applyAd(TB, T1));
      OVS_HIP(applyA(WTB[c], T2));
      multi({mk({T1}, kTabOne, VB[c], true, {Vr(i)}, 1, P[2]),
             mk({T2}, kTabOne, WB[c], true, {Wr(i)}, 1, P[3])});
      launch_gforce(P_.Fg, TB, Vr(i), WTB[c], Wr(i), F, nrhs, g, hA, hAd, l->stream);
    }
  }
  // grad_b = ubar/|b| + nbar v_1,  ubar = vbar_1 + wbar_1  (segment 0 holds v_1)
  lin({VB[0], WB[0]}, kTabOne, T1, false, {Vr(0)}, 1, P[0]);
  launch_gr_final(S, P[0], nch, l->stream);
  lin({T1, Vr(0)}, kTabFin, GB, false, {}, 0, nullptr);
  launch_unpack_f64(GB, (double2*)grad_b, nrhs, g, l->stream);
  launch_gforce_out(P_.Fg, (const double2*)l->links, g, l->bc, (double2*)grad_U, P_.fparts,
                    P_.gmu, l->stream);
  if (y) launch_unpack_f64(YA, (double2*)y, nrhs, g, l->stream);
  OVS_HIP(hipGetLastError());
  OVS_HIP(hipMemcpyAsync(grad_mu, P_.gmu, sizeof(double), hipMemcpyDeviceToHost, l->stream));
  OVS_HIP(hipStreamSynchronize(l->stream));
  return result;
}

extern "C" ovs_status ovs_link_force(ovs_lattice l, const void* U, const void* grad_U, void* force) {
  if (!l || !U || !grad_U || !force || l->parent) return OVS_ERR_ARG;
  StreamScope sc(l);
  launch_link_force((const double2*)U, (const double2*)grad_U, (double2*)force, 4L * l->g.V,
                    l->stream);
  OVS_HIP(hipGetLastError());
  return OVS_OK;
}

extern "C" ovs_status ovs_sign_apply_vjp(ovs_lattice l, const void* b, const void* chi,
                                         int32_t nrhs, int32_t k, int32_t flags, void* y,
                                         void* grad_b, double* grad_mu, void* grad_U,
                                         double* quad_err, void* workspace, size_t ws_bytes) {
  return vjp_impl(l, b, chi, nrhs, k, flags, y, grad_b, grad_mu, grad_U, quad_err, workspace,
                  workspace ? ws_bytes : 0, nullptr);
}

extern "C" ovs_status ovs_vjp_workspace_size(ovs_lattice l, int32_t nrhs, int32_t k,
                                             int32_t flags, size_t* bytes) {
  if (!bytes) return OVS_ERR_ARG;
  *bytes = 0;
  return vjp_impl(l, nullptr, nullptr, nrhs, k, flags, nullptr, nullptr, nullptr, nullptr,
                  nullptr, nullptr, 0, bytes);
}
